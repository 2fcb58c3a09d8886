"""Test glue: seeded client-side material (keys, encryptions) built from the
synthetic streams and the oracle.  Used by the CPU oracle tests and by the GPU
parity tests; the HIP library never sees the secret key."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2509_01253_amd import synth


class Client:
    """Secret key, Galois keys and encryption under seeded streams."""

    def __init__(self, prm: O.Params, seed: int):
        self.prm = prm
        root = synth.Stream(seed)
        self.keys = root.sub(synth.TAG_KEYS)
        self.enc = root.sub(synth.TAG_ENC)
        self.s = self.keys.ternary(prm.N)
        self._evk = {}

    def galois_key(self, g: int) -> np.ndarray:
        g = int(g)
        if g not in self._evk:
            prm = self.prm
            st = self.keys.sub(1000 + g)
            a = np.stack([synth.uniform_limbs(st, prm.mods, prm.N) for _ in range(prm.dnum)])
            e = np.stack([st.gaussian_int(prm.N) for _ in range(prm.dnum)])
            self._evk[g] = O.keygen_galois(prm, self.s, g, a, e)
        return self._evk[g]

    def keyset(self, rotations) -> O.KeySet:
        gal = sorted({O.galois_of(r, self.prm.log_n) for r in rotations if O.galois_of(r, self.prm.log_n) != 1})
        if not gal:
            return O.KeySet([], np.zeros((0, self.prm.dnum, 2, self.prm.L + self.prm.K, self.prm.N), np.uint64))
        return O.KeySet(gal, np.stack([self.galois_key(g) for g in gal]))

    def encrypt_slots(self, z, level: int, delta: float) -> np.ndarray:
        prm = self.prm
        m = O.encode_rns(prm, z, level, delta)
        a = synth.uniform_limbs(self.enc, prm.q[:level], prm.N)
        e = self.enc.gaussian_int(prm.N)
        return O.encrypt(prm, m, self.s, a, e, level)

    def decrypt_slots(self, ct, level: int, delta: float) -> np.ndarray:
        return O.decrypt_decode(self.prm, ct, self.s, level, delta)


def random_ct(prm: O.Params, stream, level: int) -> np.ndarray:
    """Uniform ciphertext [2][level][N] (bit-exact parity does not need a valid encryption)."""
    return np.stack([synth.uniform_limbs(stream, prm.q[:level], prm.N) for _ in range(2)])


def encode_pts(prm: O.Params, slots: np.ndarray, level: int, delta: float) -> np.ndarray:
    """Slot vectors [..., S] -> integer plaintexts [..., level + K, N] (coefficient domain,
    residues mod q_0..q_{level-1} then p_0..p_{K-1})."""
    flat = slots.reshape(-1, slots.shape[-1])
    out = np.stack([O.encode_rns(prm, z, level, delta, ext=True) for z in flat])
    return out.reshape(slots.shape[:-1] + (level + prm.K, prm.N))

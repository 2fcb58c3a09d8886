"""GPU parity of single steps against the oracle, bit-exact in the coefficient
domain: NTT (against the defining sum), rescale, rotation (key switch)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import synth
from tests.gpu_util import ctx_for, dev, host, keys_at, pad_cts
from tests.helpers import Client, random_ct

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2509_01253_amd import fhelin
    return fhelin


def _params(log_n, L, K, dnum, bits):
    return O.make_params(log_n, L, K, dnum, bits, 2.0 ** 40)


@pytest.mark.parametrize("log_n", [10, 12, 13, 15, 16])
def test_ntt_matches_definition(F, log_n):
    print(f"ntt log_n={log_n}", flush=True)
    prm = _params(log_n, 3, 1, 3, 50)
    ctx = ctx_for(F, prm)
    try:
        N = prm.N
        st = synth.Stream(1000 + log_n)
        mods = [0, 1, 2, 3, 1]
        rows = np.stack([st.uniform_mod(N, prm.mods[m]) for m in mods])
        for m in range(4):
            assert F.fhelin_ctx_root(ctx, m) == O.min_root(prm.mods[m], log_n)
        d = dev(rows)
        F.fhelin_ntt(ctx, d, mods, False)
        fw = host(d)
        if log_n <= 10:
            for r, m in enumerate(mods):
                assert np.array_equal(fw[r], O.ntt_naive(rows[r], log_n, prm.mods[m]))
        ks = [0, 1, 2, 255, 256, N // 2 - 1, N // 2, N - 1] + list(st.integers(24, 0, N - 1))
        for r, m in enumerate(mods):
            q = prm.mods[m]
            psi = O.min_root(q, log_n)
            for k in ks[: 12 if log_n >= 15 else len(ks)]:
                assert int(fw[r, k]) == O.ntt_naive_at(rows[r], int(k), log_n, q, psi), (r, k)
        F.fhelin_ntt(ctx, d, mods, True)
        assert np.array_equal(host(d), rows)
    finally:
        F.fhelin_ctx_destroy(ctx)


@pytest.mark.parametrize("log_n,L", [(12, 4), (16, 12)])
def test_rescale_bit_exact(F, log_n, L):
    print(f"rescale log_n={log_n}", flush=True)
    prm = _params(log_n, L, 3, 4, 50)
    ctx = ctx_for(F, prm)
    try:
        st = synth.Stream(2000 + log_n)
        levels = [L, 2, L - 1, 3]
        cts = [random_ct(prm, st, l) for l in levels]
        x = dev(pad_cts(cts, L, prm.N))
        y = dev(np.zeros((len(levels), 2, L, prm.N), np.uint64))
        F.fhelin_rescale(ctx, x, levels, y, [l - 1 for l in levels])
        got = host(y)
        for t, l in enumerate(levels):
            assert np.array_equal(got[t, :, : l - 1], O.rescale(prm, cts[t], l)), t
    finally:
        F.fhelin_ctx_destroy(ctx)


def test_rotate_small_full(F):
    print("rotate small", flush=True)
    prm = _params(10, 4, 2, 2, 50)
    ctx = ctx_for(F, prm)
    cl = Client(prm, 3000)
    try:
        st = synth.Stream(3001)
        steps = [1, 5, -1, 0, 100, 7]
        levels = [4, 3, 2, 4, 1, 4]
        keys = cl.keyset([s for s in steps if s % prm.S])
        ks = F.fhelin_keyset_load(ctx, keys.galois, prm.L, dev(keys_at(prm, keys, prm.L)))
        cts = [random_ct(prm, st, l) for l in levels]
        x = dev(pad_cts(cts, prm.L, prm.N))
        y = dev(np.zeros_like(pad_cts(cts, prm.L, prm.N)))
        F.fhelin_rotate(ctx, ks, x, levels, steps, y)
        got = host(y)
        for t, (l, r) in enumerate(zip(levels, steps)):
            g = O.galois_of(r, prm.log_n)
            want = cts[t] if g == 1 else O.rotate(prm, cts[t], g, cl.galois_key(g), l)
            assert np.array_equal(got[t, :, :l], want), t
        F.fhelin_keyset_release(ks)
    finally:
        F.fhelin_ctx_destroy(ctx)


def test_rotate_full_size_sampled(F):
    """N = 2^16, 12 + 3 primes, dnum 4: sampled coefficients against the oracle's
    per-coefficient key switch (definition of the ring product per output)."""
    print("rotate 2^16 sampled", flush=True)
    prm = _params(16, 12, 3, 4, 50)
    ctx = ctx_for(F, prm)
    try:
        st = synth.Stream(3100)
        levels = [12, 5]
        g_steps = [1, 1024]
        # random (not encrypted) keys suffice for bit-exact parity
        gal = [O.galois_of(r, prm.log_n) for r in g_steps]
        evk = np.stack([np.stack([np.stack([synth.uniform_limbs(st, prm.mods, prm.N) for _ in range(2)])
                                  for _ in range(prm.dnum)]) for _ in gal])
        keys = O.KeySet(gal, evk)
        ks = F.fhelin_keyset_load(ctx, gal, prm.L, dev(keys_at(prm, keys, prm.L)))
        cts = [random_ct(prm, st, l) for l in levels]
        x = dev(pad_cts(cts, prm.L, prm.N))
        y = dev(np.zeros((2, 2, prm.L, prm.N), np.uint64))
        F.fhelin_rotate(ctx, ks, x, levels, g_steps, y)
        got = host(y)
        for t, l in enumerate(levels):
            g = gal[t]
            sc = O.automorph_limbs(cts[t], g, prm.log_n, prm.q)
            for k in (0, 1, 4097, prm.N - 1):
                col = O.ks_inner_at(prm, sc[1], evk[t], l, k)
                u0 = O.moddown_at(prm, col[0], l)
                u1 = O.moddown_at(prm, col[1], l)
                want0 = [(int(u0[i]) + int(sc[0, i, k])) % prm.q[i] for i in range(l)]
                assert [int(v) for v in got[t, 0, :l, k]] == want0, (t, k)
                assert np.array_equal(got[t, 1, :l, k], u1), (t, k)
        F.fhelin_keyset_release(ks)
    finally:
        F.fhelin_ctx_destroy(ctx)

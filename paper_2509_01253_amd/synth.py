"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module holds random-number generation only: no ring, modular or
encoding arithmetic of the scheme lives here.  Every stream is SplitMix64
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) used as a counter-based generator: output i of a stream seeded
with ``s`` is ``mix64(s + (i + 1) * 0x9E3779B97F4A7C15)``, so any stream can
be produced in one vectorised numpy expression and any element addressed
directly.  Floating-point draws are built from the raw 64-bit words with
transforms defined here, so they do not depend on numpy's own generators.

Stream tags (xor-ed into the master seed): keys, encryption randomness,
weights, inputs, permutations, arrivals, levels.
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
TAG_KEYS, TAG_ENC, TAG_W, TAG_X, TAG_PERM, TAG_ARRIVAL, TAG_LEVEL = 1, 2, 3, 4, 5, 6, 7
MASTER_SEED = 20250901


def master_seed(config: int) -> int:
    """Master seed of workload ``config`` (1-based)."""
    return MASTER_SEED + int(config)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


class Stream:
    """A SplitMix64 stream; successive calls consume successive counters."""

    def __init__(self, seed: int, tag: int = 0):
        self.seed = np.uint64((int(seed) ^ int(tag)) & 0xFFFFFFFFFFFFFFFF)
        self.pos = 0

    def sub(self, tag: int) -> "Stream":
        """An independent stream keyed by ``tag`` (seed xor a mixed tag)."""
        t = int(_mix64(np.array([tag], dtype=np.uint64) + GOLDEN_GAMMA)[0])
        return Stream(int(self.seed) ^ t)

    def u64(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            idx = np.arange(self.pos + 1, self.pos + 1 + n, dtype=np.uint64)
            out = _mix64(self.seed + idx * GOLDEN_GAMMA)
        self.pos += n
        return out

    def uniform01(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def uniform(self, n: int, lo: float, hi: float) -> np.ndarray:
        return lo + (hi - lo) * self.uniform01(n)

    def normal(self, n: int) -> np.ndarray:
        """Standard normal by Box-Muller on pairs of uniforms."""
        m = (n + 1) // 2
        u1 = self.uniform01(m)
        u2 = self.uniform01(m)
        r = np.sqrt(-2.0 * np.log1p(-u1))
        t = 2.0 * np.pi * u2
        return np.concatenate([r * np.cos(t), r * np.sin(t)])[:n]

    def he_normal(self, shape, fan_in: int) -> np.ndarray:
        n = int(np.prod(shape))
        return (self.normal(n) * np.sqrt(2.0 / fan_in)).reshape(shape)

    def ternary(self, n: int) -> np.ndarray:
        """Values in {-1, 0, 1} (int8)."""
        return ((self.u64(n) % np.uint64(3)).astype(np.int64) - 1).astype(np.int8)

    def gaussian_int(self, n: int, sigma: float = 3.2, tail: float = 6.0) -> np.ndarray:
        """Rounded normal with standard deviation ``sigma``, clipped at ``tail`` sigma."""
        v = np.rint(self.normal(n) * sigma)
        lim = np.floor(tail * sigma)
        return np.clip(v, -lim, lim).astype(np.int64)

    def uniform_mod(self, n: int, q: int) -> np.ndarray:
        """Values in [0, q) (uint64): word mod q."""
        return self.u64(n) % np.uint64(q)

    def permutation(self, n: int) -> np.ndarray:
        """A uniformly random permutation of range(n) (int32), by sorting random keys."""
        return np.argsort(self.u64(n), kind="stable").astype(np.int32)

    def integers(self, n: int, lo: int, hi: int) -> np.ndarray:
        """Integers in [lo, hi] inclusive."""
        return (lo + (self.u64(n) % np.uint64(hi - lo + 1)).astype(np.int64)).astype(np.int64)

    def exponential(self, n: int, rate: float) -> np.ndarray:
        return -np.log1p(-self.uniform01(n)) / rate


def uniform_limbs(stream: Stream, moduli, n: int) -> np.ndarray:
    """[len(moduli)][n] uint64, row i uniform in [0, moduli[i])."""
    return np.stack([stream.uniform_mod(n, int(q)) for q in moduli]) if len(moduli) else np.zeros((0, n), np.uint64)

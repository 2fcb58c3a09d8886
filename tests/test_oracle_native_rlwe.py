"""Pins of the ciphertext-level oracle of the paper's own pipeline (oracle/native_rlwe.py):
ring arithmetic against exact Python-integer arithmetic modulo Phi_M (oracle/native.py's
long division), the two-term dual basis against exact Gaussian elimination, the gadget
digits against their defining sum, and every server step against what decryption must
give: the automorphism of the message, the input coefficients after the partial trace
(Sec. 4.4 lemma), and the integer layer's outputs in the packed coefficients."""
import random

import numpy as np
import pytest

from oracle import native as V
from oracle import native_rlwe as R

SMALL = [(3, 3), (5, 2), (3, 4), (7, 2)]


def _params(t, alpha, gamma=1, beta=None, log_d=9, l=3, log_p=8, sigma=2.0 ** 28):
    return R.NativeParams(t, alpha, gamma, beta if beta is not None else alpha - 1, log_d, l, log_p, sigma)


def _ints(x):
    return [int(v) for v in x]


def _u64(x):
    return np.array([v % 2 ** 64 for v in x], np.uint64)


@pytest.mark.parametrize("t,a", SMALL)
def test_ring_arithmetic_matches_exact_integers(t, a):
    P = _params(t, a, beta=1)
    Rg = V.Ring(t, a)
    rng = np.random.default_rng(t * 10 + a)
    for _ in range(3):
        x = rng.integers(0, 2 ** 64, P.N, dtype=np.uint64, endpoint=False)
        y = rng.integers(0, 2 ** 64, P.N, dtype=np.uint64, endpoint=False)
        assert np.array_equal(R.mul(P, x, y), _u64(Rg.mul(_ints(x), _ints(y))))
        d = Rg.units[rng.integers(len(Rg.units))]
        assert np.array_equal(R.automorphism(P, x, d), _u64(Rg.sigma(_ints(x), d)))
        e = int(rng.integers(P.M))
        mono = [0] * P.M
        mono[e] = 1
        assert np.array_equal(R.mul_mono(P, x, e), _u64(Rg.mul(_ints(x), Rg.reduce(mono))))


@pytest.mark.parametrize("t,a", SMALL)
def test_extraction_multipliers_are_the_dual_basis(t, a):
    """M conj(Omega*_i) = X^(M-i) - X^(M/t - r) (r = i mod M/t) equals M times the dual
    basis element found by exact elimination on the trace form."""
    Rg = V.Ring(t, a)
    B = Rg.dual_basis()
    M, Mt = Rg.M, Rg.M // t
    for i in range(Rg.N):
        x = [0] * M
        x[(M - i) % M] += 1
        x[(Mt - i % Mt) % M] -= 1
        assert Rg.reduce(x) == [M * v for v in B[i]], i


def test_gadget_digits():
    P = _params(3, 3, beta=1, log_d=9, l=3)
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2 ** 64, 500, dtype=np.uint64, endpoint=False)
    dg = R.decompose(P, a)
    assert dg.shape == (3, 500) and dg.min() >= -256 and dg.max() < 256
    for k in range(500):
        rec = sum(int(dg[i, k]) * 2 ** (64 - 9 * (i + 1)) for i in range(3)) % 2 ** 64
        err = (int(a[k]) - rec) % 2 ** 64
        err = err - 2 ** 64 if err >= 2 ** 63 else err
        assert abs(err) <= 2 ** (64 - 27 - 1), k


@pytest.mark.parametrize("t,a", SMALL)
def test_encrypt_decrypt_and_galois(t, a):
    P = _params(t, a, beta=1)
    Rg = V.Ring(t, a)
    cl = R.NativeClient(P, 7 + t)
    rng = random.Random(t)
    m = [rng.randrange(P.p) for _ in range(P.N)]
    ct = cl.encrypt(m)
    assert np.array_equal(cl.decrypt(ct), np.array(m))
    for d in P.taus():
        key = cl.ksk(d)
        out = R.apply_galois(P, ct, d, {d: key})
        want = [v % P.p for v in Rg.sigma(m, d)]
        assert np.array_equal(cl.decrypt(out), np.array(want)), d


@pytest.mark.parametrize("t,a,gamma", [(3, 3, 1), (3, 4, 2), (5, 2, 1), (5, 3, 2)])
def test_extraction_gives_the_coefficients(t, a, gamma):
    """Tr_{K/K_gamma} of each extracted row decrypts to the constant m_i (lemma on
    partial trace extraction; the trace is taken with the exact ring of native.py on
    the decrypted phase)."""
    P = _params(t, a, gamma=gamma)
    Rg = V.Ring(t, a)
    cl = R.NativeClient(P, 11)
    rng = random.Random(a)
    m = [rng.randrange(P.p) for _ in range(P.N)]
    rows = R.extract(P, cl.encrypt_powers(m))
    for i in range(0, P.N, max(1, P.N // 12)):
        ph = cl.phase(rows[i])
        tr = _u64(Rg.trace_down(_ints(ph), gamma))
        dec = cl.decode(tr)
        assert dec[0] == m[i] and not dec[1:].any(), i


@pytest.mark.parametrize("t,a,gamma,beta", [(3, 4, 1, 3), (3, 4, 2, 3), (5, 3, 1, 2), (3, 3, 1, 1), (7, 2, 1, 1)])
def test_layer_and_packing_decrypt_to_the_integer_layer(t, a, gamma, beta):
    """Extraction, an integer layer with a folded shuffle and fast packing: the packed
    ciphertexts decrypt to (W' x) mod p at o M/t^beta and to 0 elsewhere; the packing
    used t^(beta-gamma) - 1 + (alpha-beta)(t-1) key switches per packed ciphertext."""
    P = _params(t, a, gamma=gamma, beta=beta)
    cl = R.NativeClient(P, 21)
    keys = cl.keyset()
    rng = np.random.default_rng(t + a + gamma)
    n_in = P.N + P.N // 2  # two chunks, the second half used
    x = rng.integers(0, 16, n_in)
    chunks = []
    for c in range(2):
        m = np.zeros(P.N, np.int64)
        part = x[c * P.N: (c + 1) * P.N]
        m[: part.size] = part
        chunks.append(cl.encrypt_powers(m))
    n_out = P.n_pack + 3  # a full pack and a partial one
    W = rng.integers(-8, 8, (n_out, n_in))
    perm = rng.permutation(n_out)
    rows = np.concatenate([R.extract(P, c) for c in chunks])[:n_in]
    F = R.linear_rows(W[perm], rows)
    count = []
    packed = [R.pack(P, F[g: g + P.n_pack], keys, count) for g in range(0, n_out, P.n_pack)]
    assert count == [P.key_switches_per_pack()] * len(packed)
    y = (W[perm] @ x) % P.p
    pos = R.unpack_positions(P)
    for g, ct in enumerate(packed):
        dec = cl.decrypt(ct)
        want = np.zeros(P.N, np.int64)
        seg = y[g * P.n_pack: (g + 1) * P.n_pack]
        want[pos[: seg.size]] = seg
        assert np.array_equal(dec, want), g
    # the server_layer helper runs the same steps
    again = R.server_layer(P, np.stack(chunks), W, keys, perm)
    assert all(np.array_equal(cl.decrypt(c), cl.decrypt(d)) for c, d in zip(again, packed))


def test_packing_key_switch_counts_against_the_paper_table():
    """This packing's key switches per packed coefficient at the paper's largest pack
    (beta = alpha - 1) stay below the paper's table for gamma = 1, 2."""
    for t, alpha in [(3, 7), (5, 5), (7, 4)]:
        for gamma in (1, 2):
            P = _params(t, alpha, gamma=gamma, beta=alpha - 1)
            ours = P.key_switches_per_pack() / P.n_pack
            paper = V.key_switches_per_coefficient(t, alpha, gamma)
            assert ours < paper, (t, alpha, gamma, ours, paper)


def test_conv_matrix_is_the_windowed_sum():
    """conv_matrix x equals the convolution computed directly on an H x W x C_in array
    (numpy slicing of a zero-padded image), for strides 1 and 2 and kernels 1 and 3."""
    rng = np.random.default_rng(5)
    for c_in, c_out, h, w, k, s in ((2, 3, 5, 4, 3, 1), (3, 2, 6, 6, 3, 2), (4, 5, 4, 4, 1, 2), (6, 3, 1, 1, 1, 1)):
        wts = rng.integers(-8, 8, (c_out, c_in, k, k))
        img = rng.integers(0, 16, (h, w, c_in))
        pad = np.zeros((h + 2 * (k // 2), w + 2 * (k // 2), c_in), np.int64)
        pad[k // 2: k // 2 + h, k // 2: k // 2 + w] = img
        ho, wo = (h - 1) // s + 1, (w - 1) // s + 1
        direct = np.zeros((ho, wo, c_out), np.int64)
        for yo in range(ho):
            for xo in range(wo):
                win = pad[s * yo: s * yo + k, s * xo: s * xo + k]  # k x k x c_in
                direct[yo, xo] = np.einsum("yxc,ocyx->o", win, wts)
        got = R.conv_matrix(c_in, c_out, h, w, k, s, wts) @ img.reshape(-1)
        assert np.array_equal(got, direct.reshape(-1)), (c_in, c_out, h, w, k, s)


def test_gadget_digits_general_base():
    """A base that is not a power of two (the paper's 310, l = 4): digits in
    [-D/2, D/2) and sum_i d_i g_i within 2^63 / D^l (rounding to a multiple of 1/D^l)
    plus l D / 4 (each g_i = round(2^64 / D^i) off by at most 1/2) of a, modulo 2^64;
    and base 512 given explicitly decomposes exactly as log_d = 9."""
    P = R.NativeParams(5, 3, 1, 2, 0, 4, 16, 2.0 ** 13, base=310)
    assert [P.gadget(i) for i in (1, 2)] == [round(2 ** 64 / 310), round(2 ** 64 / 310 ** 2)]
    rng = np.random.default_rng(31)
    a = rng.integers(0, 2 ** 64, 2000, dtype=np.uint64, endpoint=False)
    a[:4] = [0, 2 ** 64 - 1, 2 ** 63, 2 ** 63 - 1]
    dg = R.decompose(P, a)
    assert dg.shape == (4, 2000) and dg.min() >= -155 and dg.max() < 155
    bound = 2 ** 63 / 310 ** 4 + 4 * 310 / 4
    for k in range(2000):
        rec = sum(int(dg[i, k]) * P.gadget(i + 1) for i in range(4)) % 2 ** 64
        err = (int(a[k]) - rec) % 2 ** 64
        err = err - 2 ** 64 if err >= 2 ** 63 else err
        assert abs(err) <= bound, k
    P2 = R.NativeParams(3, 3, 1, 1, 0, 3, 8, 2.0 ** 28, base=512)
    P9 = _params(3, 3, beta=1, log_d=9, l=3)
    assert np.array_equal(R.decompose(P2, a), R.decompose(P9, a))
    assert [P2.gadget(i) for i in (1, 2, 3)] == [2 ** 55, 2 ** 46, 2 ** 37]


@pytest.mark.parametrize("t,a,gamma,beta", [(5, 3, 1, 2), (3, 4, 2, 3)])
def test_base_310_key_switching_and_packing_decrypt(t, a, gamma, beta):
    """Key switching and the whole pipeline with the paper's 16-bit-set gadget (base
    310, depth 4) on small rings: every Galois key switch decrypts to the automorphism
    of the message, and the packed ciphertexts decrypt to the integer layer."""
    P = R.NativeParams(t, a, gamma, beta, 0, 4, 16, 2.0 ** 13, base=310)
    Rg = V.Ring(t, a)
    cl = R.NativeClient(P, 41 + t)
    keys = cl.keyset()
    rnd = random.Random(t + a)
    m = [rnd.randrange(P.p) for _ in range(P.N)]
    ct = cl.encrypt(m)
    for d in P.taus():
        out = R.apply_galois(P, ct, d, keys)
        assert np.array_equal(cl.decrypt(out), np.array([v % P.p for v in Rg.sigma(m, d)])), d
    rng = np.random.default_rng(t * a)
    n_in = P.N + P.N // 2
    x = rng.integers(0, 16, n_in)
    chunks = []
    for c in range(2):
        mm = np.zeros(P.N, np.int64)
        part = x[c * P.N: (c + 1) * P.N]
        mm[: part.size] = part
        chunks.append(cl.encrypt_powers(mm))
    n_out = P.n_pack + 3
    W = rng.integers(-8, 8, (n_out, n_in))
    rows = np.concatenate([R.extract(P, c) for c in chunks])[:n_in]
    F = R.linear_rows(W, rows)
    y = (W @ x) % P.p
    pos = R.unpack_positions(P)
    for g in range(0, n_out, P.n_pack):
        dec = cl.decrypt(R.pack(P, F[g: g + P.n_pack], keys))
        seg = y[g: g + P.n_pack]
        assert np.array_equal(dec[pos[: seg.size]], seg), g

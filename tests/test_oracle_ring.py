"""Pins of the oracle's ring layer: primes, roots, NTT, products, automorphisms.

Every check compares the oracle with something other than itself: a hand-worked
example, pure-Python big-integer brute force, or an algebraic law."""
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    d = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        d[k] = [int(x) for x in v]
    return d


def test_ntt_worked_example():
    g = _golden("ntt_n4_q17.txt")
    log_n, q = g["log_n"][0], g["q"][0]
    assert O.min_root(q, log_n) == g["psi"][0]
    assert list(O.ntt_naive(g["a"], log_n, q)) == g["ntt_a"]
    assert list(O.intt_naive(g["ntt_a"], log_n, q)) == g["a"]
    assert list(O.polymul_schoolbook(g["a"], g["b"], log_n, q)) == g["a_times_b"]
    assert list(O.polymul_fast(g["a"], g["b"], log_n, q)) == g["a_times_b"]


def _sieve(n):
    s = np.ones(n, bool)
    s[:2] = False
    for i in range(2, int(n ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = False
    return s


def test_is_prime_matches_sieve():
    s = _sieve(20000)
    got = np.array([O.lib().or_is_prime(i) for i in range(20000)], bool)
    assert np.array_equal(got, s)
    # strong pseudoprimes to small bases and Carmichael numbers are composite
    for c in [561, 1105, 2047, 3215031751, 3825123056546413051]:
        assert O.lib().or_is_prime(c) == 0
    for p in [2 ** 61 - 1, 2 ** 31 - 1, 1000000007]:
        assert O.lib().or_is_prime(p) == 1


@pytest.mark.parametrize("log_n,bits,count", [(12, 36, 4), (15, 50, 10), (16, 50, 15)])
def test_prime_scan(log_n, bits, count):
    pr = O.gen_primes(log_n, bits, count)
    two_n = 2 << log_n
    assert pr == sorted(pr, reverse=True) and len(set(pr)) == count
    assert all(p < 2 ** bits and p % two_n == 1 for p in pr)
    # every candidate 1 mod 2N skipped between 2^bits and the last prime is composite
    # (a Fermat witness proves it), every chosen one passes Fermat to several bases
    cand = pr[0] + two_n
    while cand < 2 ** bits:
        assert pow(2, cand - 1, cand) != 1 or pow(3, cand - 1, cand) != 1
        cand += two_n
    for hi, lo in zip(pr, pr[1:]):
        c = hi - two_n
        while c > lo:
            assert any(pow(b, c - 1, c) != 1 for b in (2, 3, 5, 7))
            c -= two_n
    for p in pr:
        assert all(pow(b, p - 1, p) == 1 for b in (2, 3, 5, 7, 11))


@pytest.mark.parametrize("q,log_n", [(17, 2), (97, 4), (257, 7), (7681, 8), (12289, 10)])
def test_min_root_brute_force(q, log_n):
    n = 1 << log_n
    brute = next(x for x in range(2, q) if pow(x, n, q) == q - 1)
    assert O.min_root(q, log_n) == brute


@pytest.mark.parametrize("log_n,bits", [(12, 36), (16, 50)])
def test_min_root_large(log_n, bits):
    q = O.gen_primes(log_n, bits, 1)[0]
    psi = O.min_root(q, log_n)
    n = 1 << log_n
    assert pow(psi, n, q) == q - 1
    # minimal among all primitive 2N-th roots psi^k, k odd (brute force over k)
    x, psi2 = psi, psi * psi % q
    for _ in range(n - 1):
        x = x * psi2 % q
        assert x >= psi


def _eval_py(a, x, q):
    acc = 0
    for c in reversed(a):
        acc = (acc * x + int(c)) % q
    return acc


def _brv(k, bits):
    return int(format(k, f"0{bits}b")[::-1], 2)


@pytest.mark.parametrize("log_n", [3, 5, 7])
def test_ntt_naive_is_evaluation(log_n):
    q = O.gen_primes(log_n, 30, 1)[0]
    psi = O.min_root(q, log_n)
    rng = np.random.default_rng(log_n)
    a = rng.integers(0, q, 1 << log_n, dtype=np.uint64)
    A = O.ntt_naive(a, log_n, q)
    for k in range(1 << log_n):
        assert int(A[k]) == _eval_py(a, pow(psi, 2 * _brv(k, log_n) + 1, q), q)
    assert np.array_equal(O.intt_naive(A, log_n, q), a)


def test_ntt_naive_at_is_evaluation():
    """The single-output form of the definition (the checker of the sampled NTT
    comparisons at N = 2^15, 2^16) against polynomial evaluation in Python integers
    at sampled k of a 2^15 ring with a 50-bit prime, and against the full-transform
    routine on every k of a 2^9 ring."""
    for log_n, bits, ks in ((15, 50, (0, 1, 12345, (1 << 15) - 1)), (9, 50, range(1 << 9))):
        q = O.gen_primes(log_n, bits, 1)[0]
        psi = O.min_root(q, log_n)
        rng = np.random.default_rng(100 + log_n)
        a = rng.integers(0, q, 1 << log_n, dtype=np.uint64)
        full = O.ntt_naive(a, log_n, q) if log_n <= 9 else None
        for k in ks:
            got = O.ntt_naive_at(a, k, log_n, q, psi)
            if full is not None:
                assert got == int(full[k]), k
            else:
                assert got == _eval_py(a, pow(psi, 2 * _brv(k, log_n) + 1, q), q), k


def _schoolbook_py(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            t = int(a[i]) * int(b[j])
            if i + j < n:
                c[i + j] += t
            else:
                c[i + j - n] -= t
    return [v % q for v in c]


def test_schoolbook_brute_force():
    q = O.gen_primes(3, 40, 1)[0]
    rng = np.random.default_rng(3)
    for _ in range(5):
        a = rng.integers(0, q, 8, dtype=np.uint64)
        b = rng.integers(0, q, 8, dtype=np.uint64)
        assert list(O.polymul_schoolbook(a, b, 3, q)) == _schoolbook_py(a, b, q)


@pytest.mark.parametrize("log_n,bits", [(6, 30), (8, 50), (10, 60), (10, 36)])
def test_products_agree(log_n, bits):
    q = O.gen_primes(log_n, bits, 1)[0]
    rng = np.random.default_rng(log_n + bits)
    a = rng.integers(0, q, 1 << log_n, dtype=np.uint64)
    b = rng.integers(0, q, 1 << log_n, dtype=np.uint64)
    sb = O.polymul_schoolbook(a, b, log_n, q)
    assert np.array_equal(O.polymul_fast(a, b, log_n, q), sb)
    if log_n <= 8:
        # NTT diagonalises the negacyclic product
        A, B = O.ntt_naive(a, log_n, q), O.ntt_naive(b, log_n, q)
        prod = np.array([(int(x) * int(y)) % q for x, y in zip(A, B)], np.uint64)
        assert np.array_equal(O.ntt_naive(sb, log_n, q), prod)


def test_fast_product_sampled_full_size():
    log_n = 16
    q = O.gen_primes(log_n, 50, 1)[0]
    rng = np.random.default_rng(16)
    a = rng.integers(0, q, 1 << log_n, dtype=np.uint64)
    b = rng.integers(0, q, 1 << log_n, dtype=np.uint64)
    f = O.polymul_fast(a, b, log_n, q)
    for k in [0, 1, 777, 32768, 65535]:
        assert int(f[k]) == O.polymul_at(a, b, k, log_n, q)


def test_automorphism_laws():
    log_n = 6
    n = 1 << log_n
    q = O.gen_primes(log_n, 40, 1)[0]
    rng = np.random.default_rng(5)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    for g in [5, 25, 2 * n - 1, 3, 77]:
        # direct definition: X^j -> X^(g j mod 2N), X^N = -1
        exp = [0] * n
        for j in range(n):
            e = g * j % (2 * n)
            if e < n:
                exp[e] = (exp[e] + int(a[j])) % q
            else:
                exp[e - n] = (exp[e - n] - int(a[j])) % q
        sa = O.automorph(a, g, log_n, q)
        assert list(sa) == exp
        # ring homomorphism
        assert np.array_equal(O.automorph(O.polymul_schoolbook(a, b, log_n, q), g, log_n, q),
                              O.polymul_schoolbook(sa, O.automorph(b, g, log_n, q), log_n, q))
    # composition and the order of 5
    g, h = 5, 77
    assert np.array_equal(O.automorph(O.automorph(a, h, log_n, q), g, log_n, q),
                          O.automorph(a, g * h % (2 * n), log_n, q))
    assert pow(5, n // 2, 2 * n) == 1
    assert np.array_equal(O.automorph(a, pow(5, n // 2, 2 * n), log_n, q), a)


def test_automorphism_is_slot_rotation():
    log_n = 8
    delta = 2.0 ** 30
    rng = np.random.default_rng(11)
    z = rng.uniform(-1, 1, 1 << (log_n - 1)) + 1j * rng.uniform(-1, 1, 1 << (log_n - 1))
    m = O.encode(z, log_n, delta)
    q = O.gen_primes(log_n, 60, 1)[0]
    for k in [1, 3, 17]:
        g = O.galois_of(k, log_n)
        assert g == pow(5, k, 2 << log_n)
        mg = O.automorph(O.to_rns(m, [q])[0], g, log_n, q).astype(np.int64)
        mg = np.where(mg > q // 2, mg - q, mg)
        assert np.abs(O.decode(mg, log_n, delta) - np.roll(z, -k)).max() < 1e-6
    # conjugation
    g = (2 << log_n) - 1
    mg = O.automorph(O.to_rns(m, [q])[0], g, log_n, q).astype(np.int64)
    mg = np.where(mg > q // 2, mg - q, mg)
    assert np.abs(O.decode(mg, log_n, delta) - np.conj(z)).max() < 1e-6

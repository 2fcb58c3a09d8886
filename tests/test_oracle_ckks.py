"""Pins of the oracle's scheme layer: encode/decode, CRT, ModUp, ModDown,
key switching, rescale and plaintext products.  Each check uses big-integer
arithmetic in Python, a closed form, or the decryption identity."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import synth
from tests.helpers import Client, random_ct


def _crt_py(res, mods):
    """Centred CRT lift in Python integers."""
    Q = 1
    for q in mods:
        Q *= q
    x = 0
    for r, q in zip(res, mods):
        Qi = Q // q
        x += int(r) * Qi * pow(Qi, -1, q)
    x %= Q
    return x - Q if x > Q // 2 else x


@pytest.fixture(scope="module")
def small():
    # c1-like but smaller ring: 4 q + 2 p, dnum 2 (alpha 2), 40-bit primes
    return O.make_params(8, 4, 2, 2, 40, 2.0 ** 25)


def test_encode_matches_definition():
    """The FFT encode against the long-double defining sum.  With |m_k| below about
    Delta * N and FP64 rounding error of order N * 2^-53 relative, a coefficient can
    round differently only within ~2^-14 of a half-integer (probability ~1e-4 per
    coefficient): over these 1168 coefficients at most one may differ, by one unit."""
    rng = np.random.default_rng(0)
    mismatches = 0
    for log_n in (4, 7, 9, 10):
        s = 1 << (log_n - 1)
        z = rng.uniform(-1, 1, s) + 1j * rng.uniform(-1, 1, s)
        d1 = O.encode(z, log_n, 2.0 ** 30)
        d2 = O.encode_direct(z, log_n, 2.0 ** 30)
        assert np.abs(d1 - d2).max() <= 1
        mismatches += int(np.sum(d1 != d2))
        back = O.decode(d1.astype(np.float64), log_n, 2.0 ** 30)
        back2 = O.decode_direct(d1.astype(np.longdouble), log_n, 2.0 ** 30)
        assert np.abs(back - back2).max() < 1e-9
        # rounding error only: |decode(encode(z)) - z| <= N/2 * 0.5 / Delta
        assert np.abs(back - z).max() <= (1 << log_n) / 2 ** 31
    assert mismatches <= 1


def test_encode_rounds_ties_to_even():
    """A constant slot vector c encodes to the constant rint(Delta c): with Delta = 1
    and c on a half-integer the rounding rule decides, ties go to the even integer
    (a biased round-half-up would give 3, -2, 5 here)."""
    for c, want in ((2.5, 2), (-2.5, -2), (4.5, 4), (3.5, 4), (-3.5, -4)):
        m = O.encode(np.full(8, c), 4, 1.0)
        assert m[0] == want and np.all(m[1:] == 0), (c, m)
        assert O.encode_direct(np.full(8, c), 4, 1.0)[0] == want


def test_encode_constant_closed_form():
    for c in (0.5, -0.3, 0.123456789):
        z = np.full(1 << 9, c)
        m = O.encode(z, 10, 2.0 ** 40)
        assert m[0] == np.rint(2.0 ** 40 * c)
        assert np.all(m[1:] == 0)
        assert np.array_equal(O.encode_direct(z, 10, 2.0 ** 40), m)


def test_encode_real_slots_give_real_symmetric_poly():
    # a single slot impulse encodes to (2/N) Re(zeta^(-k)) times Delta at slot 0
    log_n, delta = 6, 2.0 ** 40
    n = 1 << log_n
    z = np.zeros(n // 2)
    z[0] = 1.0
    m = O.encode(z, log_n, delta)
    k = np.arange(n)
    assert np.array_equal(m, np.rint(delta * 2 / n * np.cos(np.pi * k / n)).astype(np.int64))


def test_crt_centered(small):
    prm = small
    rng = np.random.default_rng(1)
    for level in (1, 2, 4):
        mods = prm.q[:level]
        m = np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in mods])
        got = O.crt_centered(prm, m, level)
        for k in (0, 5, 100, prm.N - 1):
            assert int(got[k]) == _crt_py(m[:, k], mods) or abs(float(got[k]) - _crt_py(m[:, k], mods)) <= abs(
                _crt_py(m[:, k], mods)) * 2.0 ** -62


@pytest.mark.parametrize("level", [4, 3, 1])
def test_modup_congruence_and_bound(small, level):
    prm = small
    rng = np.random.default_rng(level)
    x = np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in prm.q[:level]])
    y = O.modup(prm, x, level)
    ext = prm.q[:level] + prm.p
    for j in range(prm.beta(level)):
        lo, hi = j * prm.alpha, min((j + 1) * prm.alpha, level)
        dig = prm.q[lo:hi]
        Qj = 1
        for q in dig:
            Qj *= q
        for k in (0, 1, 17, prm.N - 1):
            Y = _crt_py(y[j, :, k], ext)
            # y = x (mod Q_j) and |y| <= (#digit primes / 2) Q_j
            assert (Y - _crt_py(x[lo:hi, k], dig)) % Qj == 0
            assert abs(Y) <= len(dig) * Qj // 2
            # the digit's own limbs are copied
            assert np.array_equal(y[j, lo:hi, k], x[lo:hi, k])


@pytest.mark.parametrize("level", [4, 2])
def test_moddown_is_division_by_P(small, level):
    prm = small
    rng = np.random.default_rng(7)
    ext = prm.q[:level] + prm.p
    Qe = 1
    for q in ext:
        Qe *= q
    P = prm.p[0] * prm.p[1]
    vals = [int(rng.integers(0, 2 ** 62)) * int(rng.integers(0, 2 ** 62)) * int(rng.integers(0, 2 ** 62)) % Qe - Qe // 2
            for _ in range(prm.N)]
    u = np.array([[v % q for v in vals] for q in ext], np.uint64)
    out = O.moddown(prm, u, level)
    Ql = 1
    for q in prm.q[:level]:
        Ql *= q
    for k in range(0, prm.N, 37):
        got = _crt_py(out[:, k], prm.q[:level])
        # out = (U - U~)/P with U~ = U (mod P), |U~| <= K P / 2  =>  |out*P - U| <= K P / 2
        diff = (got * P - vals[k]) % (Ql * P)
        diff = diff - Ql * P if diff > Ql * P // 2 else diff
        assert abs(diff) <= prm.K * P // 2
    # single-coefficient ModDown agrees
    assert np.array_equal(O.moddown_at(prm, u[:, 5], level), out[:, 5])


@pytest.mark.parametrize("level", [4, 3])
def test_rescale_is_exact_rounding(small, level):
    prm = small
    rng = np.random.default_rng(level + 10)
    ct = random_ct(prm, synth.Stream(5), level)
    out = O.rescale(prm, ct, level)
    qt = prm.q[level - 1]
    Qs = 1
    for q in prm.q[:level - 1]:
        Qs *= q
    for p in range(2):
        for k in (0, 3, 99, prm.N - 1):
            Q = Qs * qt
            C = _crt_py(ct[p, :, k], prm.q[:level]) % Q
            want = ((2 * C + qt) // (2 * qt)) % Qs  # round(C / qt), qt odd: no ties
            assert _crt_py(out[p, :, k], prm.q[:level - 1]) % Qs == want
    del rng


def test_hoisting_commutes_with_automorphism(small):
    prm = small
    level = 4
    rng = np.random.default_rng(3)
    d = np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in prm.q[:level]])
    ext = prm.q[:level] + prm.p
    for g in (5, 25, 2 * prm.N - 1):
        a = O.modup(prm, O.automorph_limbs(d, g, prm.log_n, prm.q), level)
        b = np.stack([O.automorph_limbs(O.modup(prm, d, level)[j], g, prm.log_n, ext)
                      for j in range(prm.beta(level))])
        assert np.array_equal(a, b)


def test_keyswitch_decrypt_identity(small):
    prm = small
    cl = Client(prm, 99)
    level = 4
    g = O.galois_of(3, prm.log_n)
    evk = cl.galois_key(g)
    rng = np.random.default_rng(4)
    d = np.stack([rng.integers(0, q, prm.N, dtype=np.uint64) for q in prm.q[:level]])
    u = O.keyswitch(prm, d, evk, level)
    # u0 + u1 s - d s(X^g) must be small (mod Q_l)
    s_l = O.to_rns(cl.s.astype(np.int64), prm.q[:level])
    sg = O.automorph_limbs(s_l, g, prm.log_n, prm.q)
    err = np.zeros((level, prm.N), np.uint64)
    for i, q in enumerate(prm.q[:level]):
        t1 = O.polymul_fast(u[1, i], s_l[i], prm.log_n, q)
        t2 = O.polymul_fast(d[i], sg[i], prm.log_n, q)
        err[i] = (u[0, i].astype(object) + t1.astype(object) - t2.astype(object)) % q
    e = O.crt_centered(prm, err, level).astype(np.float64)
    alpha = prm.alpha
    P = prm.p[0] * prm.p[1]
    Qj = max(prm.q[0] * prm.q[1], prm.q[2] * prm.q[3])
    bound = prm.beta(level) * prm.N * (alpha + 1) / 2 * Qj / P * 6 * 3.2 + (prm.K + 1) / 2 * (1 + prm.N)
    assert np.abs(e).max() <= bound
    assert np.abs(e).max() > 0
    # sampled inner product (definition per coefficient) + ModDown agree with the full key switch
    for k in (0, 77, prm.N - 1):
        col = O.ks_inner_at(prm, d, evk, level, k)
        assert np.array_equal(O.moddown_at(prm, col[0], level), u[0, :, k])
        assert np.array_equal(O.moddown_at(prm, col[1], level), u[1, :, k])


def test_rotation_and_schoolbook_mode(small):
    prm = small
    cl = Client(prm, 5)
    level = 3
    z = synth.Stream(6).uniform(prm.S, -1, 1)
    ct = cl.encrypt_slots(z, level, prm.scale)
    for r in (1, 5, -1):
        g = O.galois_of(r, prm.log_n)
        rc = O.rotate(prm, ct, g, cl.galois_key(g), level)
        assert np.abs(cl.decrypt_slots(rc, level, prm.scale) - np.roll(z, -r)).max() < 1e-3
    g = O.galois_of(2, prm.log_n)
    fast = O.rotate(prm, ct, g, cl.galois_key(g), level)
    O.set_schoolbook(True)
    try:
        slow = O.rotate(prm, ct, g, cl.galois_key(g), level)
    finally:
        O.set_schoolbook(False)
    assert np.array_equal(fast, slow)


def test_mul_pt_and_rescale_decrypt(small):
    prm = small
    cl = Client(prm, 8)
    level = 4
    st = synth.Stream(9)
    z = st.uniform(prm.S, -1, 1)
    w = st.uniform(prm.S, -1, 1)
    delta = 2.0 ** 36  # close to the 40-bit primes, so the rescaled scale stays large
    ct = cl.encrypt_slots(z, level, delta)
    pt = O.encode_rns(prm, w, level, delta)
    out = O.rescale(prm, O.mul_pt(prm, ct, pt, level), level)
    dec = cl.decrypt_slots(out, level - 1, delta * delta / prm.q[level - 1])
    assert np.abs(dec - z * w).max() < 1e-3
    # plaintext product equals the ring product limb by limb
    ring = np.stack([O.polymul_schoolbook(ct[1, i], pt[i], prm.log_n, q) for i, q in enumerate(prm.q[:level])])
    assert np.array_equal(O.mul_pt(prm, ct, pt, level)[1], ring)

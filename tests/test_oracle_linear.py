"""Pins of the oracle's linear layers: decrypt(linear(enc(x))) against the FP64
plaintext layer (paper Sec. 6 correctness method, with the CKKS tolerance),
special matrices whose encrypted result is known in closed form, and the
shuffle-folding algebra of paper Sec. 5."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import synth
from tests.helpers import Client, encode_pts


def _rel_err(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


def run_fc(prm, cl, W, x, n, n1, level, delta):
    sched = O.fc_schedule(n, n1)
    slots = O.fc_slots(W, n, n1, prm.S)
    pts = encode_pts(prm, slots, level, delta)
    ct = cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), level, delta)
    keys = cl.keyset(sched.rotations())
    y = O.linear(prm, ct[None], level, sched, pts, keys)[0]
    yr = O.rescale(prm, y, level)
    z = cl.decrypt_slots(yr, level - 1, delta * delta / prm.q[level - 1])
    return z.real, y, yr


@pytest.fixture(scope="module")
def c1():
    """Plain diagonal method workload: N=2^12, 3 x 36-bit q + 1 special, dnum 3, scale 2^30."""
    return O.make_params(12, 3, 1, 3, 36, 2.0 ** 30)


@pytest.mark.slow
def test_fc_plain_c1(c1):
    prm = c1
    st = synth.Stream(synth.master_seed(1))
    W = st.sub(synth.TAG_W).uniform(64 * 64, -1, 1).reshape(64, 64)
    x = st.sub(synth.TAG_X).uniform(64, -1, 1)
    cl = Client(prm, synth.master_seed(1))
    z, _, _ = run_fc(prm, cl, W, x, 64, 64, 3, prm.scale)
    ref = W @ x
    assert _rel_err(z[:64], ref) < 1e-3
    # the replicas agree too
    assert _rel_err(z[64:128], ref) < 1e-3


@pytest.fixture(scope="module")
def small():
    return O.make_params(10, 4, 2, 2, 50, 2.0 ** 40)


def test_fc_bsgs_small(small):
    prm = small
    st = synth.Stream(77)
    W = st.he_normal((64, 64), 64)
    x = st.uniform(64, 0, 1)
    cl = Client(prm, 78)
    z, _, _ = run_fc(prm, cl, W, x, 64, 8, 4, prm.scale)
    assert _rel_err(z[:64], W @ x) < 1e-3


def test_fc_nonsquare_padded(small):
    prm = small
    st = synth.Stream(79)
    W = st.he_normal((20, 64), 64)
    x = st.uniform(64, 0, 1)
    cl = Client(prm, 80)
    z, _, _ = run_fc(prm, cl, W, x, 64, 16, 3, prm.scale)
    assert _rel_err(z[:20], W @ x) < 1e-3
    assert np.abs(z[20:64]).max() < 1e-3 * np.abs(W @ x).max()


def test_identity_uses_only_diagonal_zero(small):
    """W = I: every diagonal but d_0 is zero, so the layer is pt-mult by 1s + rescale."""
    prm = small
    cl = Client(prm, 81)
    x = synth.Stream(82).uniform(64, -1, 1)
    z, y, _ = run_fc(prm, cl, np.eye(64), x, 64, 8, 3, prm.scale)
    assert _rel_err(z[:64], x) < 1e-3
    # the same result straight from pt-mult with the all-ones diagonal
    ct = cl.encrypt_slots(O.fc_input_slots(x, 64, prm.S), 3, prm.scale)  # fresh randomness: compare decryptions
    ones = O.encode_rns(prm, np.ones(prm.S), 3, prm.scale)
    direct = O.rescale(prm, O.mul_pt(prm, ct, ones, 3), 3)
    zd = cl.decrypt_slots(direct, 2, prm.scale * prm.scale / prm.q[2])
    assert np.abs(zd.real - z).max() < 1e-3


def test_single_diagonal_is_one_rotation(small):
    """W with only diagonal 5 nonzero: y = d_5 * rot_5(x)."""
    prm = small
    cl = Client(prm, 83)
    n = 64
    st = synth.Stream(84)
    dvals = st.uniform(n, -1, 1)
    W = np.zeros((n, n))
    for r in range(n):
        W[r, (r + 5) % n] = dvals[r]
    x = st.uniform(n, -1, 1)
    z, _, _ = run_fc(prm, cl, W, x, n, 8, 3, prm.scale)
    assert _rel_err(z[:n], dvals * np.roll(x, -5)) < 1e-3


def test_shuffle_folding_probes(small):
    """Paper Sec. 5: with output shuffling, probing e_i returns column i of W in
    the permuted order; with input and output shuffling, column sigma_in(i)."""
    prm = small
    cl = Client(prm, 85)
    n = 64
    st = synth.Stream(86)
    W = st.he_normal((n, n), n)
    p_out = st.permutation(n)
    p_in = st.permutation(n)
    Wp = O.fold_permutations(W, p_out, p_in)
    for i in (0, 13):
        e = np.zeros(n)
        e[i] = 1.0
        z, _, _ = run_fc(prm, cl, Wp, e, n, 8, 3, prm.scale)
        assert np.abs(z[:n] - W[p_out, p_in[i]]).max() < 1e-3 * np.abs(W).max()
    # and the folded layer computes P_out W P_in^T on a general input
    x = st.uniform(n, 0, 1)
    z, _, _ = run_fc(prm, cl, Wp, x, n, 8, 3, prm.scale)
    x_orig = np.zeros(n)
    x_orig[p_in] = x  # x'_u = x_{sigma_in(u)}
    assert _rel_err(z[:n], (W @ x_orig)[p_out]) < 1e-3


@pytest.mark.parametrize("c_in,c_out,k,n1", [(8, 8, 3, 1), (16, 16, 3, 1), (3, 16, 3, 1), (16, 8, 1, 1),
                                             (16, 16, 3, 4), (16, 8, 1, 2), (3, 16, 3, 2)])
def test_conv_multiplexed(small, c_in, c_out, k, n1):
    prm = small
    cs = O.ConvShape(c_in, c_out, 8, 8, k)
    st = synth.Stream(100 + c_in + c_out + k)
    W = st.he_normal((c_out, c_in, k, k), c_in * k * k)
    perm = st.permutation(c_out)
    Wp = O.fold_permutations(W, perm, None)
    x = st.uniform(c_in * 64, 0, 1).reshape(c_in, 8, 8)
    sched = O.conv_schedule(cs, prm.S, n1)
    level = 3
    pts = encode_pts(prm, O.conv_slots(Wp, cs, prm.S, n1), level, prm.scale)
    cl = Client(prm, 200 + c_in)
    xs = O.conv_input_slots(x, cs, prm.S)
    cts = np.stack([cl.encrypt_slots(xs[i], level, prm.scale) for i in range(sched.n_in)])
    y = O.linear(prm, cts, level, sched, pts, cl.keyset(sched.rotations()))
    dec = np.stack([cl.decrypt_slots(O.rescale(prm, y[o], level), level - 1,
                                     prm.scale * prm.scale / prm.q[level - 1]).real for o in range(sched.n_out)])
    got = O.conv_output_from_slots(dec, cs, prm.S)
    ref = O.conv_ref(Wp, x)
    assert _rel_err(got, ref) < 1e-3
    # counts: hoisted baby key switches per input ct, giant ones per output ct
    assert len([r for r in sched.rb if r]) == n1 * k * k - 1
    assert sched.G == cs.per_ct(prm.S) // n1


def test_linear_schoolbook_mode_identical():
    prm = O.make_params(7, 3, 1, 3, 40, 2.0 ** 30)
    cl = Client(prm, 300)
    st = synth.Stream(301)
    W = st.uniform(16 * 16, -1, 1).reshape(16, 16)
    sched = O.fc_schedule(16, 4)
    pts = encode_pts(prm, O.fc_slots(W, 16, 4, prm.S), 3, prm.scale)
    ct = cl.encrypt_slots(O.fc_input_slots(st.uniform(16, -1, 1), 16, prm.S), 3, prm.scale)
    keys = cl.keyset(sched.rotations())
    a = O.linear(prm, ct[None], 3, sched, pts, keys)
    O.set_schoolbook(True)
    try:
        b = O.linear(prm, ct[None], 3, sched, pts, keys)
    finally:
        O.set_schoolbook(False)
    assert np.array_equal(a, b)


def test_missing_key_reported(small):
    prm = small
    cl = Client(prm, 400)
    sched = O.fc_schedule(64, 8)
    pts = np.zeros((1, 1, sched.G, sched.B, 3 + prm.K, prm.N), np.uint64)
    ct = np.zeros((1, 2, 3, prm.N), np.uint64)
    keys = cl.keyset([1, 2])
    with pytest.raises(KeyError):
        O.linear(prm, ct, 3, sched, pts, keys)
    with pytest.raises(KeyError):
        O.linear(prm, ct, 3, sched, pts, keys, hoist_moddown=True)


# ---------------------------------------------------------------------------
# the double-hoisted schedule (ModDown hoisted out of baby and giant steps)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,n1", [(64, 8), (64, 64), (64, 1)])
def test_fc_double_hoisted_decrypts(small, n, n1):
    prm = small
    st = synth.Stream(500 + n1)
    W = st.he_normal((n, n), n)
    x = st.uniform(n, 0, 1)
    cl = Client(prm, 501)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), 4, prm.scale)
    ct = cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), 4, prm.scale)
    keys = cl.keyset(sched.rotations())
    y_dh = O.linear(prm, ct[None], 4, sched, pts, keys, hoist_moddown=True)[0]
    y_std = O.linear(prm, ct[None], 4, sched, pts, keys)[0]
    z_dh = cl.decrypt_slots(O.rescale(prm, y_dh, 4), 3, prm.scale ** 2 / prm.q[3]).real
    z_std = cl.decrypt_slots(O.rescale(prm, y_std, 4), 3, prm.scale ** 2 / prm.q[3]).real
    assert _rel_err(z_dh[:n], W @ x) < 1e-3
    # both schedules compute the same layer; they differ only in rounding noise
    assert np.abs(z_dh - z_std).max() < 1e-6 * np.abs(W @ x).max() * 1e3
    if n1 > 1:
        assert not np.array_equal(y_dh, y_std)


@pytest.mark.parametrize("n1", [1, 4])
def test_conv_double_hoisted_decrypts(small, n1):
    prm = small
    cs = O.ConvShape(16, 16, 8, 8, 3)
    st = synth.Stream(510)
    W = st.he_normal((16, 16, 3, 3), 144)
    x = st.uniform(16 * 64, 0, 1).reshape(16, 8, 8)
    sched = O.conv_schedule(cs, prm.S, n1)
    pts = encode_pts(prm, O.conv_slots(W, cs, prm.S, n1), 3, prm.scale)
    cl = Client(prm, 511)
    xs = O.conv_input_slots(x, cs, prm.S)
    cts = np.stack([cl.encrypt_slots(xs[i], 3, prm.scale) for i in range(sched.n_in)])
    y = O.linear(prm, cts, 3, sched, pts, cl.keyset(sched.rotations()), hoist_moddown=True)
    dec = np.stack([cl.decrypt_slots(O.rescale(prm, y[o], 3), 2, prm.scale ** 2 / prm.q[2]).real
                    for o in range(sched.n_out)])
    assert _rel_err(O.conv_output_from_slots(dec, cs, prm.S), O.conv_ref(W, x)) < 1e-3


def test_double_hoisted_identity_exact_division():
    """W = I with n1 = n: only the r=0 baby step and G=0 giant step contribute, so the
    result is exactly ModDown((P x0, P x1) * pt) = x * pt (the P factor divides out with
    no rounding: P*v has zero residues mod every p_k)."""
    prm = O.make_params(8, 3, 2, 3, 40, 2.0 ** 30)
    cl = Client(prm, 520)
    n = 16
    sched = O.fc_schedule(n, n)
    pts = encode_pts(prm, O.fc_slots(np.eye(n), n, n, prm.S), 3, prm.scale)
    ct = cl.encrypt_slots(O.fc_input_slots(synth.Stream(521).uniform(n, -1, 1), n, prm.S), 3, prm.scale)
    y = O.linear(prm, ct[None], 3, sched, pts, cl.keyset(sched.rotations()), hoist_moddown=True)[0]
    assert np.array_equal(y, O.mul_pt(prm, ct, pts[0, 0, 0, 0, :3], 3))


def test_double_hoisted_schoolbook_identical():
    prm = O.make_params(7, 3, 1, 3, 40, 2.0 ** 30)
    cl = Client(prm, 530)
    st = synth.Stream(531)
    W = st.uniform(16 * 16, -1, 1).reshape(16, 16)
    sched = O.fc_schedule(16, 4)
    pts = encode_pts(prm, O.fc_slots(W, 16, 4, prm.S), 3, prm.scale)
    ct = cl.encrypt_slots(O.fc_input_slots(st.uniform(16, -1, 1), 16, prm.S), 3, prm.scale)
    keys = cl.keyset(sched.rotations())
    a = O.linear(prm, ct[None], 3, sched, pts, keys, hoist_moddown=True)
    O.set_schoolbook(True)
    try:
        b = O.linear(prm, ct[None], 3, sched, pts, keys, hoist_moddown=True)
    finally:
        O.set_schoolbook(False)
    assert np.array_equal(a, b)

"""GPU parity of whole linear layers against the oracle: bit-exact output
ciphertexts (coefficient domain) from shared integer plaintexts, decryptions
within 1e-3 of the FP64 layer, batches of uneven levels, and the library's own
weight encoding (within one unit per coefficient of the oracle's encoding)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import synth
from tests.gpu_util import ctx_for, dev, host, keys_at, pad_cts
from tests.helpers import Client, encode_pts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from paper_2509_01253_amd import fhelin
    return fhelin


def _rel(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


class Layer:
    """A layer evaluated on the GPU through the C ABI."""

    def __init__(self, F, prm, keys, pts, level_keys, **desc):
        self.F, self.prm = F, prm
        self.ctx = ctx_for(F, prm)
        kind = F.FHELIN_LAYER_FC if "fc_n" in desc else F.FHELIN_LAYER_CONV
        self.plan = F.fhelin_plan_create(self.ctx, kind, **desc)
        self.info = F.fhelin_plan_info(self.plan)
        self.ks = None
        if keys.galois:
            assert F.fhelin_plan_galois(self.plan) == keys.galois
            self.ks = F.fhelin_keyset_load(self.ctx, keys.galois, level_keys, dev(keys_at(prm, keys, level_keys)))
        self.pset = None
        if pts is not None:
            self.pset = F.fhelin_pt_import(self.ctx, dev(pts.reshape(-1, pts.shape[-2], prm.N)),
                                           level=pts.shape[-2] - prm.K)

    def apply(self, cts, levels, rescale=True, stride=None, dh=False):
        prm, F = self.prm, self.F
        stride = stride or max(levels)
        x = dev(pad_cts(cts, stride, prm.N))
        n_out = len(cts) // self.info["n_in"] * self.info["n_out"]
        req_levels = [levels[r * self.info["n_in"]] for r in range(len(cts) // self.info["n_in"])]
        out_levels = [l - 1 if rescale else l for l in req_levels for _ in range(self.info["n_out"])]
        y = dev(np.zeros((n_out, 2, stride, prm.N), np.uint64))
        flags = (F.FHELIN_APPLY_RESCALE if rescale else 0) | (F.FHELIN_APPLY_HOIST_MODDOWN if dh else 0)
        F.fhelin_linear_apply(self.ctx, self.plan, self.ks, self.pset, x, levels, y, out_levels, flags)
        got = host(y)
        return [got[t, :, : out_levels[t]] for t in range(n_out)]

    def close(self):
        F = self.F
        if self.pset is not None:
            F.fhelin_ptset_release(self.pset)
        if self.ks is not None:
            F.fhelin_keyset_release(self.ks)
        F.fhelin_plan_destroy(self.plan)
        F.fhelin_ctx_destroy(self.ctx)


def test_fc_plain_c1_bit_exact(F):
    """N=2^12, 3 x 36-bit q + 1 special, dnum 3, scale 2^30, FC 64x64 U[-1,1],
    plain diagonal method (63 hoisted rotations), one rescale."""
    print("c1 plain FC", flush=True)
    prm = O.make_params(12, 3, 1, 3, 36, 2.0 ** 30)
    st = synth.Stream(synth.master_seed(1))
    W = st.sub(synth.TAG_W).uniform(64 * 64, -1, 1).reshape(64, 64)
    x = st.sub(synth.TAG_X).uniform(64, -1, 1)
    cl = Client(prm, synth.master_seed(1))
    sched = O.fc_schedule(64, 64)
    pts = encode_pts(prm, O.fc_slots(W, 64, 64, prm.S), 3, prm.scale)
    keys = cl.keyset(sched.rotations())
    ct = cl.encrypt_slots(O.fc_input_slots(x, 64, prm.S), 3, prm.scale)
    want = O.rescale(prm, O.linear(prm, ct[None], 3, sched, pts, keys)[0], 3)
    lay = Layer(F, prm, keys, pts, 3, fc_n=64, fc_out=64, fc_in=64, n1=64)
    try:
        got = lay.apply([ct], [3])[0]
        assert np.array_equal(got, want)
        z = cl.decrypt_slots(got, 2, prm.scale ** 2 / prm.q[2]).real
        assert _rel(z[:64], W @ x) < 1e-3
    finally:
        lay.close()


def test_fc_bsgs_uneven_levels_batch(F):
    """A batch of requests at different levels in one call: each output equals the
    oracle's, and equals the same request evaluated alone."""
    print("bsgs uneven batch", flush=True)
    prm = O.make_params(12, 6, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(4000)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 4001)
    keys = cl.keyset(sched.rotations())
    levels = [6, 2, 4, 5, 3, 6, 2]
    xs = [st.uniform(n, 0, 1) for _ in levels]
    cts = [cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), l, prm.scale) for x, l in zip(xs, levels)]
    lay = Layer(F, prm, keys, pts, prm.L, fc_n=n, fc_out=n, fc_in=n, n1=n1)
    try:
        got = lay.apply(cts, levels, stride=prm.L)
        for t, l in enumerate(levels):
            want = O.rescale(prm, O.linear(prm, cts[t][None], l, sched, pts, keys)[0], l)
            assert np.array_equal(got[t], want), t
            z = cl.decrypt_slots(got[t], l - 1, prm.scale ** 2 / prm.q[l - 1]).real
            assert _rel(z[:n], W @ xs[t]) < 1e-3, t
        alone = lay.apply([cts[3]], [levels[3]], stride=prm.L)[0]
        assert np.array_equal(alone, got[3])
        # no rescale: outputs at the input level
        norsc = lay.apply(cts[:2], levels[:2], rescale=False, stride=prm.L)
        for t in range(2):
            assert np.array_equal(norsc[t], O.linear(prm, cts[t][None], levels[t], sched, pts, keys)[0])
    finally:
        lay.close()


@pytest.mark.parametrize("c_in,c_out,k,n1", [(16, 16, 3, 1), (3, 16, 3, 1), (16, 8, 1, 1), (16, 16, 3, 4), (16, 8, 1, 8)])
def test_conv_multi_ct_bit_exact(F, c_in, c_out, k, n1):
    print(f"conv {c_in}->{c_out} k{k} n1={n1}", flush=True)
    prm = O.make_params(10, 4, 2, 2, 50, 2.0 ** 40)
    cs = O.ConvShape(c_in, c_out, 8, 8, k)
    st = synth.Stream(4100 + c_in + k)
    W = st.he_normal((c_out, c_in, k, k), c_in * k * k)
    sched = O.conv_schedule(cs, prm.S, n1)
    level = 3
    pts = encode_pts(prm, O.conv_slots(W, cs, prm.S, n1), level, prm.scale)
    cl = Client(prm, 4200 + c_in)
    keys = cl.keyset(sched.rotations())
    reqs = 2
    xs = [st.uniform(c_in * 64, 0, 1).reshape(c_in, 8, 8) for _ in range(reqs)]
    cts = []
    for x in xs:
        slots = O.conv_input_slots(x, cs, prm.S)
        cts += [cl.encrypt_slots(slots[i], level, prm.scale) for i in range(sched.n_in)]
    lay = Layer(F, prm, keys, pts, level, c_in=c_in, c_out=c_out, h=8, w=8, k=k, n1=n1)
    try:
        assert lay.info["n_in"] == sched.n_in and lay.info["n_out"] == sched.n_out
        assert F.fhelin_plan_rotations(lay.plan) == (sched.rb, sched.gk)
        got = lay.apply(cts, [level] * len(cts))
        for r in range(reqs):
            want = O.linear(prm, np.stack(cts[r * sched.n_in:(r + 1) * sched.n_in]), level, sched, pts, keys)
            for o in range(sched.n_out):
                assert np.array_equal(got[r * sched.n_out + o], O.rescale(prm, want[o], level)), (r, o)
            dec = np.stack([cl.decrypt_slots(got[r * sched.n_out + o], level - 1,
                                             prm.scale ** 2 / prm.q[level - 1]).real for o in range(sched.n_out)])
            assert _rel(O.conv_output_from_slots(dec, cs, prm.S), O.conv_ref(W, xs[r])) < 1e-3
    finally:
        lay.close()


def test_conv_c2_full(F):
    """ResNet-20-block conv 3x3 16->16 on 32x32, N=2^15, 8 + 2 primes (50-bit),
    dnum 4, scale 2^40, channel shuffle folded: bit-exact + decrypt 1e-3."""
    print("c2 conv full", flush=True)
    prm = O.make_params(15, 8, 2, 4, 50, 2.0 ** 40)
    cs = O.ConvShape(16, 16, 32, 32, 3)
    st = synth.Stream(synth.master_seed(2))
    W = st.sub(synth.TAG_W).he_normal((16, 16, 3, 3), 144)
    perm = st.sub(synth.TAG_PERM).permutation(16)
    Wp = O.fold_permutations(W, perm, None)
    x = st.sub(synth.TAG_X).uniform(16 * 32 * 32, 0, 1).reshape(16, 32, 32)
    sched = O.conv_schedule(cs, prm.S)
    pts = encode_pts(prm, O.conv_slots(Wp, cs, prm.S), 8, prm.scale)
    cl = Client(prm, synth.master_seed(2))
    keys = cl.keyset(sched.rotations())
    ct = cl.encrypt_slots(O.conv_input_slots(x, cs, prm.S)[0], 8, prm.scale)
    want = O.rescale(prm, O.linear(prm, ct[None], 8, sched, pts, keys)[0], 8)
    lay = Layer(F, prm, keys, pts, 8, c_in=16, c_out=16, h=32, w=32, k=3)
    try:
        got = lay.apply([ct], [8])[0]
        assert np.array_equal(got, want)
        z = cl.decrypt_slots(got, 7, prm.scale ** 2 / prm.q[7]).real
        assert _rel(O.conv_output_from_slots(z[None], cs, prm.S), O.conv_ref(Wp, x)) < 1e-3
    finally:
        lay.close()


def test_encode_within_one_unit(F):
    import torch
    print("encode", flush=True)
    for log_n in (12, 16):
        prm = O.make_params(log_n, 3, 1, 3, 50, 2.0 ** 40)
        ctx = ctx_for(F, prm)
        try:
            st = synth.Stream(4300 + log_n)
            z = np.stack([st.uniform(prm.S, -1, 1), st.he_normal(prm.S, 16), np.full(prm.S, 0.25)])
            pset = F.fhelin_pt_encode(ctx, torch.from_numpy(z).cuda(), 3, prm.scale)
            out = dev(np.zeros((3, 3 + prm.K, prm.N), np.uint64))
            F.fhelin_pt_export(ctx, pset, 3, out)
            got = host(out)
            for i in range(3):
                m = O.encode(z[i], log_n, prm.scale)
                for j, q in enumerate(prm.q[:3] + prm.p):
                    d = (got[i, j].astype(object) - O.to_rns(m, [q])[0].astype(object)) % q
                    d = np.array([v if v <= q // 2 else v - q for v in d], dtype=np.int64)
                    assert np.abs(d).max() <= 1, (log_n, i, j)
                    assert np.mean(d != 0) < 1e-3
            # the constant vector encodes exactly
            assert np.array_equal(got[2, 0], O.to_rns(O.encode(z[2], log_n, prm.scale), [prm.q[0]])[0])
            F.fhelin_ptset_release(pset)
        finally:
            F.fhelin_ctx_destroy(ctx)


@pytest.mark.parametrize("kind", ["fc", "conv", "conv_n1"])
def test_encode_weights_with_shuffle(F, kind):
    """Weights -> folded diagonals -> encode on the GPU, against the oracle's slot
    vectors and encoding (one unit per coefficient), then decrypt(layer) vs FP64."""
    import torch
    print(f"encode weights {kind}", flush=True)
    prm = O.make_params(11, 4, 2, 2, 50, 2.0 ** 40)
    st = synth.Stream(4400)
    cl = Client(prm, 4401)
    level = 4
    if kind == "fc":
        n, n1, fo, fi = 128, 16, 100, 128
        W = st.he_normal((fo, fi), fi)
        po, pi = st.permutation(fo), st.permutation(fi)
        Wp = O.fold_permutations(W, po, pi)
        sched = O.fc_schedule(n, n1)
        slots = O.fc_slots(Wp, n, n1, prm.S)
        desc = dict(fc_n=n, fc_out=fo, fc_in=fi, n1=n1)
        x = st.uniform(fi, 0, 1)
        xs = [O.fc_input_slots(x, n, prm.S)]
        ref = (Wp @ x)
    else:
        n1 = 4 if kind == "conv_n1" else 1
        cs = O.ConvShape(8, 16, 8, 8, 3)
        W = st.he_normal((16, 8, 3, 3), 72)
        po, pi = st.permutation(16), st.permutation(8)
        Wp = O.fold_permutations(W, po, pi)
        sched = O.conv_schedule(cs, prm.S, n1)
        slots = O.conv_slots(Wp, cs, prm.S, n1)
        desc = dict(c_in=8, c_out=16, h=8, w=8, k=3, n1=n1)
        x = st.uniform(8 * 64, 0, 1).reshape(8, 8, 8)
        xs = list(O.conv_input_slots(x, cs, prm.S))
        ref = O.conv_ref(Wp, x)
    keys = cl.keyset(sched.rotations())
    lay = Layer(F, prm, keys, None, level, **desc)
    try:
        lay.pset = F.fhelin_plan_encode_weights(
            lay.ctx, lay.plan, torch.from_numpy(np.ascontiguousarray(W)).cuda(),
            torch.from_numpy(po).cuda(), torch.from_numpy(pi).cuda(), level, prm.scale)
        n_pt = lay.info["n_pt"]
        out = dev(np.zeros((n_pt, level + prm.K, prm.N), np.uint64))
        F.fhelin_pt_export(lay.ctx, lay.pset, level, out)
        got = host(out)
        want = encode_pts(prm, slots, level, prm.scale).reshape(n_pt, level + prm.K, prm.N)
        # every q and p row: the residues of one integer polynomial that differs from
        # the oracle's encoding by at most one unit per coefficient, the same
        # difference on every row (both sides round in FP64, in different orders)
        d0 = None
        for j, q in enumerate(prm.q[:level] + prm.p):
            d = (got[:, j].astype(np.int64) - want[:, j].astype(np.int64))
            d = np.where(d > q // 2, d - q, np.where(d < -(q // 2), d + q, d))
            assert np.abs(d).max() <= 1, j
            if d0 is None:
                d0 = d
            assert np.array_equal(d, d0), j
        assert np.mean(d0 != 0) < 1e-3
        cts = [cl.encrypt_slots(s, level, prm.scale) for s in xs]
        res = lay.apply(cts, [level] * len(cts))
        dec = np.stack([cl.decrypt_slots(r, level - 1, prm.scale ** 2 / prm.q[level - 1]).real for r in res])
        if kind == "fc":
            assert _rel(dec[0][:100], ref) < 1e-3
        else:
            assert _rel(O.conv_output_from_slots(dec, cs, prm.S), ref) < 1e-3
    finally:
        lay.close()


# ---------------------------------------------------------------------------
# the double-hoisted schedule
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n1", [8, 64, 1])
def test_fc_double_hoisted_bit_exact(F, n1):
    print(f"dh fc n1={n1}", flush=True)
    prm = O.make_params(12, 6, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(4500 + n1)
    n = 64
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 4501)
    keys = cl.keyset(sched.rotations())
    levels = [6, 2, 5, 3]
    xs = [st.uniform(n, 0, 1) for _ in levels]
    cts = [cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), l, prm.scale) for x, l in zip(xs, levels)]
    lay = Layer(F, prm, keys, pts, prm.L, fc_n=n, fc_out=n, fc_in=n, n1=n1)
    try:
        got = lay.apply(cts, levels, stride=prm.L, dh=True)
        for t, l in enumerate(levels):
            want = O.rescale(prm, O.linear(prm, cts[t][None], l, sched, pts, keys, hoist_moddown=True)[0], l)
            assert np.array_equal(got[t], want), t
            z = cl.decrypt_slots(got[t], l - 1, prm.scale ** 2 / prm.q[l - 1]).real
            assert _rel(z[:n], W @ xs[t]) < 1e-3, t
        nr = lay.apply(cts[:1], levels[:1], rescale=False, stride=prm.L, dh=True)[0]
        assert np.array_equal(nr, O.linear(prm, cts[0][None], levels[0], sched, pts, keys, hoist_moddown=True)[0])
    finally:
        lay.close()


@pytest.mark.parametrize("c_in,c_out,k,n1", [(16, 16, 3, 1), (16, 8, 1, 1), (16, 16, 3, 4), (16, 16, 3, 2)])
def test_conv_double_hoisted_bit_exact(F, c_in, c_out, k, n1):
    print(f"dh conv {c_in}->{c_out} k{k} n1={n1}", flush=True)
    prm = O.make_params(10, 4, 2, 2, 50, 2.0 ** 40)
    cs = O.ConvShape(c_in, c_out, 8, 8, k)
    st = synth.Stream(4600 + k)
    W = st.he_normal((c_out, c_in, k, k), c_in * k * k)
    sched = O.conv_schedule(cs, prm.S, n1)
    level = 3
    pts = encode_pts(prm, O.conv_slots(W, cs, prm.S, n1), level, prm.scale)
    cl = Client(prm, 4601)
    keys = cl.keyset(sched.rotations())
    x = st.uniform(c_in * 64, 0, 1).reshape(c_in, 8, 8)
    slots = O.conv_input_slots(x, cs, prm.S)
    cts = [cl.encrypt_slots(slots[i], level, prm.scale) for i in range(sched.n_in)]
    lay = Layer(F, prm, keys, pts, level, c_in=c_in, c_out=c_out, h=8, w=8, k=k, n1=n1)
    try:
        got = lay.apply(cts, [level] * len(cts), dh=True)
        want = O.linear(prm, np.stack(cts), level, sched, pts, keys, hoist_moddown=True)
        for o in range(sched.n_out):
            assert np.array_equal(got[o], O.rescale(prm, want[o], level)), o
    finally:
        lay.close()


# ---------------------------------------------------------------------------
# tile / chunk choices and the autotuner
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dh", [False, True])
def test_tunes_bit_identical_and_autotune(F, dh):
    """Every tune (chunk, key-switch entry group, MAC requests per thread) gives the
    oracle's ciphertexts bit for bit on a batch of uneven levels; the autotuner keeps
    a valid tune and leaves the layer's result in the output."""
    print(f"tunes dh={dh}", flush=True)
    prm = O.make_params(12, 5, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(4700 + dh)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 4701)
    keys = cl.keyset(sched.rotations())
    levels = [5, 2, 4, 3, 5, 2, 3, 4, 5, 3, 2]
    cts = [cl.encrypt_slots(O.fc_input_slots(st.uniform(n, 0, 1), n, prm.S), l, prm.scale) for l in levels]
    want = [O.rescale(prm, O.linear(prm, c[None], l, sched, pts, keys, hoist_moddown=dh)[0], l)
            for c, l in zip(cts, levels)]
    lay = Layer(F, prm, keys, pts, prm.L, fc_n=n, fc_out=n, fc_in=n, n1=n1)
    try:
        assert F.fhelin_plan_get_tune(lay.plan) == {"chunk": 0, "ks_eg": 16, "mac_my": 2, "ntt_threads": 256,
                                                     "persistent": 0, "fuse_baby": 0}
        for tune in [dict(chunk=0, ks_eg=8, mac_my=2), dict(chunk=4, ks_eg=3, mac_my=4),
                     dict(chunk=1, ks_eg=16, mac_my=8), dict(chunk=5, ks_eg=1, mac_my=2),
                     dict(chunk=0, ks_eg=8, mac_my=4, fuse_baby=1), dict(chunk=3, ks_eg=4, mac_my=8, fuse_baby=1)]:
            F.fhelin_plan_set_tune(lay.plan, **tune)
            got = lay.apply(cts, levels, stride=prm.L, dh=dh)
            for t in range(len(levels)):
                assert np.array_equal(got[t], want[t]), (tune, t)
        with pytest.raises(F.FhelinError):
            F.fhelin_plan_set_tune(lay.plan, chunk=0, ks_eg=8, mac_my=3)
        with pytest.raises(F.FhelinError):
            F.fhelin_plan_set_tune(lay.plan, chunk=65, ks_eg=8, mac_my=8)
        F.fhelin_plan_set_tune(lay.plan, chunk=0, ks_eg=8, mac_my=8)
        x = dev(pad_cts(cts, prm.L, prm.N))
        y = dev(np.zeros((len(cts), 2, prm.L, prm.N), np.uint64))
        flags = F.FHELIN_APPLY_RESCALE | (F.FHELIN_APPLY_HOIST_MODDOWN if dh else 0)
        best, ms = F.fhelin_plan_autotune(lay.ctx, lay.plan, [lay.ks] * len(cts), lay.pset, x, levels, y,
                                          [l - 1 for l in levels], flags)
        print("autotune", best, f"{ms:.3f} ms", flush=True)
        assert best == F.fhelin_plan_get_tune(lay.plan)
        assert best["mac_my"] in (2, 4, 8) and best["ks_eg"] in (4, 8, 16) and best["chunk"] in (0, 32, 16, 8, 4)
        assert ms >= 0
        got = host(y)
        for t, l in enumerate(levels):
            assert np.array_equal(got[t, :, : l - 1], want[t]), t
    finally:
        lay.close()


# ---------------------------------------------------------------------------
# baby rotations inside the multiply-accumulate
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["fc", "conv"])
def test_fused_baby_rotations_bit_exact(F, kind):
    """The double-hoisted schedule with its baby rotations computed inside the
    multiply-accumulate (one key set for the chunk) against the separate rotation
    launch and the oracle, bit for bit: N = 2^12 with 12 q + 3 p primes and dnum 4
    (requests of 1 to 4 digits at uneven levels), every MAC tile (2, 4, 8 requests per
    thread); FC with 32 baby x 4 giant steps (two 16-term chunks) and a 3x3 conv over
    two input and two output ciphertexts (an identity baby step per input)."""
    print(f"fused baby rotations {kind}", flush=True)
    prm = O.make_params(12, 12, 3, 4, 50, 2.0 ** 40)
    st = synth.Stream(5400 + (kind == "conv"))
    cl = Client(prm, 5401)
    if kind == "fc":
        n, n1 = 128, 32
        W = st.he_normal((n, n), n)
        sched = O.fc_schedule(n, n1)
        pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
        levels = [12, 10, 9, 7, 4, 2, 11, 1, 6]
        cts = [cl.encrypt_slots(O.fc_input_slots(st.uniform(n, 0, 1), n, prm.S), l, prm.scale) for l in levels]
        desc = dict(fc_n=n, fc_out=n, fc_in=n, n1=n1)
        reqs = [[c] for c in cts]
    else:
        cs = O.ConvShape(16, 16, 16, 16, 3)
        W = st.he_normal((16, 16, 3, 3), 144)
        sched = O.conv_schedule(cs, prm.S)
        assert sched.n_in == 2 and sched.n_out == 2
        pts = encode_pts(prm, O.conv_slots(W, cs, prm.S), prm.L, prm.scale)
        req_levels = [12, 9, 5, 3]
        reqs = [[cl.encrypt_slots(sl, l, prm.scale)
                 for sl in O.conv_input_slots(st.uniform(16 * 256, 0, 1).reshape(16, 16, 16), cs, prm.S)]
                for l in req_levels]
        levels = [l for l in req_levels for _ in range(2)]
        cts = [c for r in reqs for c in r]
        desc = dict(c_in=16, c_out=16, h=16, w=16, k=3)
    keys = cl.keyset(sched.rotations())
    lay = Layer(F, prm, keys, pts, prm.L, **desc)
    try:
        outs = {}
        for fuse in (1, 0):
            for my in (2, 4, 8):
                F.fhelin_plan_set_tune(lay.plan, mac_my=my, fuse_baby=fuse)
                F.fhelin_profile_enable(lay.ctx, True)
                outs[(fuse, my)] = lay.apply(cts, levels, rescale=False, stride=prm.L, dh=True)
                n_fused = F.fhelin_profile_read(lay.ctx, "rot_mac")[0]
                n_rot = F.fhelin_profile_read(lay.ctx, "ks_rot")[0]
                F.fhelin_profile_enable(lay.ctx, False)
                assert (n_fused > 0, n_rot > 0) == ((True, False) if fuse else (False, True)), (fuse, my)
        n_out = sched.n_out
        for r, req in enumerate(reqs):
            l = levels[r * len(req)]
            want = O.linear(prm, np.stack(req), l, sched, pts, keys, hoist_moddown=True)
            for o in range(n_out):
                for key, got in outs.items():
                    assert np.array_equal(got[r * n_out + o], want[o]), (key, r, o, l)
    finally:
        lay.close()


# ---------------------------------------------------------------------------
# requests of several clients in one call
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dh,extra", [(False, True), (True, False), (True, True)])
def test_multi_client_batch(F, dh, extra):
    """Requests of three clients with their own secret and Galois keys share one call
    (fhelin_linear_apply_multi): every output equals the oracle evaluated with that
    client's keys and decrypts under that client's secret.  With `extra` one client's
    key set holds an additional key, so its keys sit at other indices than the
    others' (the double-hoisted schedule then runs the baby rotations one launch each
    instead of all in one)."""
    print(f"multi-client dh={dh} extra={extra}", flush=True)
    prm = O.make_params(12, 5, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(4800 + dh)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    clients = [Client(prm, 4810 + i) for i in range(3)]
    rots = sched.rotations()
    keysets = [cl.keyset(rots) for cl in clients[:2]] + [clients[2].keyset(list(rots) + ([10] if extra else []))]
    assert len(keysets[2].galois) == len(keysets[0].galois) + int(extra)
    owner = [0, 1, 2, 0, 2, 1, 2]
    levels = [5, 3, 4, 2, 5, 4, 3]
    xs = [st.uniform(n, 0, 1) for _ in owner]
    cts = [clients[o].encrypt_slots(O.fc_input_slots(x, n, prm.S), l, prm.scale) for o, x, l in zip(owner, xs, levels)]
    ctx = ctx_for(F, prm)
    try:
        plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=n, fc_out=n, fc_in=n, n1=n1)
        handles = [F.fhelin_keyset_load(ctx, ks.galois, prm.L, dev(keys_at(prm, ks, prm.L))) for ks in keysets]
        pset = F.fhelin_pt_import(ctx, dev(pts.reshape(-1, prm.L + prm.K, prm.N)), level=prm.L)
        x = dev(pad_cts(cts, prm.L, prm.N))
        y = dev(np.zeros((len(cts), 2, prm.L, prm.N), np.uint64))
        flags = F.FHELIN_APPLY_RESCALE | (F.FHELIN_APPLY_HOIST_MODDOWN if dh else 0)
        F.fhelin_linear_apply_multi(ctx, plan, [handles[o] for o in owner], pset, x, levels, y,
                                    [l - 1 for l in levels], flags)
        got = host(y)
        for t, (o, l) in enumerate(zip(owner, levels)):
            want = O.rescale(prm, O.linear(prm, cts[t][None], l, sched, pts, keysets[o], hoist_moddown=dh)[0], l)
            assert np.array_equal(got[t, :, : l - 1], want), t
            z = clients[o].decrypt_slots(got[t, :, : l - 1], l - 1, prm.scale ** 2 / prm.q[l - 1]).real
            assert _rel(z[:n], W @ xs[t]) < 1e-3, t
        F.fhelin_ptset_release(pset)
        for h in handles:
            F.fhelin_keyset_release(h)
        F.fhelin_plan_destroy(plan)
    finally:
        F.fhelin_ctx_destroy(ctx)


def test_errors_reported(F):
    """Invalid calls are rejected on the host with their status before any kernel
    runs: a key set missing a Galois element, keys loaded below the request level,
    plaintexts encoded below it, rescale at level 1, mismatched output counts or
    levels, and an out-of-range tune."""
    print("error paths", flush=True)
    prm = O.make_params(12, 4, 2, 2, 50, 2.0 ** 40)
    st = synth.Stream(4900)
    n, n1 = 32, 8
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(st.he_normal((n, n), n), n, n1, prm.S), 3, prm.scale)
    cl = Client(prm, 4901)
    keys = cl.keyset(sched.rotations())
    partial = O.KeySet(keys.galois[:-1], keys.evk[:-1])
    ctx = ctx_for(F, prm)
    try:
        plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=n, fc_out=n, fc_in=n, n1=n1)
        ks_full = F.fhelin_keyset_load(ctx, keys.galois, prm.L, dev(keys_at(prm, keys, prm.L)))
        ks_low = F.fhelin_keyset_load(ctx, keys.galois, 2, dev(keys_at(prm, keys, 2)))
        ks_part = F.fhelin_keyset_load(ctx, partial.galois, prm.L, dev(keys_at(prm, partial, prm.L)))
        pset = F.fhelin_pt_import(ctx, dev(pts.reshape(-1, 3 + prm.K, prm.N)), level=3)
        ct = lambda l: dev(pad_cts([cl.encrypt_slots(O.fc_input_slots(st.uniform(n, 0, 1), n, prm.S), l,
                                                     prm.scale)], prm.L, prm.N))
        y = dev(np.zeros((1, 2, prm.L, prm.N), np.uint64))
        R = F.FHELIN_APPLY_RESCALE

        def status(fn):
            with pytest.raises(F.FhelinError) as ei:
                fn()
            return ei.value.status

        assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks_part, pset, ct(3), [3], y, [2], R)) == -4
        assert status(lambda: F.fhelin_linear_apply(ctx, plan, None, pset, ct(3), [3], y, [2], R)) == -4
        assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks_low, pset, ct(3), [3], y, [2], R)) == -3
        assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks_full, pset, ct(4), [4], y, [3], R)) == -3
        assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks_full, pset, ct(1), [1], y, [0], R)) == -3
        assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks_full, pset, ct(3), [3], y, [3], R)) == -3
        y2 = dev(np.zeros((2, 2, prm.L, prm.N), np.uint64))
        assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks_full, pset, ct(3), [3], y2, [2, 2], R)) == -1
        assert status(lambda: F.fhelin_plan_set_tune(plan, chunk=0, ks_eg=0, mac_my=2)) == -1
        # a valid call still works afterwards
        F.fhelin_linear_apply(ctx, plan, ks_full, pset, ct(3), [3], y, [2], R)
        host(y)
        for h in (ks_full, ks_low, ks_part):
            F.fhelin_keyset_release(h)
        F.fhelin_ptset_release(pset)
        F.fhelin_plan_destroy(plan)
    finally:
        F.fhelin_ctx_destroy(ctx)


def test_reserved_workspace_then_apply_allocates_nothing(F):
    """fhelin_plan_reserve_workspace grows the stream's workspace to the plan's need
    for a batch, after which a layer call of that size on the stream allocates
    nothing and gives the same bits as the oracle."""
    print("reserve workspace", flush=True)
    prm = O.make_params(12, 6, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(4600)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 4601)
    keys = cl.keyset(sched.rotations())
    levels = [6, 3, 5]
    cts = [cl.encrypt_slots(O.fc_input_slots(st.uniform(n, 0, 1), n, prm.S), l, prm.scale) for l in levels]
    lay = Layer(F, prm, keys, pts, prm.L, fc_n=n, fc_out=n, fc_in=n, n1=n1)
    try:
        flags = F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN
        need = F.fhelin_plan_workspace_bytes(lay.ctx, lay.plan, len(levels), flags)
        m0 = F.fhelin_ctx_memory(lay.ctx)
        F.fhelin_plan_reserve_workspace(lay.ctx, lay.plan, len(levels), flags)
        m1 = F.fhelin_ctx_memory(lay.ctx)
        assert m1 - m0 >= need > 0
        F.fhelin_plan_reserve_workspace(lay.ctx, lay.plan, 1, flags)  # never shrinks
        assert F.fhelin_ctx_memory(lay.ctx) == m1
        got = lay.apply(cts, levels, stride=prm.L, dh=True)
        assert F.fhelin_ctx_memory(lay.ctx) == m1
        for t, l in enumerate(levels):
            want = O.rescale(prm, O.linear(prm, cts[t][None], l, sched, pts, keys, hoist_moddown=True)[0], l)
            assert np.array_equal(got[t], want), t
    finally:
        lay.close()


# ---------------------------------------------------------------------------
# the benchmark's moduli layout at a small ring: 12 + 3 primes, dnum 4 (alpha 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dh", [False, True])
def test_fc_four_digits_multi_client(F, dh):
    """N = 2^12 with the batched FC workload's modulus layout (12 q + 3 p of 50 bits,
    dnum 4, so levels 10..12 switch keys with 4 digits and 7..9 with 3), BSGS 16 x 8,
    requests of three clients at levels 12, 11, 10, 9, 8, 7, 4 and 1 in one call:
    every output bit-exact against the oracle under the same schedule, decrypting to
    the FP64 layer within 1e-3 (level 1 has no prime to rescale by and is run
    without rescale in a second call)."""
    print(f"four digits multi-client dh={dh}", flush=True)
    prm = O.make_params(12, 12, 3, 4, 50, 2.0 ** 40)
    assert prm.alpha == 3 and prm.beta(12) == 4 and prm.beta(9) == 3
    st = synth.Stream(4950 + dh)
    n, n1 = 128, 16
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    clients = [Client(prm, 4960 + i) for i in range(3)]
    keysets = [cl.keyset(sched.rotations()) for cl in clients]
    owner = [0, 1, 2, 1, 0, 2, 0]
    levels = [12, 11, 10, 9, 8, 7, 4]
    xs = [st.uniform(n, 0, 1) for _ in owner]
    cts = [clients[o].encrypt_slots(O.fc_input_slots(x, n, prm.S), l, prm.scale) for o, x, l in zip(owner, xs, levels)]
    ctx = ctx_for(F, prm)
    try:
        plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=n, fc_out=n, fc_in=n, n1=n1)
        handles = [F.fhelin_keyset_load(ctx, ks.galois, prm.L, dev(keys_at(prm, ks, prm.L))) for ks in keysets]
        pset = F.fhelin_pt_import(ctx, dev(pts.reshape(-1, prm.L + prm.K, prm.N)), level=prm.L)
        x = dev(pad_cts(cts, prm.L, prm.N))
        y = dev(np.zeros((len(cts), 2, prm.L, prm.N), np.uint64))
        hd = F.FHELIN_APPLY_HOIST_MODDOWN if dh else 0
        F.fhelin_linear_apply_multi(ctx, plan, [handles[o] for o in owner], pset, x, levels, y,
                                    [l - 1 for l in levels], F.FHELIN_APPLY_RESCALE | hd)
        got = host(y)
        for t, (o, l) in enumerate(zip(owner, levels)):
            want = O.rescale(prm, O.linear(prm, cts[t][None], l, sched, pts, keysets[o], hoist_moddown=dh)[0], l)
            assert np.array_equal(got[t, :, : l - 1], want), (t, l)
            z = clients[o].decrypt_slots(got[t, :, : l - 1], l - 1, prm.scale ** 2 / prm.q[l - 1]).real
            assert _rel(z[:n], W @ xs[t]) < 1e-3, (t, l)
        # a level-1 request (one digit, one prime) beside a level-12 one, no rescale
        x1 = st.uniform(n, 0, 1)
        c1 = clients[1].encrypt_slots(O.fc_input_slots(x1, n, prm.S), 1, prm.scale)
        x2 = dev(pad_cts([c1, cts[0]], prm.L, prm.N))
        y2 = dev(np.zeros((2, 2, prm.L, prm.N), np.uint64))
        F.fhelin_linear_apply_multi(ctx, plan, [handles[1], handles[0]], pset, x2, [1, 12], y2, [1, 12], hd)
        got2 = host(y2)
        assert np.array_equal(got2[0, :, :1], O.linear(prm, c1[None], 1, sched, pts, keysets[1], hoist_moddown=dh)[0])
        assert np.array_equal(got2[1, :, :12], O.linear(prm, cts[0][None], 12, sched, pts, keysets[0],
                                                         hoist_moddown=dh)[0])
        F.fhelin_ptset_release(pset)
        for h in handles:
            F.fhelin_keyset_release(h)
        F.fhelin_plan_destroy(plan)
    finally:
        F.fhelin_ctx_destroy(ctx)


def test_budget_and_handle_lifetimes(F):
    """A context's HBM budget (fhelin_ctx_set_budget) refuses key loads, plaintext
    imports and workspace growth that would exceed it with FHELIN_E_BUDGET and leaves
    the context usable; released or destroyed handles are rejected on a second
    release instead of being freed twice."""
    print("budget and handle lifetimes", flush=True)
    prm = O.make_params(12, 4, 2, 2, 50, 2.0 ** 40)
    st = synth.Stream(4990)
    n, n1 = 32, 8
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(st.he_normal((n, n), n), n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 4991)
    keys = cl.keyset(sched.rotations())
    ct = cl.encrypt_slots(O.fc_input_slots(st.uniform(n, 0, 1), n, prm.S), 4, prm.scale)
    ctx = ctx_for(F, prm)
    plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=n, fc_out=n, fc_in=n, n1=n1)
    evk, ptd = dev(keys_at(prm, keys, prm.L)), dev(pts.reshape(-1, prm.L + prm.K, prm.N))

    def status(fn):
        with pytest.raises(F.FhelinError) as ei:
            fn()
        return ei.value.status

    F.fhelin_ctx_set_budget(ctx, 1 << 20)
    assert status(lambda: F.fhelin_keyset_load(ctx, keys.galois, prm.L, evk)) == F.FHELIN_E_BUDGET
    assert status(lambda: F.fhelin_pt_import(ctx, ptd, level=prm.L)) == F.FHELIN_E_BUDGET
    F.fhelin_ctx_set_budget(ctx, 0)
    ks = F.fhelin_keyset_load(ctx, keys.galois, prm.L, evk)
    pset = F.fhelin_pt_import(ctx, ptd, level=prm.L)
    F.fhelin_ctx_trim(ctx)
    used = F.fhelin_ctx_memory(ctx)
    x = dev(pad_cts([ct], prm.L, prm.N))
    y = dev(np.zeros((1, 2, prm.L, prm.N), np.uint64))
    flags = F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN
    need = F.fhelin_plan_workspace_bytes(ctx, plan, 1, flags)
    F.fhelin_ctx_set_budget(ctx, used + need // 2)
    assert status(lambda: F.fhelin_linear_apply(ctx, plan, ks, pset, x, [4], y, [3], flags)) == F.FHELIN_E_BUDGET
    F.fhelin_ctx_set_budget(ctx, used + need)
    F.fhelin_linear_apply(ctx, plan, ks, pset, x, [4], y, [3], flags)
    want = O.rescale(prm, O.linear(prm, ct[None], 4, sched, pts, keys, hoist_moddown=True)[0], 4)
    assert np.array_equal(host(y)[0, :, :3], want)
    # second releases are rejected, not double frees
    F.fhelin_keyset_release(ks)
    assert status(lambda: F.fhelin_keyset_release(ks)) == F.FHELIN_E_INVALID_ARG
    F.fhelin_ptset_release(pset)
    assert status(lambda: F.fhelin_ptset_release(pset)) == F.FHELIN_E_INVALID_ARG
    F.fhelin_plan_destroy(plan)
    assert status(lambda: F.fhelin_plan_destroy(plan)) == F.FHELIN_E_INVALID_ARG
    F.fhelin_ctx_destroy(ctx)
    assert status(lambda: F.fhelin_ctx_destroy(ctx)) == F.FHELIN_E_INVALID_ARG


@pytest.mark.parametrize("dh", [False, True])
def test_ntt_tiles_bit_identical(F, dh):
    """The two-pass NTT kernels (N >= 2^13) at 128, 256 and 512 threads per workgroup
    give the oracle's ciphertexts bit for bit (N = 2^14, uneven levels), alone and in
    a batch; the autotuner's choice of the tile is one of them and leaves the layer's
    result in the output."""
    print(f"ntt tiles dh={dh}", flush=True)
    prm = O.make_params(14, 5, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(4980 + dh)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 4981)
    keys = cl.keyset(sched.rotations())
    levels = [5, 2, 4, 3]
    xs = [st.uniform(n, 0, 1) for _ in levels]
    cts = [cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), l, prm.scale) for x, l in zip(xs, levels)]
    want = [O.rescale(prm, O.linear(prm, c[None], l, sched, pts, keys, hoist_moddown=dh)[0], l)
            for c, l in zip(cts, levels)]
    lay = Layer(F, prm, keys, pts, prm.L, fc_n=n, fc_out=n, fc_in=n, n1=n1)
    try:
        for nt in (128, 256, 512):
            F.fhelin_plan_set_tune(lay.plan, chunk=0, ks_eg=16, mac_my=2, ntt_threads=nt)
            got = lay.apply(cts, levels, stride=prm.L, dh=dh)
            for t in range(len(levels)):
                assert np.array_equal(got[t], want[t]), (nt, t)
            z = cl.decrypt_slots(got[0], levels[0] - 1, prm.scale ** 2 / prm.q[levels[0] - 1]).real
            assert _rel(z[:n], W @ xs[0]) < 1e-3
        with pytest.raises(F.FhelinError):
            F.fhelin_plan_set_tune(lay.plan, chunk=0, ks_eg=16, mac_my=2, ntt_threads=64)
        x = dev(pad_cts(cts, prm.L, prm.N))
        y = dev(np.zeros((len(cts), 2, prm.L, prm.N), np.uint64))
        flags = F.FHELIN_APPLY_RESCALE | (F.FHELIN_APPLY_HOIST_MODDOWN if dh else 0)
        best, ms = F.fhelin_plan_autotune(lay.ctx, lay.plan, [lay.ks] * len(cts), lay.pset, x, levels, y,
                                          [l - 1 for l in levels], flags)
        print("autotune", best, f"{ms:.3f} ms", flush=True)
        assert best["ntt_threads"] in (128, 256, 512)
        got = host(y)
        for t, l in enumerate(levels):
            assert np.array_equal(got[t, :, : l - 1], want[t]), t
    finally:
        lay.close()


@pytest.mark.parametrize("dh", [False, True])
def test_persistent_modup_ntt_bit_exact(F, dh):
    """Each key switch's ModUp and forward NTT as one persistent launch (ticket-ordered
    tiles, bounded device-side waits): the oracle's ciphertexts bit for bit at
    N = 2^13 and 2^14 for requests of three clients at uneven levels (1 to 4 digits),
    the same bits as the separate launches, and no wait gave up."""
    print(f"persistent modup+ntt dh={dh}", flush=True)
    for log_n in (13, 14):
        prm = O.make_params(log_n, 7, 2, 4, 50, 2.0 ** 40)
        st = synth.Stream(5300 + 10 * log_n + dh)
        n, n1 = 64, 8
        W = st.he_normal((n, n), n)
        sched = O.fc_schedule(n, n1)
        pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
        clients = [Client(prm, 5310 + i) for i in range(3)]
        keysets = [cl.keyset(sched.rotations()) for cl in clients]
        owner = [0, 1, 2, 0, 1]
        levels = [7, 5, 2, 6, 3]
        xs = [st.uniform(n, 0, 1) for _ in owner]
        cts = [clients[o].encrypt_slots(O.fc_input_slots(x, n, prm.S), l, prm.scale)
               for o, x, l in zip(owner, xs, levels)]
        ctx = ctx_for(F, prm)
        try:
            plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=n, fc_out=n, fc_in=n, n1=n1)
            handles = [F.fhelin_keyset_load(ctx, ks.galois, prm.L, dev(keys_at(prm, ks, prm.L))) for ks in keysets]
            pset = F.fhelin_pt_import(ctx, dev(pts.reshape(-1, prm.L + prm.K, prm.N)), level=prm.L)
            x = dev(pad_cts(cts, prm.L, prm.N))
            flags = F.FHELIN_APPLY_RESCALE | (F.FHELIN_APPLY_HOIST_MODDOWN if dh else 0)
            outs = {}
            for pers in (1, 0):
                F.fhelin_plan_set_tune(plan, persistent=pers)
                y = dev(np.zeros((len(cts), 2, prm.L, prm.N), np.uint64))
                F.fhelin_linear_apply_multi(ctx, plan, [handles[o] for o in owner], pset, x, levels, y,
                                            [l - 1 for l in levels], flags)
                outs[pers] = host(y)
            assert F.fhelin_ctx_faults(ctx) == 0
            for t, (o, l) in enumerate(zip(owner, levels)):
                want = O.rescale(prm, O.linear(prm, cts[t][None], l, sched, pts, keysets[o], hoist_moddown=dh)[0], l)
                assert np.array_equal(outs[1][t, :, : l - 1], want), (log_n, t, l)
                assert np.array_equal(outs[0][t, :, : l - 1], want), (log_n, t, l)
            z = clients[0].decrypt_slots(outs[1][0, :, :6], 6, prm.scale ** 2 / prm.q[6]).real
            assert _rel(z[:n], W @ xs[0]) < 1e-3
            F.fhelin_ptset_release(pset)
            for h in handles:
                F.fhelin_keyset_release(h)
            F.fhelin_plan_destroy(plan)
        finally:
            F.fhelin_ctx_destroy(ctx)


def test_release_waits_for_the_sets_own_uses(F):
    """Key and plaintext sets released right after a layer call on one stream (no
    synchronisation by the caller) are freed only after that call's work: a key set of
    another client loaded at once on a second stream -- into the released block, which
    the context reuses -- does not disturb the first call's results (three rounds)."""
    import torch
    print("release waits for uses", flush=True)
    prm = O.make_params(12, 5, 2, 3, 50, 2.0 ** 40)
    st = synth.Stream(5600)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    cl = Client(prm, 5601)
    keys = cl.keyset(sched.rotations())
    other = Client(prm, 5602).keyset(sched.rotations())
    levels = [5, 4, 5, 3, 5, 2, 4, 5]
    cts = [cl.encrypt_slots(O.fc_input_slots(st.uniform(n, 0, 1), n, prm.S), l, prm.scale) for l in levels]
    want = [O.rescale(prm, O.linear(prm, c[None], l, sched, pts, keys, hoist_moddown=True)[0], l)
            for c, l in zip(cts, levels)]
    ctx = ctx_for(F, prm)
    try:
        plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=n, fc_out=n, fc_in=n, n1=n1)
        evk, evk2 = dev(keys_at(prm, keys, prm.L)), dev(keys_at(prm, other, prm.L))
        pt_dev = dev(pts.reshape(-1, prm.L + prm.K, prm.N))
        x = dev(pad_cts(cts, prm.L, prm.N))
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        flags = F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN
        for rnd in range(3):
            with torch.cuda.stream(s1):
                y = torch.zeros((len(cts), 2, prm.L, prm.N), dtype=torch.int64, device="cuda")
            ks = F.fhelin_keyset_load(ctx, keys.galois, prm.L, evk, stream=s1)
            pset = F.fhelin_pt_import(ctx, pt_dev, level=prm.L, stream=s1)
            F.fhelin_linear_apply(ctx, plan, ks, pset, x, levels, y, [l - 1 for l in levels], flags, stream=s1)
            F.fhelin_keyset_release(ks)
            F.fhelin_ptset_release(pset)
            ks2 = F.fhelin_keyset_load(ctx, other.galois, prm.L, evk2, stream=s2)
            s1.synchronize()
            s2.synchronize()
            got = host(y)
            for t, l in enumerate(levels):
                assert np.array_equal(got[t, :, : l - 1], want[t]), (rnd, t)
            F.fhelin_keyset_release(ks2)
        F.fhelin_plan_destroy(plan)
    finally:
        F.fhelin_ctx_destroy(ctx)

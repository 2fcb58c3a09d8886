"""Output noise of a server round and the DP report of paper Sec. 5 (the CKKS
analog of the paper's appendix noise histogram): the ResNet-20-block convolution
(3x3, 16 -> 16 channels on 32x32, N = 2^15, 8 + 2 primes of 50 bits, dnum 4,
scale 2^40, level 8) with a seeded channel shuffle folded into GPU-encoded
weights, four client inputs in one batch; the decrypted outputs' errors against
the FP64 layer are histogrammed, stay inside the 1e-3 band, are centred and
symmetric (a scale mixture of Gaussians across outputs), and yield eps0 (Gaussian
mechanism) and the amplified eps of the shuffled round."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import privacy, synth
from tests.gpu_util import ctx_for, dev, host, keys_at, pad_cts
from tests.helpers import Client

pytestmark = pytest.mark.gpu


def test_conv_round_noise_histogram_and_dp_report():
    import torch

    from paper_2509_01253_amd import fhelin as F
    print("noise report: c2 conv", flush=True)
    prm = O.make_params(15, 8, 2, 4, 50, 2.0 ** 40)
    level = 8
    cs = O.ConvShape(16, 16, 32, 32, 3)
    st = synth.Stream(synth.master_seed(2)).sub(31)
    W = st.sub(synth.TAG_W).he_normal((16, 16, 3, 3), 144)
    sp = st.sub(synth.TAG_PERM)
    po, pi = sp.permutation(16), sp.permutation(16)
    Wp = O.fold_permutations(W, po, pi)
    cl = Client(prm, synth.master_seed(2) + 31)
    sched = O.conv_schedule(cs, prm.S)
    keys = cl.keyset(sched.rotations())
    xs = [st.sub(synth.TAG_X).sub(i).uniform(16 * 32 * 32, 0, 1).reshape(16, 32, 32) for i in range(4)]
    cts = [cl.encrypt_slots(O.conv_input_slots(x, cs, prm.S)[0], level, prm.scale) for x in xs]
    ctx = ctx_for(F, prm)
    try:
        plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_CONV, c_in=16, c_out=16, h=32, w=32, k=3)
        ks = F.fhelin_keyset_load(ctx, keys.galois, level, dev(keys_at(prm, keys, level)))
        pts = F.fhelin_plan_encode_weights(ctx, plan, torch.from_numpy(np.ascontiguousarray(W)).cuda(),
                                           torch.from_numpy(po).cuda(), torch.from_numpy(pi).cuda(), level,
                                           prm.scale)
        y = dev(np.zeros((4, 2, level, prm.N), np.uint64))
        F.fhelin_linear_apply(ctx, plan, ks, pts, dev(pad_cts(cts, level, prm.N)), [level] * 4, y, [level - 1] * 4,
                              F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN)
        got = host(y)
        F.fhelin_ptset_release(pts)
        F.fhelin_keyset_release(ks)
        F.fhelin_plan_destroy(plan)
    finally:
        F.fhelin_ctx_destroy(ctx)
    errs, refmax = [], 0.0
    for i, x in enumerate(xs):
        dec = cl.decrypt_slots(got[i, :, : level - 1], level - 1, prm.scale ** 2 / prm.q[level - 1]).real
        out = O.conv_output_from_slots(dec[None], cs, prm.S)
        ref = O.conv_ref(Wp, x)
        errs.append((out - ref).ravel())
        refmax = max(refmax, float(np.abs(ref).max()))
    errs = np.concatenate(errs)
    rep = privacy.round_report(errs, n_shuffled=16, sensitivity=1e-3 * refmax, bound=1e-3 * refmax)
    h = rep["noise"]
    summary = {k: h[k] for k in ("n", "mean", "std", "max_abs", "skewness", "excess_kurtosis", "bound",
                                 "inside_bound")}
    summary.update(rel_std=h["std"] / refmax, eps0=rep.get("eps0"), eps=rep.get("eps"), note=rep.get("note"),
                   counts=h["counts"], edges=h["edges"])
    print("noise report " + json.dumps(summary), flush=True)
    if os.path.isdir("gpurun_out"):
        with open(os.path.join("gpurun_out", "noise_report_c2_conv.json"), "w") as f:
            json.dump(rep, f, indent=1)
    assert h["n"] == 4 * 16 * 32 * 32
    assert h["inside_bound"] == 1.0                  # every output decrypts within 1e-3
    assert 0 < h["std"] < 1e-5 * refmax                # scale 2^40: noise far below the band
    assert abs(h["mean"]) < 0.1 * h["std"]             # centred
    # symmetric; heavier-tailed than one Gaussian (measured excess kurtosis ~3): each
    # output's error is a sum of many independent rounding and key-switching terms, but
    # its variance differs between outputs (weights, zero padding at the image border),
    # so the pooled errors form a scale mixture of Gaussians
    assert abs(h["skewness"]) < 0.1 and 0.0 < h["excess_kurtosis"] < 6.0
    # 16 shuffled channels are too few for the amplification theorem at delta = 1e-6
    assert rep["eps"] is None and rep["eps0"] > 0
    # the same noise over the 256 neurons of the batched FC workload's shuffle, for a
    # sensitivity of a hundredth of the noise: inside the theorem's range, amplified
    big = privacy.round_report(errs, n_shuffled=1 << 20, sensitivity=0.01 * h["std"])
    assert big["eps"] is not None and big["eps"] < big["eps0"]

"""The serving loop on the GPU: requests of two ring degrees, several clients
with their own keys, uneven levels and a burst followed by Poisson arrivals go
through continuous batching on several streams (requests share launches, and
launches overlap on the device); every result is bit-identical to the same
request evaluated alone, matches the oracle, and decrypts to the plaintext
layer."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_01253_amd import synth
from tests.gpu_util import dev, host, keys_at, pad_cts
from tests.helpers import Client, encode_pts

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone_and_oracle():
    import torch

    from paper_2509_01253_amd import fhelin as F
    from paper_2509_01253_amd.serving import GpuExecutor, Request, Server, poisson_timeline
    print("serving mix", flush=True)
    st = synth.Stream(synth.master_seed(5))
    ex = GpuExecutor(n_streams=3)
    flags = ex.flags
    prms = {"A": O.make_params(12, 5, 2, 3, 50, 2.0 ** 40), "B": O.make_params(13, 4, 2, 2, 50, 2.0 ** 40)}
    layers = {}
    for name, prm in prms.items():
        ex.add_params(name, prm.log_n, prm.q, prm.p, prm.dnum)
    # layer "fc" on A: FC 64x64, n1 = 8; layer "conv" on B: conv 8 -> 8 on 16x16
    Wfc = st.he_normal((64, 64), 64)
    sched_fc = O.fc_schedule(64, 8)
    pts_fc = encode_pts(prms["A"], O.fc_slots(Wfc, 64, 8, prms["A"].S), prms["A"].L, prms["A"].scale)
    cs = O.ConvShape(8, 8, 16, 16, 3)
    Wcv = st.he_normal((8, 8, 3, 3), 72)
    sched_cv = O.conv_schedule(cs, prms["B"].S)
    pts_cv = encode_pts(prms["B"], O.conv_slots(Wcv, cs, prms["B"].S), prms["B"].L, prms["B"].scale)
    for lname, pname, kind, kw, pts, sched in [
            ("fc", "A", F.FHELIN_LAYER_FC, dict(fc_n=64, fc_out=64, fc_in=64, n1=8), pts_fc, sched_fc),
            ("conv", "B", F.FHELIN_LAYER_CONV, dict(c_in=8, c_out=8, h=16, w=16, k=3), pts_cv, sched_cv)]:
        prm = prms[pname]
        pset = F.fhelin_pt_import(ex.params[pname]["ctx"], dev(pts.reshape(-1, prm.L + prm.K, prm.N)), level=prm.L)
        ex.add_layer(lname, pname, kw, kind, pset)
        layers[lname] = (pname, pts, sched, pset)
    clients = {}
    for ci in range(4):
        cname = f"c{ci}"
        for pname, prm in prms.items():
            cl = Client(prm, 9000 + ci * 10 + len(pname) + prm.log_n)
            lname = "fc" if pname == "A" else "conv"
            keys = cl.keyset(layers[lname][2].rotations())
            evk = keys_at(prm, keys, prm.L)
            clients[(cname, pname)] = (cl, keys)
            ex.add_client_keys(cname, pname, (lambda g=keys.galois, e=evk, L=prm.L: (lambda s: (g, L, dev(e))))(),
                               int(evk.nbytes))
    srv = Server(ex, hbm_budget=8 << 30, streams=3, max_batch=8)
    for ci in range(4):
        srv.open_session(f"s{ci}", f"c{ci}")
    reqs, plain = [], {}
    rounds = [1, 1, 1, 1]
    # a burst of 12 requests at t = 0 (they queue behind the first launches and share
    # later ones), then 12 Poisson arrivals at 2000 req/s that come while those run
    arrivals = np.concatenate([np.zeros(12), poisson_timeline(2000.0, 12, st.sub(synth.TAG_ARRIVAL))])
    lv = st.sub(synth.TAG_LEVEL)
    for i in range(24):
        ci = i % 4
        lname = "fc" if (i // 4) % 2 == 0 else "conv"
        pname, pts, sched, _ = layers[lname]
        prm = prms[pname]
        cl, keys = clients[(f"c{ci}", pname)]
        level = int(lv.integers(1, 2, prm.L)[0])
        if lname == "fc":
            x = st.uniform(64, 0, 1)
            cts = [cl.encrypt_slots(O.fc_input_slots(x, 64, prm.S), level, prm.scale)]
        else:
            x = st.uniform(8 * 256, 0, 1).reshape(8, 16, 16)
            cts = [cl.encrypt_slots(s, level, prm.scale) for s in O.conv_input_slots(x, cs, prm.S)]
        t = dev(pad_cts(cts, prm.L, prm.N))
        reqs.append((float(arrivals[i]), Request(i, f"c{ci}", f"s{ci}", rounds[ci], lname, level, t)))
        plain[i] = (lname, pname, cts, level, x)
        rounds[ci] += 1
    # one stale request
    reqs.append((float(arrivals[-1]) + 1e-3, Request(99, "c0", "s0", 1, "fc", 2, reqs[0][1].x)))
    torch.cuda.synchronize()
    res = srv.run(reqs)
    stats = srv.stats(res)
    print(stats, flush=True)
    assert res[-1].status.startswith("stale")
    assert stats["completed"] == 24 and stats["batches"] < 24  # some requests shared a launch
    assert stats["max_inflight"] >= 2  # batches overlapped on the device (separate streams)
    for r in res[:-1]:
        assert r.status == "ok"
        lname, pname, cts, level, x = plain[r.rid]
        prm = prms[pname]
        _, pts, sched, pset = layers[lname]
        got = host(r.y)
        # alone: a direct call with this client's keys only
        cl, keys = clients[(f"c{r.rid % 4}", pname)]
        ctx = ex.params[pname]["ctx"]
        ks = F.fhelin_keyset_load(ctx, keys.galois, prm.L, dev(keys_at(prm, keys, prm.L)))
        xin = dev(pad_cts(cts, prm.L, prm.N))
        n_out = sched.n_out
        y1 = dev(np.zeros((n_out, 2, prm.L, prm.N), np.uint64))
        F.fhelin_linear_apply(ctx, ex.layers[lname]["plan"], ks, pset, xin, [level] * len(cts), y1,
                              [level - 1] * n_out, flags)
        alone = host(y1)
        F.fhelin_keyset_release(ks)
        assert np.array_equal(got[:, :, : level - 1], alone[:, :, : level - 1]), r.rid
        if r.rid < 8 and level >= 2:
            want = O.linear(prm, np.stack(cts), level, sched, pts, keys, hoist_moddown=True)
            for o in range(n_out):
                assert np.array_equal(got[o, :, : level - 1], O.rescale(prm, want[o], level)), r.rid
        if level >= 2:
            dec = np.stack([cl.decrypt_slots(got[o, :, : level - 1], level - 1, prm.scale ** 2 / prm.q[level - 1]).real
                            for o in range(n_out)])
            if lname == "fc":
                ref, out = Wfc @ x, dec[0][:64]
            else:
                ref, out = O.conv_ref(Wcv, x), O.conv_output_from_slots(dec, cs, prm.S)
            assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-3, r.rid
    ex.close()


def test_served_shuffled_rounds_fold_the_session_permutations():
    """Per-session, per-round shuffles (paper Sec. 4.4): each request's plaintexts are
    encoded on the GPU with its session's sigma_r on the outputs and sigma_{r-1}^-1 on
    the inputs (the network's last layer unshuffled).  Every served result equals the
    same request evaluated alone with the same permutations and decrypts to the
    permuted FP64 layer W'[t][u] = W[sigma_r[t]][sigma_{r-1}[u]] within 1e-3."""
    import torch

    from paper_2509_01253_amd import fhelin as F
    from paper_2509_01253_amd.serving import GpuExecutor, Request, Server, SessionShuffler
    print("serving shuffled rounds", flush=True)
    st = synth.Stream(synth.master_seed(5)).sub(77)
    prm = O.make_params(12, 5, 2, 3, 50, 2.0 ** 40)
    shuf = SessionShuffler(b"server secret for the shuffles of this test")
    ex = GpuExecutor(n_streams=2, shuffler=shuf)
    ex.add_params("A", prm.log_n, prm.q, prm.p, prm.dnum)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    Wd = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    kw = dict(fc_n=n, fc_out=n, fc_in=n, n1=n1)
    ex.add_shuffled_layer("hidden", "A", kw, F.FHELIN_LAYER_FC, Wd, n, n, prm.scale)
    ex.add_shuffled_layer("last", "A", kw, F.FHELIN_LAYER_FC, Wd, n, n, prm.scale, shuffle_out=False)
    sched = O.fc_schedule(n, n1)
    clients = {}
    for ci in range(3):
        cl = Client(prm, 9100 + ci)
        keys = cl.keyset(sched.rotations())
        evk = keys_at(prm, keys, prm.L)
        clients[ci] = (cl, keys)
        ex.add_client_keys(f"c{ci}", "A", (lambda g=keys.galois, e=evk: (lambda s: (g, prm.L, dev(e))))(),
                           int(evk.nbytes))
    srv = Server(ex, hbm_budget=8 << 30, streams=2, max_batch=8)
    reqs, plain = [], {}
    for ci in range(3):
        srv.open_session(f"s{ci}", f"c{ci}")
    rid = 0
    for rnd in range(1, 5):  # rounds 1..3 hidden, round 4 the last layer
        for ci in range(3):
            cl, keys = clients[ci]
            level = [5, 4, 3][ci]
            x = st.uniform(n, 0, 1)
            ct = cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), level, prm.scale)
            lname = "hidden" if rnd < 4 else "last"
            reqs.append((0.0, Request(rid, f"c{ci}", f"s{ci}", rnd, lname, level, dev(pad_cts([ct], prm.L, prm.N)))))
            plain[rid] = (ci, rnd, lname, ct, level, x)
            rid += 1
    torch.cuda.synchronize()
    res = srv.run(reqs)
    stats = srv.stats(res)
    print(stats, flush=True)
    assert stats["completed"] == 12 and stats["mean_batch"] > 1  # sessions shared launches
    ctx = ex.params["A"]["ctx"]
    flags = ex.flags
    seen = set()
    for r in res:
        assert r.status == "ok"
        ci, rnd, lname, ct, level, x = plain[r.rid]
        cl, keys = clients[ci]
        po = shuf.perm(f"s{ci}", rnd, n) if lname == "hidden" else None
        pi = shuf.perm(f"s{ci}", rnd - 1, n)
        assert (pi is None) == (rnd == 1)
        if po is not None:
            seen.add(tuple(po))
        got = host(r.y)
        # alone, with the same permutations and the same GPU encode
        ks = F.fhelin_keyset_load(ctx, keys.galois, prm.L, dev(keys_at(prm, keys, prm.L)))
        pts = F.fhelin_plan_encode_weights(ctx, ex.layers[lname]["plan"], Wd,
                                           None if po is None else torch.from_numpy(po).cuda(),
                                           None if pi is None else torch.from_numpy(pi).cuda(), level, prm.scale)
        y1 = dev(np.zeros((1, 2, prm.L, prm.N), np.uint64))
        F.fhelin_linear_apply(ctx, ex.layers[lname]["plan"], ks, pts, dev(pad_cts([ct], prm.L, prm.N)), [level], y1,
                              [level - 1], flags)
        alone = host(y1)
        F.fhelin_ptset_release(pts)
        F.fhelin_keyset_release(ks)
        assert np.array_equal(got[:, :, : level - 1], alone[:, :, : level - 1]), r.rid
        dec = cl.decrypt_slots(got[0, :, : level - 1], level - 1, prm.scale ** 2 / prm.q[level - 1]).real[:n]
        ref = O.fold_permutations(W, po, pi) @ x
        assert np.abs(dec - ref).max() / np.abs(ref).max() < 1e-3, r.rid
    assert len(seen) == 9  # every (session, hidden round) drew its own permutation
    ex.close()


def test_served_with_batch_size_dependent_schedules():
    """A layer registered with two schedules by batch size (per-rotation ModDown for a
    request alone, double-hoisted for batches): every served result equals the oracle's
    layer under the schedule its batch selected and decrypts to the FP64 layer; and an
    N = 2^15 convolution (12 3x3 channels, uniform keys) served in batches equals each
    request evaluated alone."""
    import torch

    from paper_2509_01253_amd import fhelin as F
    from paper_2509_01253_amd.serving import GpuExecutor, Request, Server
    print("serving two schedules", flush=True)
    st = synth.Stream(synth.master_seed(5)).sub(91)
    rot = F.FHELIN_APPLY_RESCALE
    dh = F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN
    ex = GpuExecutor(n_streams=2)
    prm = O.make_params(12, 5, 2, 3, 50, 2.0 ** 40)
    ex.add_params("A", prm.log_n, prm.q, prm.p, prm.dnum)
    n, n1 = 64, 8
    W = st.he_normal((n, n), n)
    sched = O.fc_schedule(n, n1)
    pts = encode_pts(prm, O.fc_slots(W, n, n1, prm.S), prm.L, prm.scale)
    pset = F.fhelin_pt_import(ex.params["A"]["ctx"], dev(pts.reshape(-1, prm.L + prm.K, prm.N)), level=prm.L)
    ex.add_layer("fc", "A", dict(fc_n=n, fc_out=n, fc_in=n, n1=n1), F.FHELIN_LAYER_FC, pset,
                 flags=[(1, rot), (8, dh)])
    # the N = 2^15 convolution with uniform keys and plaintexts
    pb = O.make_params(15, 6, 2, 3, 50, 2.0 ** 40)
    ex.add_params("B", pb.log_n, pb.q, pb.p, pb.dnum)
    cs = O.ConvShape(12, 12, 32, 32, 3)
    sched_b = O.conv_schedule(cs, pb.S)
    lvl_b = 4
    n_pt_b = sched_b.n_out * sched_b.n_in * sched_b.G * sched_b.B
    pts_b = np.stack([synth.uniform_limbs(st, pb.q[:lvl_b] + pb.p, pb.N) for _ in range(n_pt_b)])
    pset_b = F.fhelin_pt_import(ex.params["B"]["ctx"], dev(pts_b), level=lvl_b)
    ex.add_layer("conv", "B", dict(c_in=12, c_out=12, h=32, w=32, k=3), F.FHELIN_LAYER_CONV, pset_b)
    gal_b = F.fhelin_plan_galois(ex.layers["conv"]["plan"])
    clients = []
    for ci in range(3):
        cl = Client(prm, 9200 + ci)
        keys = cl.keyset(sched.rotations())
        evk = keys_at(prm, keys, prm.L)
        ex.add_client_keys(f"c{ci}", "A", (lambda g=keys.galois, e=evk: (lambda s: (g, prm.L, dev(e))))(),
                           int(evk.nbytes))
        kb = np.stack([np.stack([np.stack([synth.uniform_limbs(st, pb.q[:lvl_b] + pb.p, pb.N) for _ in range(2)])
                                 for _ in range(pb.beta(lvl_b))]) for _ in gal_b])
        ex.add_client_keys(f"c{ci}", "B", (lambda g=gal_b, e=kb: (lambda s: (g, lvl_b, dev(e))))(), int(kb.nbytes))
        clients.append((cl, keys, kb))
    srv = Server(ex, hbm_budget=16 << 30, streams=2, max_batch=8)
    for ci in range(3):
        srv.open_session(f"s{ci}", f"c{ci}")
    reqs, plain, rnd = [], {}, [1, 1, 1]
    # a burst (batched, double-hoisted) then spaced arrivals (alone, per-rotation), then
    # a burst of convolutions
    times = [0.0] * 6 + [0.3, 0.6, 0.9] + [1.2] * 6
    for i, tt in enumerate(times):
        ci = i % 3
        cl, keys, kb = clients[ci]
        if i < 9:
            level = [5, 4, 3][i % 3]
            x = st.uniform(n, 0, 1)
            ct = cl.encrypt_slots(O.fc_input_slots(x, n, prm.S), level, prm.scale)
            t = dev(pad_cts([ct], prm.L, prm.N))
            reqs.append((tt, Request(i, f"c{ci}", f"s{ci}", rnd[ci], "fc", level, t)))
            plain[i] = ("fc", ci, ct, level, x)
        else:
            cts = [np.stack([synth.uniform_limbs(st, pb.q[:lvl_b], pb.N) for _ in range(2)])
                   for _ in range(sched_b.n_in)]
            t = dev(pad_cts(cts, pb.L, pb.N))
            reqs.append((tt, Request(i, f"c{ci}", f"s{ci}", rnd[ci], "conv", lvl_b, t)))
            plain[i] = ("conv", ci, cts, lvl_b, None)
        rnd[ci] += 1
    torch.cuda.synchronize()
    res = srv.run(reqs)
    print(srv.stats(res), flush=True)
    sizes = {r.rid: r.batch for r in res}
    assert any(sizes[i] == 1 for i in range(6, 9)) and any(sizes[i] > 1 for i in range(6))
    for r in res:
        assert r.status == "ok", r.rid
        kind, ci, cts, level, x = plain[r.rid]
        got = host(r.y)
        if kind == "fc":
            cl, keys, _ = clients[ci]
            fl = ex.layer_flags("fc", r.batch)
            want = O.rescale(prm, O.linear(prm, cts[None], level, sched, pts, keys,
                                           hoist_moddown=bool(fl & F.FHELIN_APPLY_HOIST_MODDOWN))[0], level)
            assert np.array_equal(got[0, :, : level - 1], want), (r.rid, r.batch)
            z = cl.decrypt_slots(want, level - 1, prm.scale ** 2 / prm.q[level - 1]).real[:n]
            assert np.abs(z - W @ x).max() / np.abs(W @ x).max() < 1e-3, r.rid
        else:
            ctx = ex.params["B"]["ctx"]
            ks = F.fhelin_keyset_load(ctx, gal_b, lvl_b, dev(clients[ci][2]))
            y1 = dev(np.zeros((sched_b.n_out, 2, pb.L, pb.N), np.uint64))
            F.fhelin_linear_apply(ctx, ex.layers["conv"]["plan"], ks, pset_b, dev(pad_cts(cts, pb.L, pb.N)),
                                  [lvl_b] * len(cts), y1, [lvl_b - 1] * sched_b.n_out, ex.layer_flags("conv", 1))
            alone = host(y1)
            F.fhelin_keyset_release(ks)
            assert np.array_equal(got[:, :, : lvl_b - 1], alone[:, :, : lvl_b - 1]), r.rid
    ex.close()

"""Throughput benchmark of the encrypted linear-layer path on one MI355X.

Workload (default): a batch of 64 independent RNS-CKKS ciphertexts at
N = 2^16 with levels drawn uniformly from 4..12 (12 x 50-bit q, 3 special
primes, dnum 4), each applying a 256x256 FC layer (He-normal FP64 weights,
a seeded output and input neuron permutation folded into the plaintext
weights) with the baby-step giant-step diagonal method (32 x 8: 38 rotations
and 256 plaintext multiply-accumulates per ciphertext; --n1 16 gives 16 x 16
with 30 rotations), then one rescale.

One timed step = load the evaluation keys (coefficient domain -> NTT, resident),
encode the layer weights (diagonals, shuffle folding, FP64 embedding, RNS,
NTT), and apply the layer with rescale to the whole batch.  Inputs (key
material, weights, ciphertexts) are resident in HBM before timing.  The keys
and ciphertexts are uniform residues: RLWE samples are indistinguishable from
uniform, and bit-exactness of the kernels is covered by the test suite.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=8, help="level of the oracle's sampled request")
    ap.add_argument("--schedule", choices=["rotation", "hoisted"], default="hoisted",
                    help="per-rotation ModDown, or the double-hoisted schedule")
    ap.add_argument("--n1", type=int, default=32, help="baby steps of the 256x256 FC (power of two; 32 x 8 is the "
                                                       "fastest split measured on MI355X)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the plan on the batch before warmup (default: the plan's default tune)")
    ap.add_argument("--persistent", type=int, default=-1,
                    help="1: each key switch's ModUp and forward NTT in one persistent launch, 0: separate launches "
                         "(default: the plan's default tune)")
    ap.add_argument("--ntt-threads", type=int, default=0, help="workgroup size of the two-pass NTT kernels")
    ap.add_argument("--with-native", type=int, default=1,
                    help="1: add the paper's own pipeline (ResNet-20 linear layers at its 8-bit set, gamma 1 and 2) "
                         "to the default run's line; 0: skip")
    ap.add_argument("--native-engine", type=int, default=0,
                    help="key-switch products of the native pipeline: 0 int8 matrix cores, 1 64-bit ALU")
    ap.add_argument("--native-bits", type=int, choices=[8, 12, 16], default=8,
                    help="parameter set of --native: the paper's 8-, 12- or 16-bit precision set")
    ap.add_argument("--native", type=int, default=0,
                    help="only the paper's own pipeline at this gamma (1 or 2): one JSON line")
    ap.add_argument("--fuse-baby", type=int, default=-1,
                    help="1: baby rotations computed inside the multiply-accumulate, 0: written by their own launch "
                         "(default: the plan's default tune)")
    ap.add_argument("--no-one-at-a-time", action="store_true",
                    help="skip the extra one-request-at-a-time comparison after the timed steps")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests per arrival rate in the serving run after the timed steps (0 = no serving run)")
    ap.add_argument("--serve-rates", type=str, default="100", help="Poisson arrival rates (req/s)")
    ap.add_argument("--serve-clients", type=int, default=32)
    ap.add_argument("--serve-schedule", choices=["fastest", "hoisted", "rotation"], default="hoisted",
                    help="schedule of each served layer: one of the two for every batch (default: the "
                         "double-hoisted one, so a request's result is bit-identical however it is batched), or "
                         "'fastest': the faster of the two timed at the layer's middle level for single requests "
                         "(used for batches of 1) and for batches of 4 (used for larger batches)")
    ap.add_argument("--serve-reserve", type=int, default=64,
                    help="requests per batch the serving executor sizes every stream's workspace for at start-up "
                         "(0: grow on demand when a larger batch arrives)")
    ap.add_argument("--serve-budget-gib", type=str, default="200",
                    help="HBM budget of the serving run (GiB): key sets, plaintexts and workspaces are admitted "
                         "against it and idle clients' key sets are evicted when it is full; '+X' means the "
                         "resident layer data and reserved workspaces plus X GiB for key sets and batches")
    ap.add_argument("--serve-streams", type=str, default="2",
                    help="streams (batches in flight at once) of the continuous-batching server; a comma list "
                         "runs one server per value")
    ap.add_argument("--with-resnet18", type=int, default=1,
                    help="after the timed steps, also time the ResNet-18-shaped stack (see --resnet18) for this many "
                         "inferences per batch and report it under 'resnet18' (0 = skip)")
    ap.add_argument("--resnet18", type=int, default=0,
                    help="instead of the FC benchmark: time every linear layer of the ResNet-18-shaped stack on "
                         "64x64x3 inputs at N=2^16, level 3, for this many inferences per batch")
    ap.add_argument("--resnet18-schedule", choices=["fastest", "hoisted", "rotation"], default="fastest",
                    help="schedule of each ResNet-18 layer: the faster of the double-hoisted and the per-rotation "
                         "ModDown schedule timed on the layer's batch (default), or one of them for every layer")
    ap.add_argument("--conv-n1", type=int, default=1,
                    help="convolutions (ResNet-18 stack, serving) split their channel rotations into baby and giant "
                         "steps (1, default) or run every channel offset as a giant step (0)")
    ap.add_argument("--pmc-summary", type=str, default="",
                    help="instead of the benchmark: FETCH,WRITE,CALIB_FETCH,CALIB_WRITE rocprofv3 --pmc output "
                         "directories -> the measured-traffic file used for roofline.traffic")
    ap.add_argument("--alu-rates", action="store_true",
                    help="instead of the benchmark: issue rates of the integer ALU instructions the kernels use and "
                         "of the register-resident NTT butterfly (fhelin_diag_alu_rate)")
    ap.add_argument("--calib-copy", type=float, default=0.0,
                    help="instead of the benchmark: copy this many GiB device-to-device 3 times (traffic-counter "
                         "calibration)")
    return ap.parse_args()


WORKLOAD = dict(log_n=16, L=12, K=3, dnum=4, bits=50, scale=2.0 ** 40, fc=256, n1=32, lmin=4, lmax=12)

# Integer-ALU ceilings, from the chip's unit counts and clock and from instruction
# counts of this build: 256 CUs x 4 SIMDs x 16 lanes issue one wave64 VALU instruction
# per SIMD every 4 clocks at 2.4 GHz (39.3 T lane-instructions/s).  The instructions the
# butterfly and the multiply-accumulate product compile to (v_mad_u64_u32, v_mul_lo_u32,
# v_mul_hi_u32, 64-bit shifts, adds) all issue at that rate on MI355X (measured with
# fhelin_diag_alu_rate, `bench.py --alu-rates`; the register-resident butterfly issues
# at about 4 clocks per instruction).  Instructions per unit, from the gfx950 assembly
# of the probes (`python -m paper_2509_01253_amd.build --isa ...`):
#   lazy forward butterfly with 53-bit twiddle companions (the product's low words as
#   two chained multiply-adds with the negated modulus): 352 VALU per 16 = 22;
#   packed 28-bit product with one Montgomery reduction per 32: 725 VALU per 128 = 5.66.
ALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
BFLY_VALU_OPS = 22
PEAK_BFLY = ALU_LANE_OPS / BFLY_VALU_OPS / 1e12  # T butterflies (= modular multiplies) per second
MAC_VALU_OPS = 725 / 128
PEAK_MAC = ALU_LANE_OPS / MAC_VALU_OPS / 1e12  # T modular products per second
HBM_PEAK_GBPS = 8000.0
# roofline of each kernel class: (bound, unit of `achieved`, peak)
ROOF = {k: ("alu", "T modmul-butterflies/s", PEAK_BFLY) for k in
        ("ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols", "modup_ntt")}
ROOF["mac"] = ("alu", "T modular products/s", PEAK_MAC)
# the fused baby-rotation multiply-accumulate counts the rotations' key products with
# the plaintext products (its key products also carry a reduction every beta terms)
ROOF["rot_mac"] = ("alu", "T modular products/s", PEAK_MAC)
for _k in ("ks_inner", "ks_rot", "ks_sum", "modup", "moddown_fbc", "combine", "copy", "rescale", "mont"):
    ROOF[_k] = ("hbm", "GB/s", HBM_PEAK_GBPS)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
KERNELS = ["ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols", "mac", "ks_inner", "ks_rot", "ks_sum", "modup",
           "moddown_fbc", "combine", "rescale", "copy", "mont", "encode", "modup_ntt", "rot_mac"]


def _lib_digest() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2509_01253_amd", "libfhelin.so"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, launches: int, args):
    """HBM bytes per launch of `kernel` measured with rocprofv3 FETCH_SIZE / WRITE_SIZE on
    this workload and tune (calibrated against a copy kernel), if the stored measurement
    was taken with the library that is loaded now; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("library_sha256") != _lib_digest() or t.get("bench_args") != traffic_args(args):
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_dispatch"]


def traffic_args(args) -> dict:
    out = {"batch": args.batch, "n1": args.n1, "schedule": args.schedule, "autotune": bool(args.autotune)}
    # tune overrides, when given, change the launches the counters were taken from
    for k, unset in (("persistent", -1), ("ntt_threads", 0), ("fuse_baby", -1)):
        v = getattr(args, k, unset)
        if v != unset:
            out[k] = v
    return out


def stream_rates(a, b) -> dict:
    """Attainable streaming rates of plain library kernels over two equal device
    buffers (context for the kernels' HBM fractions): device copy (read + write),
    write-only fill, read-mostly sum; GB/s over 10 back-to-back launches each."""
    import torch
    nb = a.numel() * a.element_size()
    rates = {}
    for name, fn, nbytes in (("copy", lambda: b.copy_(a), 2 * nb), ("fill", lambda: b.fill_(3), nb),
                             ("sum", lambda: a.sum(), nb)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        rates[name + "_GBps"] = round(10 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    return rates


def pmc_summary(dirs: str, args) -> None:
    """Write the traffic file from four rocprofv3 --pmc output directories: FETCH_SIZE
    and WRITE_SIZE of this benchmark run with the same workload flags, then of the
    --calib-copy 1 run (a 1 GiB device copy: the scale of each counter)."""
    import csv
    import glob
    fetch, write, cfetch, cwrite = dirs.split(",")

    def per_kernel(d):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        acc = {}
        for r in csv.DictReader(open(files[0])):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("fl::", "")
            name = name.split("<")[0]
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
        return acc

    def copy_kib(d):
        return max(per_kernel(d)["__amd_rocclr_copyBuffer"])

    gib = 1 << 20  # KiB in 1 GiB: the calibration copy moves 1 GiB each way
    f_scale, w_scale = gib / copy_kib(cfetch), gib / copy_kib(cwrite)
    fk, wk = per_kernel(fetch), per_kernel(write)
    # kernel -> the library's profiling class (several kernels may share one class)
    names = {"k_mac": "mac", "k_rot_mac": "rot_mac", "k_ks_inner": "ks_inner", "k_ks_rot": "ks_rot", "k_ks_sum": "ks_sum",
             "k_ntt_fwd_rows": "ntt_fwd_rows", "k_ntt_fwd_cols": "ntt_fwd_cols", "k_ntt_inv_rows": "ntt_inv_rows",
             "k_ntt_inv_cols": "ntt_inv_cols", "k_modup": "modup", "k_modup_ntt": "modup_ntt",
             "k_moddown_fbc": "moddown_fbc", "k_moddown_coef": "moddown_fbc", "k_moddown_combine": "combine",
             "k_copy_rows": "copy", "k_ext_lift_add": "copy", "k_rescale": "rescale", "k_to_mont": "mont"}
    out = {"library_sha256": _lib_digest(), "bench_args": traffic_args(args), "fetch_scale": f_scale,
           "write_scale": w_scale, "kernels": {}}
    acc = {}
    for raw, cls in names.items():
        if raw in fk and raw in wk:
            a = acc.setdefault(cls, [0, 0.0, 0.0])
            a[0] += len(fk[raw])
            a[1] += sum(fk[raw]) * 1024 * f_scale
            a[2] += sum(wk[raw]) * 1024 * w_scale
    for cls, (n, fb, wb) in acc.items():
        out["kernels"][cls] = {"dispatches": n, "fetch_bytes_per_dispatch": fb / n, "write_bytes_per_dispatch": wb / n,
                               "bytes_per_dispatch": (fb + wb) / n}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: round(v["bytes_per_dispatch"] / 2**30, 3) for k, v in out["kernels"].items()}))


def algo_bytes(level: int, n_baby: int, n_giant: int, n_mac: int, K: int, alpha: int, N: int) -> int:
    """Algorithmic HBM bytes of one request at `level` under per-ciphertext accounting
    (every key and plaintext charged to each ciphertext that uses it, as the workload's
    metric is defined; not a physical rate -- a batch shares its keys and plaintexts):
    a hoisted baby rotation reads its evaluation key (2 beta (level + K) limbs) and
    writes its output (2 level limbs), the hoisted ModUp's input being shared; a giant
    rotation is a full key switch, key plus a ciphertext in and out (4 level limbs); each
    pt-ct MAC reads its plaintext (level limbs)."""
    beta = -(-level // alpha)
    key = 2 * beta * (level + K)
    limbs = n_baby * (key + 2 * level) + n_giant * (key + 4 * level) + n_mac * level
    return limbs * N * 8


def cpu_baseline(level: int, n1: int, hoisted: bool) -> dict:
    """The oracle (plain C + numpy, OpenMP over limbs) on one request of the same
    workload and schedule at a single level; layers/s = 1 / time."""
    from oracle import oracle as O
    from paper_2509_01253_amd import synth

    w = WORKLOAD
    prm = O.make_params(w["log_n"], w["L"], w["K"], w["dnum"], w["bits"], w["scale"])
    st = synth.Stream(synth.master_seed(3)).sub(99)
    sched = O.fc_schedule(w["fc"], n1)
    gal = [O.galois_of(r, prm.log_n) for r in sched.rotations()]
    evk = np.stack([np.stack([np.stack([synth.uniform_limbs(st, prm.mods, prm.N) for _ in range(2)])
                              for _ in range(prm.dnum)]) for _ in gal])
    keys = O.KeySet(gal, evk)
    pts = np.stack([synth.uniform_limbs(st, prm.q[:level] + prm.p, prm.N) for _ in range(w["fc"])])
    pts = pts.reshape(1, 1, sched.G, sched.B, level + prm.K, prm.N)
    ct = np.stack([synth.uniform_limbs(st, prm.q[:level], prm.N) for _ in range(2)])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    y = O.linear(prm, ct[None], level, sched, pts, keys, hoist_moddown=hoisted)
    O.rescale(prm, y[0], level)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "layers/s", "cores": threads, "kind": "oracle",
            "sample": f"one request (FC 256x256, n1={n1}, {'double-hoisted' if hoisted else 'per-rotation'} "
                      f"schedule, 256 pt-MACs, rescale) at level {level} of the N=2^16 workload; {dt:.1f} s"}


def cpu_baseline_more() -> dict:
    """The oracle on the other workloads: the plain 64x64 FC at N=2^12 and the
    ResNet-20-block convolution at N=2^15, level 8, as whole layers (layers/s), and
    the ResNet-18-shaped stack at N=2^16, level 3, extrapolated from one key-switched
    rotation, one plaintext-ciphertext product and one rescale at level 3 times the
    stack's counts (5273 rotations, 91712 products, 21 rescales)."""
    from oracle import oracle as O
    from paper_2509_01253_amd import synth

    st = synth.Stream(synth.master_seed(3)).sub(98)

    def keys(prm, sched):
        gal = sorted({O.galois_of(r, prm.log_n) for r in sched.rotations()} - {1})
        return O.KeySet(gal, np.stack([np.stack([np.stack([synth.uniform_limbs(st, prm.mods, prm.N)
                                                           for _ in range(2)]) for _ in range(prm.dnum)])
                                       for _ in gal]))

    def layer(prm, sched, level):
        ks = keys(prm, sched)
        n_pt = sched.n_out * sched.n_in * sched.G * sched.B
        pts = np.stack([synth.uniform_limbs(st, prm.q[:level] + prm.p, prm.N) for _ in range(n_pt)])
        pts = pts.reshape(sched.n_out, sched.n_in, sched.G, sched.B, level + prm.K, prm.N)
        cts = np.stack([np.stack([synth.uniform_limbs(st, prm.q[:level], prm.N) for _ in range(2)])
                        for _ in range(sched.n_in)])
        t0 = time.perf_counter()
        ys = O.linear(prm, cts, level, sched, pts, ks)
        for y in ys:
            O.rescale(prm, y, level)
        return time.perf_counter() - t0

    out = {}
    t = layer(O.make_params(12, 3, 1, 3, 36, 2.0 ** 30), O.fc_schedule(64, 64), 3)
    out["fc64_n4096"] = {"layers_per_s": 1.0 / t, "s": t, "kind": "measured",
                         "workload": "plain 64x64 FC (63 rotations, 64 pt-MACs), N=2^12, level 3, rescale"}
    t = layer(O.make_params(15, 8, 2, 4, 50, 2.0 ** 40), O.conv_schedule(O.ConvShape(16, 16, 32, 32, 3), 1 << 14), 8)
    out["conv16_n32768"] = {"layers_per_s": 1.0 / t, "s": t, "kind": "measured",
                            "workload": "conv 3x3 16->16 @32x32 (8 + 15 rotations, 144 pt-MACs), N=2^15, level 8"}
    prm = O.make_params(16, 12, 3, 4, 50, 2.0 ** 40)
    g = O.galois_of(1, 16)
    evk = keys(prm, O.fc_schedule(2, 1)).evk[0]
    ct = np.stack([synth.uniform_limbs(st, prm.q[:3], prm.N) for _ in range(2)])
    pt = synth.uniform_limbs(st, prm.q[:3], prm.N)
    t0 = time.perf_counter()
    O.rotate(prm, ct, g, evk, 3)
    t_ks = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.mul_pt(prm, ct, pt, 3)
    t_mac = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.rescale(prm, ct, 3)
    t_rs = time.perf_counter() - t0
    stack = 5273 * t_ks + 91712 * t_mac + 21 * t_rs
    out["resnet18_stack_n65536"] = {"inferences_per_s": 1.0 / stack, "s": stack, "kind": "extrapolated",
                                    "from": {"rotation_s": t_ks, "pt_mac_s": t_mac, "rescale_s": t_rs},
                                    "workload": "21 linear layers of the ResNet-18-shaped stack at level 3: "
                                                "5273 rotations, 91712 pt-MACs, 21 rescales"}
    return out


def fastest_schedule(F, ctx, plan, pts, sched_flags, N, L, K, beta, mods, level, dev, batches=(1, 4)) -> dict:
    """The faster schedule of a layer for batches of each size in `batches`, requests at
    `level`: a key set of uniform residues is loaded, every schedule is applied once to
    warm up and then three times (HIP events, median); the key set is released
    afterwards and the context trimmed (call it before the context has reserved
    workspaces that must stay).  Returns the choice per batch size and the
    (max_batch, schedule) pairs for the executor: a batch up to the first size takes
    the first choice, and so on."""
    import torch

    g = torch.Generator(device=dev)
    g.manual_seed(12345)
    gal = F.fhelin_plan_galois(plan)
    info = F.fhelin_plan_info(plan)
    evk = torch.empty((len(gal), beta, 2, L + K, N), dtype=torch.int64, device=dev)
    for m, qm in enumerate(mods):
        evk[:, :, :, m].random_(0, qm, generator=g)
    ks = F.fhelin_keyset_load(ctx, gal, L, evk)
    trial, pairs = {}, []
    for b in batches:
        x = torch.empty((b * info["n_in"], 2, L, N), dtype=torch.int64, device=dev)
        for m in range(level):
            x[:, :, m].random_(0, mods[m], generator=g)
        y = torch.zeros((b * info["n_out"], 2, L, N), dtype=torch.int64, device=dev)
        tb = {}
        for name, fl in sched_flags.items():
            out_level = level - 1 if fl & F.FHELIN_APPLY_RESCALE else level

            def apply():
                F.fhelin_linear_apply(ctx, plan, ks, pts, x, [level] * (b * info["n_in"]), y,
                                      [out_level] * (b * info["n_out"]), fl)

            apply()
            torch.cuda.synchronize()
            times = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                apply()
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            tb[name] = round(float(np.median(times)), 3)
        trial[str(b)] = tb
        pairs.append((b, min(tb, key=tb.get)))
        del x, y
    torch.cuda.synchronize()
    F.fhelin_keyset_release(ks)
    del evk
    F.fhelin_ctx_trim(ctx)  # the trial's workspaces and blocks: not held against the serving budget
    return {"level": level, "trial_ms": trial, "by_batch": pairs}


def serve_bench(args) -> dict:
    """Serving run: Poisson arrivals mixing an N=2^15 job (ResNet-20-block conv 3x3
    16->16 on 32x32, 8 + 2 primes, levels 2..8) and an N=2^16 job (ResNet-18 stage-1
    conv 3x3 64->64 on 64x64, 8 input and 8 output ciphertexts, 12 + 3 primes, levels
    2..12), up to 32 clients with their own key sets, admitted by an HBM budget, with
    continuous batching on `--serve-streams` streams; compared with the same requests
    served one at a time on one stream."""
    import torch

    from paper_2509_01253_amd import fhelin as F
    from paper_2509_01253_amd import resnet, synth
    from paper_2509_01253_amd.serving import GpuExecutor, Request, Server, poisson_timeline

    root = synth.Stream(synth.master_seed(5))
    dev = torch.device("cuda:0")
    jobs = {
        "conv16": dict(params="N15", log_n=15, L=8, K=2, dnum=4, c=16, hw=32, lmin=2),
        "conv64": dict(params="N16", log_n=16, L=12, K=3, dnum=4, c=64, hw=64, lmin=2),
    }
    ex = GpuExecutor(n_streams=max(int(k) for k in args.serve_streams.split(",")), reserve_requests=args.serve_reserve)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(root.sub(synth.TAG_KEYS).u64(1)[0] & 0x7FFFFFFFFFFFFFFF))
    info = {}
    sched_flags = {"hoisted": F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN,
                   "rotation": F.FHELIN_APPLY_RESCALE}
    schedule = {}
    for name, j in jobs.items():
        pr = F.fhelin_primes_generate(j["log_n"], 50, j["K"] + j["L"])
        p, q = pr[: j["K"]], pr[j["K"]:]
        ex.add_params(j["params"], j["log_n"], q, p, j["dnum"])
        ctx = ex.params[j["params"]]["ctx"]
        kw = dict(c_in=j["c"], c_out=j["c"], h=j["hw"], w=j["hw"], k=3)
        if args.conv_n1:
            kw["n1"] = resnet.conv_channel_babies(resnet.LayerSpec("", "conv", j["c"], j["c"], j["hw"], j["hw"]),
                                                  1 << (j["log_n"] - 1))
        plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_CONV, **kw)
        W = torch.from_numpy(root.sub(synth.TAG_W).sub(j["c"]).he_normal((j["c"], j["c"], 3, 3), 9 * j["c"])).to(dev)
        pts = F.fhelin_plan_encode_weights(ctx, plan, W, None, None, j["L"], 2.0 ** 40)
        N, L, K = 1 << j["log_n"], j["L"], j["K"]
        beta = -(-L // -(-L // j["dnum"]))
        mods = q + p
        if args.serve_schedule == "fastest":
            schedule[name] = fastest_schedule(F, ctx, plan, pts, sched_flags, N, L, K, beta, mods,
                                              (j["lmin"] + L) // 2, dev)
            print(f"serving layer {name}: schedule {schedule[name]}", file=sys.stderr, flush=True)
        else:
            schedule[name] = {"by_batch": [(1, args.serve_schedule)]}
        F.fhelin_plan_destroy(plan)
        ex.add_layer(name, j["params"], kw, F.FHELIN_LAYER_CONV, pts,
                     flags=[(m, sched_flags[sc]) for m, sc in schedule[name]["by_batch"]])
        gal = ex.layers[name]["galois"]

        def source(stream, gal=gal, N=N, L=L, K=K, beta=beta, mods=mods):
            evk = torch.empty((len(gal), beta, 2, L + K, N), dtype=torch.int64, device=dev)
            for m, qm in enumerate(mods):
                evk[:, :, :, m].random_(0, qm, generator=gen)
            return gal, L, evk

        nbytes = len(gal) * beta * 2 * (L + K) * N * 8
        for ci in range(args.serve_clients):
            ex.add_client_keys(f"c{ci}", j["params"], source, nbytes)
        info[name] = dict(n_in=ex.layers[name]["n_in"], N=N, L=L, q=q)
    torch.cuda.synchronize()
    fixed = ex.library_bytes()  # resident plaintexts and reserved workspaces
    bg = args.serve_budget_gib.strip()
    budget = int(fixed + float(bg[1:]) * (1 << 30)) if bg.startswith("+") else int(float(bg) * (1 << 30))
    key_set_bytes = {name: ex.key_size[("c0", j["params"])] for name, j in jobs.items()}

    def make_requests(rate, seed):
        st = root.sub(synth.TAG_ARRIVAL).sub(seed)
        times = poisson_timeline(rate, args.serve_requests, st)
        lv = root.sub(synth.TAG_LEVEL).sub(seed)
        reqs, rounds = [], {}
        for i in range(args.serve_requests):
            name = "conv16" if i % 2 == 0 else "conv64"
            j, I = jobs[name], info[name]
            ci = int(st.integers(1, 0, args.serve_clients - 1)[0])
            level = int(lv.integers(1, j["lmin"], I["L"])[0])
            x = torch.empty((I["n_in"], 2, level, I["N"]), dtype=torch.int64, device=dev)
            for li in range(level):
                x[:, :, li].random_(0, I["q"][li], generator=gen)
            sess = f"s{ci}"
            rounds[sess] = rounds.get(sess, 0) + 1
            reqs.append((float(times[i]), Request(i, f"c{ci}", sess, rounds[sess], name, level, x)))
        torch.cuda.synchronize()
        return reqs

    out = {"workload": "Poisson mix of conv 16->16 @32x32 (N=2^15, levels 2..8) and conv 64->64 @64x64 "
                       "(N=2^16, 8 in / 8 out ciphertexts, levels 2..12), "
                       f"{args.serve_clients} clients with their own keys, HBM budget {budget / (1 << 30):.1f} GiB",
           "budget_bytes": budget, "fixed_bytes": fixed, "key_set_bytes": key_set_bytes,
           "schedule": schedule, "rates": {}}
    for ri, rate in enumerate(float(r) for r in args.serve_rates.split(",")):
        row = {}
        modes = [(f"continuous_s{k}" if "," in args.serve_streams else "continuous", int(k), 64)
                 for k in args.serve_streams.split(",")] + [("one_at_a_time", 1, 1)]
        for mode, streams, mb in modes:
            print(f"serving rate {rate:g} req/s, {mode}: start (budget {budget / (1 << 30):.1f} GiB, resident "
                  f"{fixed / (1 << 30):.1f} GiB)", file=sys.stderr, flush=True)
            reqs = make_requests(rate, ri)
            srv = Server(ex, hbm_budget=budget, streams=streams, max_batch=mb)
            for ci in range(args.serve_clients):
                srv.open_session(f"s{ci}", f"c{ci}")
            res = srv.run(reqs)
            st = srv.stats(res)
            row[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            print(f"serving rate {rate:g} req/s, {mode}: {row[mode]}", file=sys.stderr, flush=True)
            for k in list(srv.keys):
                ex.release_keys(srv.keys.pop(k).handle)
            del reqs, res
            torch.cuda.synchronize()
        out["rates"][str(int(rate))] = row
    ex.close()
    return out


def resnet18_bench(args) -> dict:
    """The linear layers of a ResNet-18-shaped network on 64x64x3 inputs (3x3 stride-1
    stem, four stages of widths 64..512, 1x1 downsampling convolutions, FC 512 -> 200;
    paper Sec. 4 rounds, one per layer, each layer's seeded channel shuffle and the previous
    round's unshuffle folded into its weights), each a fresh ciphertext set at level 3 of the
    N = 2^16 context (12 + 3 primes of 50 bits, dnum 4).  Per layer: weights encoded on
    the GPU and a key set for the layer's rotations loaded (untimed), the layer captured
    into a graph for a batch of `args.resnet18` inferences, and the graph replayed; the
    time is the median replay (HIP events on the replay stream).  With the default
    `--resnet18-schedule fastest` each layer is first captured and timed under both
    schedules (double-hoisted, per-rotation ModDown) and the faster one is captured again
    and timed for the result.  The stack time is the
    sum over the layers.  Keys and inputs are uniform residues (RLWE samples are
    indistinguishable from uniform, so the cost is the same)."""
    import torch

    from paper_2509_01253_amd import fhelin as F
    from paper_2509_01253_amd import resnet, synth

    w = WORKLOAD
    dev = torch.device("cuda:0")
    primes = F.fhelin_primes_generate(w["log_n"], w["bits"], w["K"] + w["L"])
    p, q = primes[: w["K"]], primes[w["K"]:]
    N, K, level, B = 1 << w["log_n"], w["K"], 3, args.resnet18
    mods = q[:level] + p
    ctx = F.fhelin_ctx_create(w["log_n"], q, p, w["dnum"])
    sched_flags = {"hoisted": F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN,
                   "rotation": F.FHELIN_APPLY_RESCALE}
    candidates = list(sched_flags) if args.resnet18_schedule == "fastest" else [args.resnet18_schedule]
    root = synth.Stream(synth.master_seed(4))
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(root.sub(synth.TAG_KEYS).u64(1)[0] & 0x7FFFFFFFFFFFFFFF))
    stream = torch.cuda.Stream()
    specs = resnet.resnet18_layers(64, 64)
    weights = resnet.init_weights(specs, root.sub(synth.TAG_W))
    perms = resnet.shuffle_perms(specs, root.sub(synth.TAG_PERM))
    rows, total = [], 0.0
    for sp in specs:
        if sp.kind == "conv":
            n1 = resnet.conv_channel_babies(sp, N // 2) if args.conv_n1 else 1
            plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_CONV, c_in=sp.c_in, c_out=sp.c_out, h=sp.h, w=sp.w, k=sp.k,
                                        n1=n1)
        else:
            plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=sp.fc_n, fc_out=sp.c_out, fc_in=sp.c_in,
                                        n1=min(16, sp.fc_n))
        info = F.fhelin_plan_info(plan)
        gal = F.fhelin_plan_galois(plan)
        Wd = torch.from_numpy(np.ascontiguousarray(weights[sp.name])).to(dev)
        po, pi = (None if v is None else torch.from_numpy(v).to(dev) for v in perms[sp.name])
        pts = F.fhelin_plan_encode_weights(ctx, plan, Wd, po, pi, level, w["scale"])
        ks = None
        if gal:
            evk = torch.empty((len(gal), 1, 2, level + K, N), dtype=torch.int64, device=dev)
            for m, qm in enumerate(mods):
                evk[:, :, :, m].random_(0, qm, generator=gen)
            ks = F.fhelin_keyset_load(ctx, gal, level, evk)
            del evk
        x = torch.empty((B * info["n_in"], 2, level, N), dtype=torch.int64, device=dev)
        for m in range(level):
            x[:, :, m].random_(0, q[m], generator=gen)
        y = torch.zeros((B * info["n_out"], 2, level, N), dtype=torch.int64, device=dev)
        torch.cuda.synchronize()

        def capture(fl):
            with torch.cuda.stream(stream):
                return F.fhelin_graph_capture_linear(ctx, plan, ks, pts, x, [level] * (B * info["n_in"]), y,
                                                     [level - 1] * (B * info["n_out"]), fl, stream=stream)

        def replay_ms(g):
            F.fhelin_graph_launch(g, stream=stream)  # warm-up replay
            times = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                F.fhelin_graph_launch(g, stream=stream)
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            return float(np.median(times))

        # the layer's schedule: the given one, or the faster of the two on this batch (both
        # are exact functions of their inputs; they round differently)
        trial = {}
        for name in candidates:
            g = capture(sched_flags[name])
            trial[name] = replay_ms(g)
            torch.cuda.synchronize()
            F.fhelin_graph_destroy(g)
        chosen = min(trial, key=trial.get)
        graph = capture(sched_flags[chosen])
        ms = replay_ms(graph)
        total += ms
        rot = F.fhelin_plan_rotations(plan)
        row = {"layer": sp.name, "ms": round(ms, 3), "schedule": chosen, "n_in": info["n_in"],
               "n_out": info["n_out"], "baby": len(rot[0]), "giant": len(rot[1]), "keys": len(gal),
               "pts": info["n_pt"]}
        if len(trial) > 1:
            row["trial_ms"] = {k: round(v, 3) for k, v in trial.items()}
        rows.append(row)
        print(f"resnet18 layer {row}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        F.fhelin_graph_destroy(graph)
        F.fhelin_ptset_release(pts)
        if ks is not None:
            F.fhelin_keyset_release(ks)
        F.fhelin_plan_destroy(plan)
        F.fhelin_ctx_trim(ctx)
        del x, y
    F.fhelin_ctx_destroy(ctx)
    return {"workload": "ResNet-18-shaped linear layers on 64x64x3 inputs, per-layer seeded channel shuffles "
                        "folded into the weights, N=2^16, level 3, 12+3 primes of 50 bits, "
                        f"dnum 4, schedule per layer: {args.resnet18_schedule} (double-hoisted or per-rotation "
                        "ModDown), rescale, one graph per layer",
            "inferences_per_batch": B, "stack_ms": round(total, 3),
            "inferences_per_s": round(B / (total / 1e3), 3), "layers": rows}


ALU_PROBES = {0: "v_add_u32", 1: "v_mul_lo_u32", 2: "v_mul_hi_u32", 3: "v_mad_u64_u32", 4: "v_fma_f64",
              6: "v_lshl_add_u64", 7: "v_lshrrev_b64", 5: "ntt_butterfly", 8: "mac_product",
              9: "mfma_i32_16x16x64_i8"}


# The paper's own pipeline (RLWE over Z_{2^64}[X]/Phi_M): its 8-bit parameter set
# (M = 3^7, gadget D = 2^9, l = 3, p = 2^8) with packs of phi(3^6) = 486 outputs.
NATIVE = {"t": 3, "alpha": 7, "beta": 6, "log_d": 9, "l": 3, "log_p": 8, "base": 0}
# the table's other sets (gamma in [1, 2] columns): 12 bits M = 7^4, D = 2^16, l = 2;
# 16 bits M = 5^5, D = 310, l = 4; packs of phi(t^(alpha-1)) outputs
NATIVE_SETS = {8: NATIVE,
               12: {"t": 7, "alpha": 4, "beta": 3, "log_d": 16, "l": 2, "log_p": 12, "base": 0},
               16: {"t": 5, "alpha": 5, "beta": 4, "log_d": 0, "l": 4, "log_p": 16, "base": 310}}
# 64-bit products per key-switch product in the packing GEMM's inner loop (gfx950
# assembly of k_nat_ksprod: one v_mad_u64_u32 on the key's low word, one v_mul_lo_u32 on
# its high word and half a v_add3_u32 per product: 327 VALU per 128 products)
NAT_KS_VALU_OPS = 327 / 128
PEAK_NAT_KS = ALU_LANE_OPS / NAT_KS_VALU_OPS / 1e12
# the convolution on extracted rows: 64-bit products with offset weights, two
# v_mad_u64_u32 each and the window sum (gfx950 assembly of k_nat_conv's inner loop:
# 35 VALU per 16 products)
NAT_CONV_VALU_OPS = 35 / 16
PEAK_NAT_CONV = ALU_LANE_OPS / NAT_CONV_VALU_OPS / 1e12
# the int8 matrix-core engine: each 64-bit product is 2 digit pieces (3 for gadget
# bases above 2^9) x 8 key bytes int8 multiply-adds (2 ops each), priced against
# MI355X's dense int8 peak
INT8_OPS_PER_PRODUCT = 32
PEAK_INT8_TOPS = 5000.0


def resnet20_layers() -> list:
    """The linear layers of ResNet-20 on CIFAR-10 (32x32x3): a 3x3 stem, three stages of
    three basic blocks (16, 32, 64 channels; the first convolution of stages 2 and 3
    has stride 2 and a 1x1 stride-2 projection on the skip path), FC 64 -> 10 after the
    client's average pooling: (c_in, c_out, h, w, k, stride), the FC as a 1x1
    convolution on a 1x1 input."""
    L = [(3, 16, 32, 32, 3, 1)] + [(16, 16, 32, 32, 3, 1)] * 6
    for c_in, c, h in ((16, 32, 32), (32, 64, 16)):
        L += [(c_in, c, h, h, 3, 2), (c_in, c, h, h, 1, 2)] + [(c, c, h // 2, h // 2, 3, 1)] * 5
    return L + [(64, 10, 1, 1, 1, 1)]


def native_bench(gamma: int, reps: int = 2, engine: int = 0, bits: int = 8) -> dict:
    """Server compute of one ResNet-20 inference under the paper's own pipeline at its
    `bits`-bit parameter set (8 by default) and extraction level gamma: per layer, partial trace extraction
    of the input chunks (ceil(E / N) chunks of phi(t^gamma) encrypted powers), the
    convolution on the extracted rows (4-bit weights, the round's shuffle as the output
    rows' order) and fast packing of the outputs (486 per packed ciphertext).
    Keys and input ciphertexts are uniform (RLWE samples are indistinguishable from
    uniform, so the cost is the same).  Times: HIP events on the launch stream, best of
    `reps` passes after a warm-up pass; per-kernel-class rooflines from the pipeline's own
    profiler over one more pass."""
    import torch

    from paper_2509_01253_amd import fhelin as F

    c = NATIVE_SETS[bits]
    t, alpha, beta = c["t"], c["alpha"], c["beta"]
    M = t ** alpha
    N = M - M // t
    n_pack = (t - 1) * t ** (beta - 1)
    phig = (t - 1) * t ** (gamma - 1)
    nt = F.fhelin_native_create(t, alpha, gamma, beta, c["log_d"], c["l"], c["log_p"], engine, c["base"])
    rng = np.random.default_rng(20 + gamma)
    gen = torch.Generator(device="cuda").manual_seed(20 + gamma)

    def uniform(*shape):
        return torch.randint(-2 ** 63, 2 ** 63 - 1, shape, dtype=torch.int64, device="cuda", generator=gen)

    F.fhelin_native_keys_load(nt, uniform(alpha - gamma, c["l"], 2, N))
    layers = []
    for (c_in, c_out, h, w, k, stride) in resnet20_layers():
        E = c_in * h * w
        n_out = c_out * ((h - 1) // stride + 1) * ((w - 1) // stride + 1)
        n_chunks = (E + N - 1) // N
        wts = rng.integers(-8, 8, (c_out, c_in, k, k)).astype(np.int32)
        layers.append(dict(
            shape=(c_in, c_out, h, w, k, stride), E=E, n_out=n_out, n_chunks=n_chunks,
            wts=torch.from_numpy(wts).cuda(), out_row=torch.from_numpy(rng.permutation(n_out).astype(np.int32)).cuda(),
            chunks=uniform(n_chunks, phig, 2, N), rows=torch.empty((n_chunks * N, 2, N), dtype=torch.int64, device="cuda"),
            out=torch.empty((n_out, 2, N), dtype=torch.int64, device="cuda"),
            packed=torch.empty(((n_out + n_pack - 1) // n_pack, 2, N), dtype=torch.int64, device="cuda")))

    def run_pass():
        ev = []
        for L in layers:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record()
            F.fhelin_native_extract(nt, L["chunks"], L["rows"])
            e[1].record()
            F.fhelin_native_conv(nt, *L["shape"], L["wts"], L["out_row"], L["rows"], L["out"])
            e[2].record()
            F.fhelin_native_pack(nt, L["out"], L["packed"])
            e[3].record()
            ev.append(e)
        torch.cuda.synchronize()
        return [(a.elapsed_time(b), b.elapsed_time(cc), cc.elapsed_time(d)) for a, b, cc, d in ev]

    run_pass()
    best = None
    for _ in range(reps):
        r = run_pass()
        if best is None or sum(map(sum, r)) < sum(map(sum, best)):
            best = r
    F.fhelin_native_profile_enable(nt, True)
    run_pass()
    roof = {}
    for kname, bound in (("ksprod", "alu"), ("extract", "hbm"), ("linear", "alu"), ("aut_decomp", "hbm"),
                         ("merge", "hbm"), ("leaves", "hbm")):
        n_l, ms_k, units, byts = F.fhelin_native_profile_read(nt, kname)
        if n_l == 0 or ms_k <= 0:
            continue
        if kname == "linear":
            ach, peak, unit = units / (ms_k / 1e3) / 1e12, PEAK_NAT_CONV, "T 64-bit products/s"
        elif bound == "alu" and engine == 0:
            bound = "mfma"
            pieces = 3 if (c["base"] or 1 << c["log_d"]) > 512 else 2
            ach, peak, unit = (units * INT8_OPS_PER_PRODUCT * pieces / 2 / (ms_k / 1e3) / 1e12, PEAK_INT8_TOPS,
                               "T int8 ops/s")
        elif bound == "alu":
            ach, peak, unit = units / (ms_k / 1e3) / 1e12, PEAK_NAT_KS, "T 64-bit products/s"
        else:
            ach, peak, unit = byts / (ms_k / 1e3) / 1e9, HBM_PEAK_GBPS, "GB/s"
        roof[kname] = {"bound": bound, "achieved": round(ach, 4), "peak": round(peak, 4), "unit": unit,
                       "frac": round(ach / peak, 4),
                       "hbm_frac": round(byts / (ms_k / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                       "launches": n_l, "ms_per_inference": round(ms_k, 3),
                       "avg_launch_ms": round(ms_k / n_l, 4)}
    F.fhelin_native_profile_enable(nt, False)
    F.fhelin_native_destroy(nt)
    tot = [sum(x[i] for x in best) for i in range(3)]
    packs = sum(L["packed"].shape[0] for L in layers)
    ks = packs * (t ** (beta - gamma) - 1 + (alpha - beta) * (t - 1))
    ms = sum(tot)
    dstr = str(c["base"]) if c["base"] else f"2^{c['log_d']}"
    return {"workload": f"ResNet-20 / CIFAR-10 linear layers ({len(layers)}: 21 convolutions incl. two 1x1 "
                        f"projections, FC 64->10), paper's {bits}-bit set: M = {t}^{alpha}, N = {N}, D = {dstr}, "
                        f"l = {c['l']}, p = 2^{c['log_p']}, "
                        f"gamma = {gamma}, beta = {beta} ({n_pack} outputs per packed ciphertext), 4-bit weights, "
                        f"uniform keys and inputs",
            "gamma": gamma, "engine": "int8 matrix cores" if engine == 0 else "64-bit ALU",
            "per_inference_ms": round(ms, 3), "inferences_per_s": round(1e3 / ms, 3),
            "extract_ms": round(tot[0], 3), "linear_ms": round(tot[1], 3), "pack_ms": round(tot[2], 3),
            "packed_ciphertexts": packs, "key_switches": ks, "key_switches_per_s": round(ks / (tot[2] / 1e3), 1),
            "rooflines": roof, "dominant": max(roof, key=lambda k: roof[k]["ms_per_inference"]) if roof else None}


def alu_rates(F) -> dict:
    """Clocks per wave-level instruction on one SIMD for the instructions the NTT and
    multiply-accumulate kernels are built from, and the rate of the register-resident
    lazy NTT butterfly, at 4 and 8 waves per SIMD, and of the int8 matrix-core
    product at 2 and 4 (fhelin_diag_alu_rate)."""
    out = {}
    for op, name in ALU_PROBES.items():
        iters = (1 << 14) if op in (5, 9) else (1 << 16) if op == 8 else (1 << 18)
        for wps in ((2, 4) if op == 9 else (4, 8)):
            ghz, clk, ops = F.fhelin_diag_alu_rate(op, wps, iters)
            out.setdefault(name, {})[f"waves_per_simd_{wps}"] = {
                "ghz": round(ghz, 4), "clk_per_wave_op": round(clk, 3), "lane_ops_per_s": ops}
            print(f"{name} waves/SIMD {wps}: {ghz:.3f} GHz, {clk:.3f} clk per wave-op, {ops / 1e12:.3f} T/s",
                  file=sys.stderr, flush=True)
    return {"alu_rates": out}


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: requests scale out by routing clients to GPUs, not by splitting a "
                                   "layer; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2509_01253_amd import fhelin as F
    from paper_2509_01253_amd import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.resnet18 > 0:
        print(json.dumps({"resnet18": resnet18_bench(args)}))
        return
    if args.alu_rates:
        print(json.dumps(alu_rates(F)), flush=True)
        return
    if args.native > 0:
        print(json.dumps({"native_resnet20": native_bench(args.native, engine=args.native_engine,
                                                          bits=args.native_bits)}), flush=True)
        return
    if args.calib_copy > 0:
        n = int(args.calib_copy * (1 << 30)) // 8
        a = torch.ones(n, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8, "copies": 3,
                          **stream_rates(a, b)}))
        return
    dev = torch.device("cuda:0")
    w = WORKLOAD
    primes = F.fhelin_primes_generate(w["log_n"], w["bits"], w["K"] + w["L"])
    p, q = primes[: w["K"]], primes[w["K"]:]
    N, L, K, dnum = 1 << w["log_n"], w["L"], w["K"], w["dnum"]
    alpha = -(-L // dnum)
    beta = -(-L // alpha)
    t_setup = time.perf_counter()
    ctx = F.fhelin_ctx_create(w["log_n"], q, p, dnum)
    t_ctx = time.perf_counter() - t_setup
    plan = F.fhelin_plan_create(ctx, F.FHELIN_LAYER_FC, fc_n=w["fc"], fc_out=w["fc"], fc_in=w["fc"], n1=args.n1)
    flags = F.FHELIN_APPLY_RESCALE | (F.FHELIN_APPLY_HOIST_MODDOWN if args.schedule == "hoisted" else 0)
    galois = F.fhelin_plan_galois(plan)
    info = F.fhelin_plan_info(plan)
    n_rot = sum(1 for r in F.fhelin_plan_rotations(plan)[0] if r) + sum(1 for r in F.fhelin_plan_rotations(plan)[1] if r)

    root = synth.Stream(synth.master_seed(3))
    sk = root.sub(synth.TAG_KEYS)
    mods = q + p
    # evaluation keys, coefficient domain [n_keys][beta][2][L+K][N], uniform residues
    evk = torch.empty((len(galois), beta, 2, L + K, N), dtype=torch.int64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(sk.u64(1)[0] & 0x7FFFFFFFFFFFFFFF))
    for m, qm in enumerate(mods):
        evk[:, :, :, m].random_(0, qm, generator=gen)
    sw = root.sub(synth.TAG_W)
    W = torch.from_numpy(sw.he_normal((w["fc"], w["fc"]), w["fc"])).to(dev)
    sp = root.sub(synth.TAG_PERM)
    perm_out = torch.from_numpy(sp.permutation(w["fc"])).to(dev)
    perm_in = torch.from_numpy(sp.permutation(w["fc"])).to(dev)
    levels = [int(v) for v in root.sub(synth.TAG_LEVEL).integers(args.batch, w["lmin"], w["lmax"])]
    x = torch.empty((args.batch, 2, L, N), dtype=torch.int64, device=dev)
    for i in range(L):
        x[:, :, i].random_(0, q[i], generator=gen)
    y = torch.zeros((args.batch, 2, L, N), dtype=torch.int64, device=dev)
    out_levels = [l - 1 for l in levels]
    torch.cuda.synchronize()

    def step():
        ks = F.fhelin_keyset_load(ctx, galois, L, evk)
        pts = F.fhelin_plan_encode_weights(ctx, plan, W, perm_out, perm_in, L, w["scale"])
        F.fhelin_linear_apply(ctx, plan, ks, pts, x, levels, y, out_levels, flags)
        return ks, pts

    def release(h):
        F.fhelin_ptset_release(h[1])
        F.fhelin_keyset_release(h[0])

    if args.persistent >= 0 or args.ntt_threads or args.fuse_baby >= 0:
        t = F.fhelin_plan_get_tune(plan)
        if args.persistent >= 0:
            t["persistent"] = args.persistent
        if args.fuse_baby >= 0:
            t["fuse_baby"] = args.fuse_baby
        if args.ntt_threads:
            t["ntt_threads"] = args.ntt_threads
        F.fhelin_plan_set_tune(plan, **t)
    tune_info = {"autotuned": False, "tune": F.fhelin_plan_get_tune(plan)}
    if args.autotune:
        ks, pts = step()
        best, best_ms = F.fhelin_plan_autotune(ctx, plan, [ks] * args.batch, pts, x, levels, y, out_levels, flags)
        torch.cuda.synchronize()
        release((ks, pts))
        tune_info = {"autotuned": True, "tune": best, "apply_ms_at_tune": round(best_ms, 3)}
    for _ in range(args.warmup):
        release(step())
        torch.cuda.synchronize()
    # apply-only timing (keys and weights resident), for the breakdown
    ks, pts = step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    F.fhelin_linear_apply(ctx, plan, ks, pts, x, levels, y, out_levels, flags)
    ev1.record()
    torch.cuda.synchronize()
    apply_ms = ev0.elapsed_time(ev1)
    release((ks, pts))

    torch.cuda.synchronize()
    F.fhelin_profile_enable(ctx, True)
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        h = step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - s0) * 1e3)
        release(h)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms = float(np.mean(lat))
    prof = {}
    for kname in KERNELS:
        n, kms, units, byts = F.fhelin_profile_read(ctx, kname)
        if n:
            prof[kname] = {"launches": n, "ms_per_step": round(kms / args.steps, 3), "units": units, "bytes": byts}
    F.fhelin_profile_enable(ctx, False)
    busy = sum(v["ms_per_step"] for v in prof.values())
    for v in prof.values():
        v["share"] = round(v["ms_per_step"] / busy, 4) if busy else 0.0
    rooflines = {}
    for kname, d in prof.items():
        if kname not in ROOF:
            continue
        bound, unit, peak = ROOF[kname]
        avg_s = d["ms_per_step"] * args.steps / d["launches"] / 1e3
        per_launch = (d["bytes"] if bound == "hbm" else d["units"]) / d["launches"]
        achieved = per_launch / avg_s / (1e9 if bound == "hbm" else 1e12)
        rooflines[kname] = {"bound": bound, "achieved": round(achieved, 4), "peak": round(peak, 4), "unit": unit,
                            "frac": round(achieved / peak, 4), "avg_launch_ms": round(avg_s * 1e3, 4),
                            "per_launch": per_launch,
                            "hbm_frac": round(d["bytes"] / d["launches"] / avg_s / 1e9 / HBM_PEAK_GBPS, 4)}
    dom = max(rooflines, key=lambda k: prof[k]["ms_per_step"])
    roofline = dict(rooflines[dom], kernel=dom, traffic=measured_traffic(dom, prof[dom]["launches"], args))
    layers_per_s = args.batch / (ms / 1e3)
    res = {
        "metric": "encrypted linear layers/s (N=2^16, 256x256 FC, batch of 64 at levels 4..12)",
        "value": round(layers_per_s, 3),
        "unit": "layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "batched FC 256x256, 64 RNS-CKKS ciphertexts, N=2^16, levels U{4..12}, "
                               "12+3 primes of 50 bits, dnum 4, baby-step giant-step, rescale",
                   "batch": args.batch, "levels": levels, "n1": args.n1, "n2": w["fc"] // args.n1,
                   "schedule": args.schedule},
        "ks_rotations_per_s": round(args.batch * n_rot / (ms / 1e3), 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)},
        "apply_only_ms": round(apply_ms, 3),
        "layers_per_s_apply_only": round(args.batch / (apply_ms / 1e3), 3),
        "ctx_setup_ms": round(t_ctx * 1e3, 1),
        "plan": info,
        "timed_wall_s": round(total, 3),
        "roofline": roofline,
        "rooflines": {k: {kk: v[kk] for kk in ("bound", "achieved", "unit", "frac", "hbm_frac", "avg_launch_ms")}
                      for k, v in sorted(rooflines.items(), key=lambda kv: -prof[kv[0]]["ms_per_step"])},
        "kernels": {k: {"ms_per_step": v["ms_per_step"], "share": v["share"], "launches": v["launches"]}
                    for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms_per_step"])},
    }
    res["tune"] = tune_info
    faults = F.fhelin_ctx_faults(ctx)
    if faults:
        res["device_wait_faults"] = faults
    if not args.no_one_at_a_time:
        # the same requests one at a time (keys and weights resident): the unbatched GPU path
        ks, pts = step()
        torch.cuda.synchronize()
        one_lat = []
        for r in range(args.batch):
            s0 = time.perf_counter()
            F.fhelin_linear_apply(ctx, plan, ks, pts, x[r:r + 1], levels[r:r + 1], y[r:r + 1], out_levels[r:r + 1],
                                  flags)
            torch.cuda.synchronize()
            one_lat.append((time.perf_counter() - s0) * 1e3)
        release((ks, pts))
        res["one_at_a_time"] = {
            "layers_per_s": round(args.batch / (sum(one_lat) / 1e3), 3),
            "latency_ms": {"p50": round(float(np.percentile(one_lat, 50)), 3),
                           "p99": round(float(np.percentile(one_lat, 99)), 3)},
            "batched_speedup_apply_only": round((sum(one_lat) / 1e3) / (apply_ms / 1e3), 3),
        }
    # HBM rate of the step from the library's own byte model: every launch's input and
    # output streams once, each distinct evaluation key once per launch (shared by the
    # batch), summed over the step's launches; beside it the measured traffic of the same
    # launches (rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, copy-calibrated) when the
    # stored counters were taken with the library that is loaded
    step_bytes = sum(v["bytes"] for v in prof.values()) / args.steps
    meas = {k: measured_traffic(k, v["launches"], args) for k, v in prof.items()}
    have = [k for k in prof if meas[k] is not None]
    # measured bytes of the classes the counters cover (all but the encode, whose FFT
    # kernels are not mapped to a class); null when none is covered
    meas_step = sum(meas[k] * prof[k]["launches"] for k in have) / args.steps if have else None
    res["hbm_step"] = {"model_bytes_per_step": round(step_bytes), "achieved_GBps": round(step_bytes / (ms / 1e3) / 1e9, 1),
                       "peak_GBps": HBM_PEAK_GBPS, "frac": round(step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                       "measured_bytes_per_step": None if meas_step is None else round(meas_step),
                       "measured_GBps": None if meas_step is None else round(meas_step / (ms / 1e3) / 1e9, 1),
                       "measured_classes": sorted(have)}
    # per-ciphertext accounting of the workload's metric (each request charged for the keys
    # and plaintexts it uses, although the batch reads them once): a ratio, not a rate
    rb, gk = F.fhelin_plan_rotations(plan)
    n_baby, n_giant = sum(1 for r in rb if r), sum(1 for r in gk if r)
    n_mac = info["n_pt"] // max(1, info["n_out"])
    byts = sum(algo_bytes(l, n_baby, n_giant, n_mac, K, alpha, N) for l in levels)
    res["hbm_per_ciphertext"] = {"bytes_per_step": byts, "GBps_equivalent": round(byts / (ms / 1e3) / 1e9, 1),
                                 "peak_GBps": HBM_PEAK_GBPS, "frac": round(byts / (ms / 1e3) / 8e12, 4)}
    F.fhelin_plan_destroy(plan)
    F.fhelin_ctx_destroy(ctx)
    # what a plain 1 GiB device copy attains on this GPU, measured after the timed region
    ca = torch.ones(1 << 27, dtype=torch.int64, device=dev)
    copy_gbps = stream_rates(ca, torch.empty_like(ca))["copy_GBps"]
    del ca
    res["hbm_step"]["copy_GBps"] = copy_gbps
    if args.serve_requests > 0:
        res["serving"] = serve_bench(args)
    if args.with_resnet18 > 0:
        import copy
        rargs = copy.copy(args)
        rargs.resnet18 = args.with_resnet18
        rn = resnet18_bench(rargs)
        res["resnet18"] = {k: rn[k] for k in ("workload", "inferences_per_batch", "stack_ms", "inferences_per_s")}
        res["resnet18"]["per_inference_ms"] = round(rn["stack_ms"] / rn["inferences_per_batch"], 3)
    if args.with_native:
        res["native_resnet20"] = [native_bench(g) for g in (1, 2)]
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.cpu_level, args.n1, args.schedule == "hoisted")
        res["cpu_baseline"]["other_workloads"] = cpu_baseline_more()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

"""Host logic of bench.py (no GPU): the one-GPU refusal, the rocprofv3 counter
summary and its calibration, the gating of measured traffic on the loaded library,
and the algorithmic byte model."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _args(**kw):
    a = dict(batch=64, n1=32, schedule="hoisted", autotune=False)
    a.update(kw)
    return types.SimpleNamespace(**a)


def _counter_dir(tmp_path, name, rows):
    """A rocprofv3 --pmc output directory with one counter_collection.csv."""
    d = tmp_path / name / "host" / "pid"
    d.mkdir(parents=True)
    with open(d / "123_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (kern, val) in enumerate(rows):
            f.write(f'{i},"{kern}",X,{val}\n')
    return str(tmp_path / name)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_pmc_summary_scales_by_the_copy_and_averages_dispatches(tmp_path, monkeypatch):
    gib_kib = 1 << 20
    # the copy's FETCH_SIZE reads half its bytes, WRITE_SIZE all of them
    cfetch = _counter_dir(tmp_path, "cf", [("__amd_rocclr_copyBuffer", gib_kib / 2)] * 3)
    cwrite = _counter_dir(tmp_path, "cw", [("__amd_rocclr_copyBuffer", gib_kib)] * 3)
    fetch = _counter_dir(tmp_path, "f", [("void fl::k_mac<true, 2, 2, 4>(fl::MacArgs, fl::Batch)", 100.0),
                                         ("void fl::k_mac<true, 2, 2, 4>(fl::MacArgs, fl::Batch)", 300.0),
                                         ("void fl::k_ks_rot<true, 4, 4>(fl::Batch)", 50.0)])
    write = _counter_dir(tmp_path, "w", [("void fl::k_mac<true, 2, 2, 4>(fl::MacArgs, fl::Batch)", 10.0),
                                         ("void fl::k_mac<true, 2, 2, 4>(fl::MacArgs, fl::Batch)", 30.0),
                                         ("void fl::k_ks_rot<true, 4, 4>(fl::Batch)", 500.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    monkeypatch.setattr(bench, "_lib_digest", lambda: "abc")
    bench.pmc_summary(",".join([fetch, write, cfetch, cwrite]), _args())
    t = json.loads(out.read_text())
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    mac = t["kernels"]["mac"]
    assert mac["dispatches"] == 2
    assert mac["fetch_bytes_per_dispatch"] == pytest.approx(200.0 * 1024 * 2)
    assert mac["write_bytes_per_dispatch"] == pytest.approx(20.0 * 1024)
    assert mac["bytes_per_dispatch"] == pytest.approx(200.0 * 1024 * 2 + 20.0 * 1024)
    assert t["kernels"]["ks_rot"]["bytes_per_dispatch"] == pytest.approx(50 * 1024 * 2 + 500 * 1024)
    assert t["library_sha256"] == "abc" and t["bench_args"] == bench.traffic_args(_args())


def test_measured_traffic_only_for_the_measured_library_and_workload(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"library_sha256": "abc", "bench_args": bench.traffic_args(_args()),
                             "kernels": {"mac": {"bytes_per_dispatch": 123.0}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "_lib_digest", lambda: "abc")
    assert bench.measured_traffic("mac", 1, _args()) == 123.0
    assert bench.measured_traffic("ks_rot", 1, _args()) is None
    assert bench.measured_traffic("mac", 1, _args(n1=16)) is None  # another split
    monkeypatch.setattr(bench, "_lib_digest", lambda: "changed")
    assert bench.measured_traffic("mac", 1, _args()) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("mac", 1, _args()) is None


def test_algorithmic_bytes_closed_form():
    N, K, alpha = 1 << 16, 3, 3
    # level 4: beta = 2 digits.  A hoisted baby rotation reads its key, 2 * 2 * (4 + 3)
    # limbs, and writes 2 * 4 output limbs; a giant rotation (a full key switch) reads the
    # key and moves 2 + 2 ciphertext limbs per level; a MAC reads one plaintext limb per level
    assert bench.algo_bytes(4, 1, 0, 0, K, alpha, N) == (2 * 2 * 7 + 2 * 4) * N * 8
    assert bench.algo_bytes(4, 0, 1, 0, K, alpha, N) == (2 * 2 * 7 + 4 * 4) * N * 8
    assert bench.algo_bytes(4, 0, 0, 1, K, alpha, N) == 4 * N * 8
    # level 3 needs one digit, level 4 two
    assert bench.algo_bytes(3, 0, 1, 0, K, alpha, N) == (2 * 1 * 6 + 4 * 3) * N * 8
    # linear in the counts
    assert bench.algo_bytes(12, 31, 7, 256, K, alpha, N) == \
        31 * bench.algo_bytes(12, 1, 0, 0, K, alpha, N) + 7 * bench.algo_bytes(12, 0, 1, 0, K, alpha, N) + \
        256 * bench.algo_bytes(12, 0, 0, 1, K, alpha, N)
    # the survey's per-unit figures at level 12 (beta 4): hoisted extra rotation 60 MiB of key
    # plus 12 MiB out; full key switch 84 MiB
    assert bench.algo_bytes(12, 1, 0, 0, K, alpha, N) == (60 + 12) << 20
    assert bench.algo_bytes(12, 0, 1, 0, K, alpha, N) == 84 << 20


def test_pmc_summary_merges_kernels_of_one_class(tmp_path, monkeypatch):
    """Kernels the library profiles under one class (the coefficient-domain and the
    NTT-domain ModDown conversions) are pooled: bytes per dispatch over all of them."""
    gib_kib = 1 << 20
    cfetch = _counter_dir(tmp_path, "cf", [("__amd_rocclr_copyBuffer", gib_kib)])
    cwrite = _counter_dir(tmp_path, "cw", [("__amd_rocclr_copyBuffer", gib_kib)])
    fetch = _counter_dir(tmp_path, "f", [("fl::k_moddown_coef(fl::Batch)", 10.0), ("fl::k_moddown_fbc(fl::Batch)", 30.0)])
    write = _counter_dir(tmp_path, "w", [("fl::k_moddown_coef(fl::Batch)", 1.0), ("fl::k_moddown_fbc(fl::Batch)", 3.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    monkeypatch.setattr(bench, "_lib_digest", lambda: "abc")
    bench.pmc_summary(",".join([fetch, write, cfetch, cwrite]), _args())
    k = json.loads(out.read_text())["kernels"]["moddown_fbc"]
    assert k["dispatches"] == 2
    assert k["bytes_per_dispatch"] == pytest.approx((20.0 + 2.0) * 1024)


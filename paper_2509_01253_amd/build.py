"""Build step for the HIP library ``libfhelin.so`` (gfx950).

``python -m paper_2509_01253_amd.build`` compiles every source under ``csrc/``
with hipcc into the package directory.  Runs on a machine without a GPU
(hipcc cross-compiles)."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfhelin.so")
ARCH = os.environ.get("FHELIN_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden",
    f"--offload-arch={ARCH}",
    # no packed-FP32 instructions: the kernels are integer / FP64 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def isa_loop_histogram(source: str, kernel: str) -> dict:
    """Instruction histograms of the loops of one kernel in the gfx950 assembly of a
    library source (``hipcc -S`` of this build): used to count the VALU instructions
    per butterfly / product behind the ALU rooflines.  `kernel` is a substring of the
    (mangled) symbol; the first kernel matching it is taken.  Every backward branch
    closes a loop: {header label: {mnemonic: count}} over the instructions from the
    header to that branch (nested loops included once)."""
    import re
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory() as td:
        asm = os.path.join(td, "out.s")
        cmd = [hipcc, "-O3", "-std=c++17", "-S", "--cuda-device-only", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", asm, os.path.join(CSRC, source)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc -S failed:\n" + r.stderr)
        lines = open(asm).read().splitlines()
    start = next(i for i, ln in enumerate(lines)
                 if re.match(r"^[A-Za-z_]\S*:\s*(;.*)?$", ln) and kernel in ln.split(":")[0])
    end = next(i for i in range(start, len(lines)) if lines[i].strip().startswith(".Lfunc_end"))
    body = lines[start:end]
    where = {}
    for i, ln in enumerate(body):
        m = re.match(r"^(\.LBB\w+):", ln)
        if m:
            where[m.group(1)] = i
    loops = {}
    for i, ln in enumerate(body):
        t = ln.strip().split()
        if len(t) >= 2 and t[0].startswith("s_cbranch") or (len(t) >= 2 and t[0] == "s_branch"):
            tgt = t[1]
            if tgt in where and where[tgt] < i:
                hist = {}
                for k in range(where[tgt] + 1, i + 1):
                    u = body[k].strip()
                    if not u or u.startswith(";") or u.startswith(".") or u.endswith(":"):
                        continue
                    op = u.split()[0]
                    hist[op] = hist.get(op, 0) + 1
                loops[tgt] = hist
    return {"kernel": body[0].split(":")[0], "loops": loops}


def _isa_summary(h: dict) -> dict:
    out = {"kernel": h["kernel"], "loops": {}}
    for lab, hist in h["loops"].items():
        valu = {k: v for k, v in hist.items() if k.startswith("v_")}
        out["loops"][lab] = {"valu": sum(valu.values()), "salu": sum(v for k, v in hist.items() if k.startswith("s_")),
                             "lds": sum(v for k, v in hist.items() if k.startswith("ds_")),
                             "global": sum(v for k, v in hist.items() if k.startswith(("global_", "buffer_"))),
                             "valu_ops": dict(sorted(valu.items(), key=lambda kv: -kv[1]))}
    return out


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "--isa":
        import json
        print(json.dumps(_isa_summary(isa_loop_histogram(sys.argv[2], sys.argv[3])), indent=1))
    else:
        print(build(verbose="-v" in sys.argv))

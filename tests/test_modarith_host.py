"""The library's device modular arithmetic (modarith.h) compiled for the host with
g++ and checked against 128-bit integer arithmetic: Montgomery reduction of lazy
sums of up to 32 (packed) or 16 products, restarted at a reduced value, for the packed 28-bit
accumulator (moduli below 2^55) and the 128-bit one, including operands next to q."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2509_01253_amd", "csrc")


def test_lazy_accumulators_match_int128(tmp_path):
    exe = tmp_path / "modarith_host"
    subprocess.check_call(["g++", "-O2", "-I", CSRC, "-I", "/opt/rocm/include", "-o", str(exe),
                           os.path.join(HERE, "native", "modarith_host.cpp")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "mismatches 0" in out.stdout

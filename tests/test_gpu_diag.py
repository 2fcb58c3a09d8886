"""Issue-rate probes behind the ALU and matrix-core rooflines (fhelin_diag_alu_rate):
on the GPU they return a core clock and per-instruction costs in the range the
hardware allows (a wave64 VALU instruction issues in at least 4 clocks on a 16-lane
SIMD; a 16 x 16 x 64 int8 matrix instruction in at least 16)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op,wps,iters,lo,hi", [
    (3, 4, 1 << 14, 4.0, 12.0),      # v_mad_u64_u32
    (5, 4, 1 << 12, 22 * 4.0, 22 * 8.0),  # lazy forward butterfly, 22 VALU
    (9, 2, 1 << 12, 16.0, 40.0),     # v_mfma_i32_16x16x64_i8
])
def test_issue_rate_probes(op, wps, iters, lo, hi):
    from paper_2509_01253_amd import fhelin as F
    print(f"probe op={op} waves/SIMD={wps}", flush=True)
    ghz, clk, ops = F.fhelin_diag_alu_rate(op, wps, iters)
    assert 0.5 < ghz < 3.5, ghz
    assert lo * 0.98 <= clk <= hi, clk
    assert ops > 0
    if op == 9:  # int8 operations per second: at most the chip's published dense peak
        assert 1e14 < ops < 5.2e15, ops

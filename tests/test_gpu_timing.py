"""Per-family kernel timing (mg_timing_enable / mg_timing_read), the source of
bench.py's roofline figure.

* every family that a 2D solve launches reports launches, a positive
  duration and the algorithmic bytes of those launches;
* the finest family's bytes per launch are the out-of-place kernel's (f,
  v2 and the previous iterate read; the new iterate and the next
  evaluation's restricted residual written) at the sizes where it runs;
* summed kernel time stays below the solve's wall time, and timing does not
  change the result.
"""
import time

import pytest
import torch

from paper_math_9907190_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmg():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_math_9907190_amd import dmg as D
    return D


def fused_finest_bytes(n, es=8):
    """A single FP64 problem's out-of-place step: f and the previous iterate
    read, the new one written at the interior points, the correction of the
    level below the first diagonal level read (the diagonal level's residual
    is restricted inside the kernel, not read), and the next evaluation's
    residual restricted onto that lower level written ((n/2 - 1)^2 points)"""
    inter, M = (n - 1) ** 2, n // 2
    return es * (inter + (M + 1) ** 2) + 16 * inter + es * (M - 1) ** 2


@pytest.mark.parametrize("n", [64, 512])
def test_families_report_time_and_bytes(dmg, n):
    f = torch.from_numpy(W.uniform(2, n, 21)).cuda()
    S = dmg.Solver(2, n, p=(1.052,))
    u_ref = torch.zeros_like(f)
    st, cyc_ref, rr_ref, _ = S.solve(u_ref, f, rtol=1e-10, max_cycles=40)
    assert st == dmg.MG_OK
    fams = [dmg.MG_K_RESIDUAL, dmg.MG_K_FINEST, dmg.MG_K_COARSE, dmg.MG_K_NORM]
    if n >= 512:   # at 65^2 every level below the finest runs in the coarse kernel
        fams += [dmg.MG_K_RESTRICT, dmg.MG_K_JACOBI]
    for fam in fams:
        print("n=%d family %d" % (n, fam), flush=True)
        u = torch.zeros_like(f)
        torch.cuda.synchronize()
        S.timing(fam)
        t0 = time.perf_counter()
        st, cyc, rr, _ = S.solve(u, f, rtol=1e-10, max_cycles=40)
        torch.cuda.synchronize()
        wall_ms = 1e3 * (time.perf_counter() - t0)
        ms, cnt, by = S.timing_read()
        S.timing(-1)
        assert st == dmg.MG_OK and cyc == cyc_ref and rr == rr_ref
        assert torch.equal(u, u_ref), fam
        assert cnt > 0 and ms > 0 and by > 0, (fam, ms, cnt, by)
        assert ms < wall_ms, (fam, ms, wall_ms)
        if fam == dmg.MG_K_FINEST and n >= 128:
            # one launch per cycle, plus a gated one after the last unless the
            # residual trend predicted that the last cycle was the last
            assert cnt in (cyc, cyc + 1)
            assert by == pytest.approx(cnt * fused_finest_bytes(n), rel=1e-12)
    S.close()

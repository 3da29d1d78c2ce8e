"""Batched 2D solves (one launch per aligned level for the whole batch).

* every problem's batched result is bitwise equal to its single-problem
  solve (batches run per-level launches where a single problem runs the
  fused and paired ones; the arithmetic is the same, so are the bits);
* FP64 batched solves match the CPU oracle (1e-12) with the same cycle count;
* single-precision cycles with FP64 refinement reach 1e-10 on an uneven batch;
* the hipGraph-captured iteration gives bitwise the same results as eager
  launches, over several replays with other GPU work in between;
* the autotuner keeps results within the FP64 bar and writes its cache;
* a problem that fails (NaN in f) stops alone; the others converge.
"""
import os

import numpy as np
import pytest
import torch

from paper_math_9907190_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmg():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_math_9907190_amd import dmg as D
    return D


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def relerr(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


NS = [8, 64, 16, 512, 64, 128, 2, 4, 256, 1024]


def problems(ns, seed=4):
    return [W.batch_problem(n, b, base_seed=seed) for b, n in enumerate(ns)]


def test_batched_equals_single_bitwise(dmg):
    fs = problems(NS)
    B = dmg.BatchSolver(NS, precision=dmg.MG_FP64)
    us = [dev(np.zeros_like(f)) for f in fs]
    fd = [dev(f) for f in fs]
    print("batched solve of", NS, flush=True)
    st, cyc, rr, sts = B.solve(us, fd, rtol=1e-10, max_cycles=40)
    assert st == dmg.MG_OK and all(s == dmg.MG_OK for s in sts)
    for i, (n, f) in enumerate(zip(NS, fs)):
        S = dmg.Solver(2, n, p=(1.052,))
        u1 = dev(np.zeros_like(f))
        st1, c1, r1, h1 = S.solve(u1, dev(f), rtol=1e-10, max_cycles=40)
        assert st1 == dmg.MG_OK and c1 == cyc[i]
        assert torch.equal(u1, us[i]), i
        # a single FP64 problem sums its residual norm in the finest kernel's
        # blocks: the same squares, added in another order
        assert r1 == pytest.approx(rr[i], rel=1e-12)


def test_batched_fp64_matches_oracle(dmg, orc):
    fs = problems(NS, seed=40)
    B = dmg.BatchSolver(NS, precision=dmg.MG_FP64)
    us = [dev(np.zeros_like(f)) for f in fs]
    st, cyc, rr, sts = B.solve(us, [dev(f) for f in fs], rtol=1e-10, max_cycles=40)
    for i, f in enumerate(fs):
        uo, co, ro, ho, so = orc.solve(np.zeros_like(f), f, p=(1.052,), rtol=1e-10, max_cycles=40)
        assert sts[i] == so and cyc[i] == co, i
        assert relerr(us[i].cpu().numpy(), uo) <= 1e-11, i


def test_batched_mixed_precision_uneven_sizes(dmg, orc):
    ns = W.batch_sizes(count=12, seed=4)
    fs = [W.batch_problem(n, b) for b, n in enumerate(ns)]
    B = dmg.BatchSolver(ns, precision=dmg.MG_FP32_REFINED)
    us = [dev(np.zeros_like(f)) for f in fs]
    st, cyc, rr, sts = B.solve(us, [dev(f) for f in fs], rtol=1e-10, max_cycles=40)
    assert st == dmg.MG_OK and max(rr) <= 1e-10
    for i in (0, int(np.argmax(ns))):
        f = fs[i]
        uo, co, ro, ho, so = orc.solve(np.zeros_like(f), f, p=(1.052,), rtol=1e-12, max_cycles=40)
        # both are within ~rtol of the discrete solution
        assert relerr(us[i].cpu().numpy(), uo) <= 1e-9, i


def test_graph_replays_match_eager(dmg):
    fs = problems(NS, seed=7)
    fd = [dev(f) for f in fs]
    Bg = dmg.BatchSolver(NS, precision=dmg.MG_FP64)
    os.environ["DMG_NO_GRAPH"] = "1"
    try:
        Be = dmg.BatchSolver(NS, precision=dmg.MG_FP64)
    finally:
        del os.environ["DMG_NO_GRAPH"]
    for rep in range(3):
        ug = [dev(np.zeros_like(f)) for f in fs]
        ue = [dev(np.zeros_like(f)) for f in fs]
        r1 = Bg.solve(ug, fd, rtol=1e-10, max_cycles=40)
        junk = torch.randn(1 << 20, device="cuda").sum()   # other GPU work between replays
        torch.cuda.synchronize()
        r2 = Be.solve(ue, fd, rtol=1e-10, max_cycles=40)
        assert r1[1] == r2[1] and r1[3] == r2[3], rep
        for a, b in zip(ug, ue):
            assert torch.equal(a, b), rep
        del junk


def test_autotune_and_cache(dmg, orc, tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["DMG_TUNE_CACHE"] = str(cache)
    try:
        ns = [1024, 512, 128]
        fs = problems(ns, seed=11)
        B = dmg.BatchSolver(ns, precision=dmg.MG_FP64)
        B.autotune()
        assert cache.exists() and len(cache.read_text().split()) >= 8
        us = [dev(np.zeros_like(f)) for f in fs]
        st, cyc, rr, sts = B.solve(us, [dev(f) for f in fs], rtol=1e-10, max_cycles=40)
        assert st == dmg.MG_OK
        for i, f in enumerate(fs):
            uo, co, ro, ho, so = orc.solve(np.zeros_like(f), f, p=(1.052,), rtol=1e-10, max_cycles=40)
            assert cyc[i] == co
            assert relerr(us[i].cpu().numpy(), uo) <= 1e-11, i
        B2 = dmg.BatchSolver(ns, precision=dmg.MG_FP64)   # reads the cache at setup
        us2 = [dev(np.zeros_like(f)) for f in fs]
        B2.solve(us2, [dev(f) for f in fs], rtol=1e-10, max_cycles=40)
        for a, b in zip(us, us2):
            assert torch.equal(a, b)
    finally:
        del os.environ["DMG_TUNE_CACHE"]


def test_one_failing_problem_stops_alone(dmg):
    ns = [64, 128, 64]
    fs = problems(ns, seed=13)
    fs[1] = fs[1].copy()
    fs[1][10, 10] = np.nan
    B = dmg.BatchSolver(ns, precision=dmg.MG_FP64)
    us = [dev(np.zeros_like(f)) for f in fs]
    st, cyc, rr, sts = B.solve(us, [dev(f) for f in fs], rtol=1e-10, max_cycles=40)
    assert sts == [dmg.MG_OK, dmg.MG_ERR_NONFINITE, dmg.MG_OK]
    assert st == dmg.MG_ERR_NONFINITE
    assert rr[0] <= 1e-10 and rr[2] <= 1e-10


def test_paired_levels_equal_per_level_bitwise(dmg):
    """A 2049^2 problem alone runs the Jacobi and restriction pairs at levels
    16 and 18; in a batch of two it runs every one of those levels per level.
    The solves agree to the bit."""
    ns = [2048, 64]
    fs = problems(ns, seed=17)
    B = dmg.BatchSolver(ns, precision=dmg.MG_FP64)
    us = [dev(np.zeros_like(f)) for f in fs]
    st, cyc, rr, sts = B.solve(us, [dev(f) for f in fs], rtol=1e-10, max_cycles=40)
    assert st == dmg.MG_OK
    S = dmg.Solver(2, 2048, p=(1.052,))
    u1 = dev(np.zeros_like(fs[0]))
    st1, c1, r1, h1 = S.solve(u1, dev(fs[0]), rtol=1e-10, max_cycles=40)
    assert st1 == dmg.MG_OK and c1 == cyc[0] and r1 == pytest.approx(rr[0], rel=1e-12)
    assert torch.equal(u1, us[0])

"""The per-step single-precision bound (tests/stepcheck.py), checked on the
CPU against the oracle's own single-precision cycle: every level of that cycle
is one single-precision step of its inputs, so it must meet the bound; and a
level that is off by what the bound should catch (a few hundred float ulps of
its inputs, or a wrong neighbour) must fail it."""
import numpy as np
import pytest

import stepcheck
from paper_math_9907190_amd import workloads as W

P = {2: (1.052,), 3: (1.11, 1.42, 1.08, 0.99)}


def rand_u(dim, n, seed):
    rng = np.random.default_rng(seed)
    u = np.zeros((n + 1,) * dim)
    u[(slice(1, -1),) * dim] = rng.standard_normal((n - 1,) * dim)
    return u


@pytest.mark.parametrize("dim,n,order", [(2, 2, 2), (2, 16, 2), (2, 128, 2), (2, 64, 4), (3, 2, 2), (3, 8, 2),
                                         (3, 32, 2), (3, 16, 4)])
def test_oracle_single_cycle_meets_the_step_bound(orc, dim, n, order):
    u0, f = rand_u(dim, n, 3 + n), W.uniform(dim, n, 4 + n)
    uo, rs, vs = orc.vcycle_trace(u0, f, P[dim], prec=1, order=order)
    worst = stepcheck.check_fp32_cycle(orc, dim, n, P[dim], u0, f, uo, rs, vs[1:], order=order)
    assert worst <= 1.0
    # the bound is not loose by orders of magnitude: the largest observed
    # rounding is a visible fraction of it
    assert worst > 1e-3, worst


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_step_bound_catches_small_level_errors(orc, dim, n):
    u0, f = rand_u(dim, n, 7), W.uniform(dim, n, 8)
    uo, rs, vs = orc.vcycle_trace(u0, f, P[dim], prec=1)
    D = len(rs) - 1
    c = (slice(1, 2),) * dim            # an interior point of every level with side >= 2
    for d in (1, D // 2, D):
        for which in ("r", "v"):
            rs2 = [a.copy() for a in rs]
            vs2 = [a.copy() for a in vs]
            tgt = rs2 if which == "r" else vs2
            if not np.any(tgt[d][c]):   # not a point of this level
                continue
            scale = np.abs(rs[d - 1] if which == "r" else vs[d]).max()
            tgt[d][c] += 400 * stepcheck.EPS32 * scale
            with pytest.raises(AssertionError):
                stepcheck.check_fp32_cycle(orc, dim, n, P[dim], u0, f, uo, rs2, vs2[1:])


@pytest.mark.parametrize("dim,n,order", [(2, 2, 2), (2, 64, 2), (2, 32, 4), (3, 2, 2), (3, 16, 2), (3, 8, 4)])
def test_oracle_single_usual_cycle_meets_the_step_bound(orc, dim, n, order):
    u0, f = rand_u(dim, n, 13 + n), W.uniform(dim, n, 14 + n)
    p = 1.121 if dim == 2 else 1.30
    uo, rs, vs = orc.vcycle_usual_trace(u0, f, p, prec=1, order=order)
    worst = stepcheck.check_fp32_cycle_usual(orc, dim, n, p, u0, f, uo, rs, vs[1:], order=order)
    assert worst <= 1.0
    if n > 2:
        assert worst > 1e-3, worst


def test_usual_step_bound_catches_small_level_errors(orc):
    dim, n, p = 2, 32, 1.121
    u0, f = rand_u(dim, n, 17), W.uniform(dim, n, 18)
    uo, rs, vs = orc.vcycle_usual_trace(u0, f, p, prec=1)
    for d in (1, 2, len(rs) - 1):
        for which in ("r", "v"):
            rs2 = [a.copy() for a in rs]
            vs2 = [a.copy() for a in vs]
            tgt = rs2 if which == "r" else vs2
            scale = np.abs(rs[d - 1] if which == "r" else (vs[d + 1] if d + 1 < len(vs) else rs[d])).max()
            tgt[d][1, 1] += 400 * stepcheck.EPS32 * max(scale, np.abs(tgt[d]).max())
            with pytest.raises(AssertionError):
                stepcheck.check_fp32_cycle_usual(orc, dim, n, p, u0, f, uo, rs2, vs2[1:])

"""Pins of the parameter search (Sections 2.4 and 3.4) on the oracle's cycle.

The factor is the tail of a power iteration of the error map measured on
residual norms (paper_math_9907190_amd/tune.py); run on the oracle it must
* reproduce the paper's 2D figure: about 0.052 at p = 1.052 on 65^2, with the
  Nelder-Mead optimum from p = 1 within 0.01 of the paper's 1.052;
* in 3D on 17^3 give about the paper's 0.043 at its tuned parameters, and the
  search from there must end no worse (the paper's simplex started from
  coarser-grid optima; a better point exists nearby, see below);
* come close to the spectral radius of the same cycle (2D, p = 1: 0.0954
  after 30 cycles against the 0.099 of Table tbl:2d).
"""
import json
import os

import numpy as np
import pytest

from paper_math_9907190_amd import tune

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def oracle_factor(orc, dim, n, cycles=30, tail=10, seed=0):
    from paper_math_9907190_amd import workloads as W

    def factor(p):
        if min(p) <= 0:
            return 1e3
        u = W.uniform(dim, n, seed)
        f = np.zeros_like(u)
        norms = []
        for k in range(cycles + 1):
            norms.append(orc.relres(u, f))
            if k < cycles:
                u = orc.vcycle(u, f, p)
        return tune.tail_factor(norms, tail)
    return factor


def test_2d_factor_and_optimum(orc):
    t = GOLD["tbl_2d"]
    n = t["grid_points_per_side"] - 1
    fac = oracle_factor(orc, 2, n)
    assert abs(fac((1.0,)) - t["diagonal_h2"]["rho0"]) < 0.005   # 30 cycles: 0.0954
    assert abs(fac((t["diagonal_h2"]["p"],)) - t["diagonal_h2"]["rho"]) < 0.003
    p, f, nfev = tune.nelder_mead(fac, (1.0,))
    assert abs(p[0] - t["diagonal_h2"]["p"]) < 0.01, p
    assert f <= fac((t["diagonal_h2"]["p"],)) + 1e-4
    assert nfev < 60


def test_3d_factor_and_search(orc):
    t = GOLD["tbl_3dopt"]["diagonal_h2"]
    n = GOLD["tbl_3d"]["grid_points_per_side"] - 1
    fac = oracle_factor(orc, 3, n)
    paper = (t["p_m"], t["p_r1"], t["p_r2"], t["p_g"])
    f0 = fac(paper)
    assert abs(f0 - t["rho"]) < 0.004, f0
    p, f, nfev = tune.nelder_mead(fac, paper, maxfev=150)
    assert f <= f0 + 1e-4, (p, f, f0)
    assert all(0.5 < x < 2.0 for x in p), p


def test_tail_factor():
    assert tune.tail_factor([8.0, 4.0, 2.0, 1.0], 3) == pytest.approx(0.5)
    assert tune.tail_factor([1.0, 0.1, 0.05, 0.0125], 2) == pytest.approx(0.125 ** 0.5)

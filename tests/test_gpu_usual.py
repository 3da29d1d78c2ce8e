"""Parity of the conventional comparison cycle (MG_USUAL; Sections 2.1-2.3,
3.1-3.3) on the GPU with the oracle's conventional cycle, through the C ABI.

Every level of one cycle element by element (FP64 bar: max-norm relative
1e-12); single-precision levels one step at a time within a few float ulps of
the step's inputs (tests/stepcheck.py); sizes from the single-node grid up to
several 64 x 16 (2D) and 32 x 8 x 4 (3D) tiles with partial edge tiles; ten
cycles at 65^2; solves (same cycle count, u to 1e-11); the fourth-order
residual; full-size 4097^2 and 257^3 solves from u = 0 to 1e-10.
"""
import numpy as np
import pytest
import torch

import stepcheck
from paper_math_9907190_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PU = {2: 1.121, 3: 1.30}
PU4 = {2: 1.216, 3: 1.70}


@pytest.fixture(scope="module")
def dmg():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_math_9907190_amd import dmg as D
    return D


def relerr(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def rand_u(dim, n, seed, boundary=False):
    rng = np.random.default_rng(seed)
    u = np.zeros((n + 1,) * dim)
    u[(slice(1, -1),) * dim] = rng.standard_normal((n - 1,) * dim)
    return u


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def one_cycle(dmg, orc, dim, n, prec, seed, order=2):
    p = (PU if order == 2 else PU4)[dim]
    u = rand_u(dim, n, seed)
    f = W.uniform(dim, n, seed + 1)
    uo, rs, vs = orc.vcycle_usual_trace(u, f, p, prec=prec, order=order)
    rel_o = orc.relres(u, f, order=order)
    S = dmg.Solver(dim, n, precision=prec, p=(p,), scheme="usual", order=order)
    ud, fd = to_dev(u), to_dev(f)
    print("usual cycle dim=%d n=%d prec=%d order=%d" % (dim, n, prec, order), flush=True)
    rel_g = S.vcycle(ud, fd, want_relres=True)
    torch.cuda.synchronize()
    gr = [S.level(d, 0).cpu().numpy() for d in range(S.num_levels)]
    gv = [S.level(d, 1).cpu().numpy() for d in range(1, S.num_levels)]
    ug = ud.cpu().numpy()
    S.close()
    return u, f, p, uo, rs, vs, ug, gr, gv, rel_g, rel_o


@pytest.mark.parametrize("dim,n", [(2, 2), (2, 4), (2, 8), (2, 64), (2, 128), (2, 256), (2, 1024), (3, 2), (3, 4),
                                   (3, 8), (3, 32), (3, 64), (3, 128)])
def test_every_level_of_one_usual_cycle_fp64(dmg, orc, dim, n):
    u, f, p, uo, rs, vs, ug, gr, gv, rel_g, rel_o = one_cycle(dmg, orc, dim, n, 0, 31 + n)
    assert len(gr) == len(rs)
    for d in range(len(rs)):
        assert relerr(gr[d], rs[d]) <= TOL64, ("r", d)
    for d in range(1, len(vs)):
        assert relerr(gv[d - 1], vs[d]) <= TOL64, ("v", d)
    assert relerr(ug - u, uo - u) <= TOL64
    assert abs(rel_g - rel_o) <= 1e-12 * rel_o
    edge = np.ones(u.shape, bool)
    edge[(slice(1, -1),) * dim] = False
    assert np.array_equal(ug[edge], u[edge])


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 512), (3, 8), (3, 64)])
def test_every_level_of_one_usual_cycle_fp32(dmg, orc, dim, n):
    u, f, p, uo, rs, vs, ug, gr, gv, rel_g, rel_o = one_cycle(dmg, orc, dim, n, 1, 41 + n)
    worst = stepcheck.check_fp32_cycle_usual(orc, dim, n, p, u, f, ug, gr, gv)
    print("largest step error / bound: %.3f" % worst)
    assert relerr(ug - u, uo - u) <= 1e-5


@pytest.mark.parametrize("dim,n", [(2, 64), (3, 16)])
def test_one_usual_cycle_order4(dmg, orc, dim, n):
    u, f, p, uo, rs, vs, ug, gr, gv, rel_g, rel_o = one_cycle(dmg, orc, dim, n, 0, 51 + n, order=4)
    for d in range(len(rs)):
        assert relerr(gr[d], rs[d]) <= TOL64, ("r", d)
    assert relerr(ug - u, uo - u) <= TOL64
    assert abs(rel_g - rel_o) <= 1e-12 * rel_o


def test_usual_ten_cycles_65(dmg, orc):
    n = 64
    f = W.square_uniform_plus_mode(n, seed=1)
    S = dmg.Solver(2, n, scheme="usual")
    ud, fd = to_dev(np.zeros_like(f)), to_dev(f)
    uo = np.zeros_like(f)
    for k in range(10):
        S.vcycle(ud, fd)
        uo = orc.vcycle_usual(uo, f, PU[2])
        assert relerr(ud.cpu().numpy(), uo) <= TOL64, k


@pytest.mark.parametrize("dim,n,prec", [(2, 512, 0), (2, 512, 1), (3, 64, 0), (3, 64, 1)])
def test_usual_solve_matches_oracle(dmg, orc, dim, n, prec):
    f = W.uniform(dim, n, 60 + n)
    uo, co, ro, ho, so = orc.solve_usual(np.zeros_like(f), f, PU[dim], prec=prec, rtol=1e-10, max_cycles=100)
    S = dmg.Solver(dim, n, precision=prec, scheme="usual")
    ud, fd = to_dev(np.zeros_like(f)), to_dev(f)
    print("usual solve dim=%d n=%d prec=%d" % (dim, n, prec), flush=True)
    st, cyc, rr, hist = S.solve(ud, fd, rtol=1e-10, max_cycles=100)
    ug = ud.cpu().numpy()
    assert st == so == dmg.MG_OK and rr <= 1e-10
    if prec == 0:
        assert cyc == co
        assert relerr(ug, uo) <= 1e-11
        for g, o in zip(hist, ho):
            assert abs(g - o) <= 1e-6 * o + 1e-14
    else:
        assert abs(cyc - co) <= 1
        assert relerr(ug, uo) <= 1e-8


@pytest.mark.parametrize("dim,n,make", [(2, 4096, lambda: W.square_modes_noise(4096, seed=2)),
                                        (3, 256, lambda: W.cube_uniform(256, seed=3))])
def test_full_size_usual_solve(dmg, orc, dim, n, make):
    """The comparison the benchmark times: the conventional cycle on the
    4097^2 and 257^3 workloads from u = 0 to 1e-10, FP64, against the
    oracle's conventional solve (same cycles, u to 1e-11)."""
    f = make()
    uo, co, ro, ho, so = orc.solve_usual(np.zeros_like(f), f, PU[dim], rtol=1e-10, max_cycles=100)
    S = dmg.Solver(dim, n, scheme="usual")
    ud, fd = to_dev(np.zeros_like(f)), to_dev(f)
    print("usual full-size solve dim=%d" % dim, flush=True)
    st, cyc, rr, hist = S.solve(ud, fd, rtol=1e-10, max_cycles=100)
    ug = ud.cpu().numpy()
    S.close()
    assert st == so == dmg.MG_OK and rr <= 1e-10
    assert cyc == co, (cyc, co)
    err = relerr(ug, uo)
    print("usual dim=%d: %d cycles, error vs oracle %.2e" % (dim, cyc, err))
    assert err <= 1e-11

"""Pins of the oracle's fourth-order residuals (Section 2.3 Eq. Efos2, Section
3.3 Eq. Efos4), the cycle driven by them and the two-stage solve.

* sine-mode symbol: on u = prod sin(k_i pi x_i) and f = prod sin(l_i pi x_i)
  the residual is sigma(l) f - lambda(k) u with the closed forms
  sigma = (8 + 2 c_1 + 2 c_2)/12, lambda = (-20 + 8(c_1 + c_2) + 4 c_1 c_2)/(6h^2)
  in 2D and sigma = (6 + 2 sum c_i)/12,
  lambda = (-24 + 4 sum c_i + 4 sum_{i<j} c_i c_j)/(6h^2) in 3D
  (c_i = cos(k_i pi h)); distinct asymmetric modes catch a wrong weight, sign
  or neighbour index;
* polynomial exactness: the residual of a polynomial u with f = Lap u is zero
  up to degree 5 and not at degree 6 (the schemes are fourth order, and the
  second-order residual already fails at degree 4);
* fixed point: the converged order-4 solve is the discrete sine transform
  solution u = sigma f / lambda, and on a manufactured smooth solution the
  error falls 16-fold per halving of h (4-fold at order 2);
* convergence factors: the spectral radius of the order-4 cycle on 65^2 and
  17^3 reproduces Tables tbl:2d and tbl:3d / tbl:3dopt (0.333 at p = 1, 0.200
  at p = 1.20; 0.659 with all parameters 1, 0.39 tuned);
* the two-stage solve (second-order cycles first, Sections 2.3 / 3.3) reaches
  the same fourth-order solution in fewer fourth-order cycles.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.sparse.linalg as sla

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def coords(dim, n):
    x = np.arange(n + 1) / n
    g = np.meshgrid(*([x] * dim), indexing="ij")   # g[0] varies along axis 0 = z (3D) / y (2D)
    return g[::-1]                                   # X[0] = x (fastest axis), X[1] = y, ...


def sine(dim, n, k):
    X = coords(dim, n)
    return np.prod([np.sin(k[a] * np.pi * X[a]) for a in range(dim)], axis=0)


def symbols(dim, n, k):
    h = 1.0 / n
    c = [np.cos(k[a] * np.pi * h) for a in range(dim)]
    if dim == 2:
        sig = (8 + 2 * c[0] + 2 * c[1]) / 12
        lam = (-20 + 8 * (c[0] + c[1]) + 4 * c[0] * c[1]) / (6 * h * h)
    else:
        sig = (6 + 2 * sum(c)) / 12
        lam = (-24 + 4 * sum(c) + 4 * (c[0] * c[1] + c[1] * c[2] + c[0] * c[2])) / (6 * h * h)
    return sig, lam


@pytest.mark.parametrize("dim,n,ku,kf", [(2, 16, (3, 5), (2, 7)), (2, 32, (1, 30), (17, 4)),
                                        (3, 8, (1, 2, 5), (3, 6, 1)), (3, 16, (7, 2, 13), (4, 9, 2))])
def test_residual4_sine_mode_symbol(orc, dim, n, ku, kf):
    u, f = sine(dim, n, ku), sine(dim, n, kf)
    r = orc.residual(u, f, order=4)
    sig_f, _ = symbols(dim, n, kf)
    _, lam_u = symbols(dim, n, ku)
    want = sig_f * f - lam_u * u
    inner = (slice(1, -1),) * dim
    scale = np.abs(want[inner]).max()
    assert np.abs(r[inner] - want[inner]).max() <= 1e-12 * scale
    assert not np.any(r[tuple([0] + [slice(None)] * (dim - 1))])   # boundary stays 0


def poly(dim, n, deg, seed):
    """u = random homogeneous polynomial of degree deg, f = Lap u, both on every node."""
    rng = np.random.default_rng(seed)
    X = coords(dim, n)
    X = [x + 0.3 for x in X]   # off-centre, so odd and even parts both matter
    u = np.zeros((n + 1,) * dim)
    f = np.zeros_like(u)
    for e in itertools.product(range(deg + 1), repeat=dim):
        if sum(e) != deg:
            continue
        c = rng.standard_normal()
        u += c * np.prod([X[a] ** e[a] for a in range(dim)], axis=0)
        for a in range(dim):
            if e[a] >= 2:
                ee = list(e)
                ee[a] -= 2
                f += c * e[a] * (e[a] - 1) * np.prod([X[b] ** ee[b] for b in range(dim)], axis=0)
    return u, f


@pytest.mark.parametrize("dim", [2, 3])
def test_residual4_polynomial_exactness(orc, dim):
    n = 8
    inner = (slice(1, -1),) * dim
    for deg in range(0, 7):
        u, f = poly(dim, n, deg, 10 + deg)
        r4 = orc.residual(u, f, order=4)[inner]
        r2 = orc.residual(u, f, order=2)[inner]
        tol = 1e-12 * (np.abs(u).max() * n * n + np.abs(f).max() + 1)
        if deg <= 5:
            assert np.abs(r4).max() <= tol, (deg, np.abs(r4).max())
        else:
            assert np.abs(r4).max() > 1e3 * tol, deg
        if deg <= 3:
            assert np.abs(r2).max() <= tol, (deg, np.abs(r2).max())
        elif deg == 4:
            assert np.abs(r2).max() > 1e3 * tol


def dst_solve4(f):
    dim = f.ndim
    n = f.shape[0] - 1
    inner = (slice(1, -1),) * dim
    F = sfft.dstn(f[inner], type=1)
    k = np.arange(1, n)
    grids = np.meshgrid(*([k] * dim), indexing="ij")[::-1]
    sig, lam = symbols(dim, n, grids)
    u = np.zeros_like(f)
    u[inner] = sfft.idstn(F * sig / lam, type=1)
    return u


@pytest.mark.parametrize("dim,n", [(2, 16), (2, 64), (3, 8), (3, 16)])
def test_fixed_point_is_dst_solve4(orc, dim, n):
    rng = np.random.default_rng(n + dim)
    f = np.zeros((n + 1,) * dim)
    f[(slice(1, -1),) * dim] = rng.uniform(-1, 1, (n - 1,) * dim)
    u, cyc, rr, _, st = orc.solve(np.zeros_like(f), f, orc.P2D_H4 if dim == 2 else orc.P3D_H4,
                                  rtol=1e-13, max_cycles=200, order=4)
    assert st == orc.OK and rr <= 1e-13
    want = dst_solve4(f)
    assert np.abs(u - want).max() <= 1e-11 * np.abs(want).max()


def manufactured(dim, n):
    """u* = e^x prod sin(pi x_i): zero on the boundary, Lap u* is not."""
    X = coords(dim, n)
    s = np.prod([np.sin(np.pi * X[a]) for a in range(1, dim)], axis=0)
    u = np.exp(X[0]) * np.sin(np.pi * X[0]) * s
    f = np.exp(X[0]) * s * ((1 - dim * np.pi ** 2) * np.sin(np.pi * X[0]) + 2 * np.pi * np.cos(np.pi * X[0]))
    return u, f


@pytest.mark.parametrize("dim,sizes", [(2, (16, 32, 64)), (3, (8, 16, 32))])
def test_fourth_order_convergence(orc, dim, sizes):
    errs = {2: [], 4: []}
    for n in sizes:
        ustar, f = manufactured(dim, n)
        for order in (2, 4):
            p = (orc.P2D_H4 if dim == 2 else orc.P3D_H4) if order == 4 else None
            u, _, rr, _, st = orc.solve(np.zeros_like(f), f, p, rtol=1e-13, max_cycles=300, order=order)
            assert st == orc.OK
            errs[order].append(np.abs(u - ustar).max())
    for order, lo, hi in ((2, 3.5, 4.5), (4, 13.0, 19.0)):
        ratios = [a / b for a, b in zip(errs[order], errs[order][1:])]
        assert all(lo <= q <= hi for q in ratios), (order, ratios)
    assert errs[4][-1] < 0.01 * errs[2][-1]


def spectral_radius4(orc, dim, n, p):
    N = (n - 1) ** dim
    inner = (slice(1, -1),) * dim
    f = np.zeros((n + 1,) * dim)

    def mv(x):
        u = np.zeros((n + 1,) * dim)
        u[inner] = x.reshape((n - 1,) * dim)
        return orc.vcycle(u, f, p, order=4)[inner].ravel()   # f = 0: the cycle maps the error

    op = sla.LinearOperator((N, N), matvec=mv, dtype=np.float64)
    w = sla.eigs(op, k=3, which="LM", return_eigenvectors=False, tol=1e-9,
                 v0=np.random.default_rng(0).standard_normal(N))
    return float(np.max(np.abs(w)))


def test_table_2d_order4_spectral_radius(orc):
    t = GOLD["tbl_2d"]
    n = t["grid_points_per_side"] - 1
    h4 = t["diagonal_h4"]
    assert abs(spectral_radius4(orc, 2, n, (1.0,)) - h4["rho0"]) < 0.0015
    assert abs(spectral_radius4(orc, 2, n, (h4["p"],)) - h4["rho"]) < 0.0015


def test_table_3d_order4_spectral_radius(orc):
    t0, t1 = GOLD["tbl_3d"], GOLD["tbl_3dopt"]["diagonal_h4"]
    n = t0["grid_points_per_side"] - 1
    assert abs(spectral_radius4(orc, 3, n, (1.0,) * 4) - t0["diagonal_h4"]["rho0"]) < 0.003
    tuned = (t1["p_m"], t1["p_r1"], t1["p_r2"], t1["p_g"])
    assert abs(spectral_radius4(orc, 3, n, tuned) - t1["rho"]) < 0.005


def test_order4_flop_model():
    t2, t3 = GOLD["tbl_2d"], GOLD["tbl_3d"]
    f2, f3 = GOLD["flops_2d"], GOLD["flops_3d"]
    # only the finest residual changes: 2D 25N + (12 - 7)N, 3D 35 5/7 N + 13N
    assert f2["total_N"] + f2["residual4_per_point"] - f2["residual_per_point"] == t2["diagonal_h4"]["per_iter_N"]
    assert f3["total_N"] + f3["residual4_extra_per_point"] == pytest.approx(t3["diagonal_h4"]["per_iter_N"], abs=0.05)
    for t in (t2["diagonal_h4"], t3["diagonal_h4"]):
        assert t["per_iter_N"] / -np.log10(t["rho0"]) == pytest.approx(t["per_dig0_N"], rel=0.01)
    for t in (t2["diagonal_h4"], GOLD["tbl_3dopt"]["diagonal_h4"]):
        assert t["per_iter_N"] / -np.log10(t["rho"]) == pytest.approx(t["per_dig_N"], rel=0.01)


@pytest.mark.parametrize("dim,n", [(2, 256), (3, 32)])
def test_two_stage_solve(orc, dim, n):
    """Smooth data: once the second-order cycles have converged to the
    second-order solution (O(h^2) away from the fourth-order one), fewer
    fourth-order cycles remain, and the flop total (per-cycle counts of
    Tables tbl:2d / tbl:3d) drops."""
    _, f = manufactured(dim, n)
    p4 = orc.P2D_H4 if dim == 2 else orc.P3D_H4
    u1, c1, c2, rr = orc.solve_two_stage(np.zeros_like(f), f, rtol1=1e-4, rtol=1e-10)
    assert rr <= 1e-10 and orc.relres(u1, f, order=4) == rr
    u4, cd, rd, _, st = orc.solve(np.zeros_like(f), f, p4, rtol=1e-10, order=4)
    assert st == orc.OK
    scale = np.abs(u4).max()
    assert np.abs(u1 - u4).max() <= 1e-8 * scale
    t = GOLD["tbl_2d" if dim == 2 else "tbl_3d"]
    w2, w4 = t["diagonal_h2"]["per_iter_N"], t["diagonal_h4"]["per_iter_N"]
    assert c2 < cd and w2 * c1 + w4 * c2 < w4 * cd, (c1, c2, cd)


@pytest.mark.parametrize("dim,n,ku,kf", [(2, 32, (3, 5), (2, 7)), (3, 16, (1, 2, 5), (3, 6, 1))])
def test_relres4_is_relative_to_the_rhs_combination(orc, dim, n, ku, kf):
    """The order-4 relative residual divides by ||r(0)||, the norm of the
    right-hand side combination of f, not by ||f||."""
    u, f = sine(dim, n, ku), sine(dim, n, kf)
    sig_f, _ = symbols(dim, n, kf)
    _, lam_u = symbols(dim, n, ku)
    inner = (slice(1, -1),) * dim
    want = np.linalg.norm((sig_f * f - lam_u * u)[inner]) / np.linalg.norm((sig_f * f)[inner])
    assert orc.relres(u, f, order=4) == pytest.approx(want, rel=1e-12)
    assert orc.relres(np.zeros_like(f), f, order=4) == pytest.approx(1.0, rel=1e-14)


def test_order_argument_checked(orc):
    u = np.zeros((9, 9))
    r = np.zeros_like(u)
    assert orc.lib().orc_residual_ord(2, 8, 3, orc._ptr(u), orc._ptr(u), orc._ptr(r)) == orc.ERR_ARG
    # order 2 through the order-aware entry points is the plain residual
    f = np.random.default_rng(1).uniform(-1, 1, (9, 9))
    assert np.array_equal(orc.residual(f, f, order=2), orc.residual(f, f))

"""Pins of the oracle's whole V-cycle and outer iteration.

* fixed point: the iteration converges to the discrete solution A^-1 f,
  obtained independently by a dense direct solve (tiny grids) and by the
  discrete sine transform (larger grids);
* manufactured mode: f = -d pi^2 prod sin(pi x_i) has the closed-form discrete
  solution (pi^2 h^2 / (4 sin^2(pi h/2))) prod sin(pi x_i);
* linearity of one cycle in (u, f) (the cycle is an affine map);
* invariance under the symmetries of the square (8) and of the cube (48): the
  hierarchy is symmetric because n/sigma is even on every level, so a wrongly
  permuted face stencil in the red-magenta step breaks this;
* the single-precision cycle with double residual and update (iterative
  refinement) still converges to 1e-10.
"""
import itertools

import numpy as np
import pytest
import scipy.fft as sfft


def dense_laplacian(dim, n):
    """5-/7-point Dirichlet Laplacian on the interior unknowns (x fastest)."""
    M = n - 1
    N = M ** dim
    h2 = (1.0 / n) ** 2
    A = np.zeros((N, N))
    shape = (M,) * dim
    for flat in range(N):
        idx = np.unravel_index(flat, shape)
        A[flat, flat] = -2 * dim / h2
        for ax in range(dim):
            for s in (-1, 1):
                j = list(idx)
                j[ax] += s
                if 0 <= j[ax] < M:
                    A[flat, np.ravel_multi_index(tuple(j), shape)] = 1 / h2
    return A


def dst_solve(f):
    dim = f.ndim
    n = f.shape[0] - 1
    h = 1.0 / n
    inner = (slice(1, -1),) * dim
    F = sfft.dstn(f[inner], type=1)
    s = np.sin(np.arange(1, n) * np.pi * h / 2) ** 2
    lam = 0
    for ax in range(dim):
        shp = [1] * dim
        shp[ax] = n - 1
        lam = lam + s.reshape(shp)
    lam = -(4 / h**2) * lam
    u = np.zeros_like(f)
    u[inner] = sfft.idstn(F / lam, type=1)
    return u


def rand_f(dim, n, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros((n + 1,) * dim)
    f[(slice(1, -1),) * dim] = rng.uniform(-1, 1, (n - 1,) * dim)
    return f


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 16), (3, 4), (3, 8)])
def test_fixed_point_is_dense_solve(orc, dim, n):
    f = rand_f(dim, n, 10 + n)
    A = dense_laplacian(dim, n)
    inner = (slice(1, -1),) * dim
    x = np.linalg.solve(A, f[inner].ravel())
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), f, rtol=0.0, max_cycles=25, check=False)
    assert st == orc.ERR_NOT_CONVERGED and rr < 1e-13, (cyc, rr)
    np.testing.assert_allclose(u[inner].ravel(), x, rtol=0, atol=1e-12 * np.abs(x).max())
    assert np.all(u[tuple(np.r_[0])] == 0)


@pytest.mark.parametrize("dim,n", [(2, 64), (2, 128), (3, 32)])
def test_fixed_point_is_dst_solve(orc, dim, n):
    f = rand_f(dim, n, 20 + n)
    ue = dst_solve(f)
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), f, rtol=0.0, max_cycles=25, check=False)
    assert st == orc.ERR_NOT_CONVERGED and rr < 1e-12, (cyc, rr)
    np.testing.assert_allclose(u, ue, rtol=0, atol=1e-11 * np.abs(ue).max())


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_manufactured_mode(orc, dim, n):
    h = 1.0 / n
    x = np.arange(n + 1) * h
    s = np.sin(np.pi * x)
    prod = s
    for _ in range(dim - 1):
        prod = np.multiply.outer(prod, s)
    f = -dim * np.pi**2 * prod
    exact = (np.pi**2 * h**2 / (4 * np.sin(np.pi * h / 2) ** 2)) * prod
    # 20 cycles reach the rounding floor (rtol 0: run them all)
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), f, rtol=0.0, max_cycles=20, check=False)
    assert st == orc.ERR_NOT_CONVERGED and cyc == 20 and rr < 1e-12
    np.testing.assert_allclose(u, exact, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_cycle_is_affine(orc, dim, n):
    rng = np.random.default_rng(3)
    inner = (slice(1, -1),) * dim
    u1, u2 = np.zeros((n + 1,) * dim), np.zeros((n + 1,) * dim)
    u1[inner] = rng.standard_normal((n - 1,) * dim)
    u2[inner] = rng.standard_normal((n - 1,) * dim)
    f1, f2 = rand_f(dim, n, 4), rand_f(dim, n, 5)
    a, b = 0.7, -1.9
    lhs = orc.vcycle(a * u1 + b * u2, a * f1 + b * f2)
    rhs = a * orc.vcycle(u1, f1) + b * orc.vcycle(u2, f2)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13 * np.abs(rhs).max())


def _square_syms():
    for T in (False, True):
        for fy in (False, True):
            for fx in (False, True):
                def g(a, T=T, fy=fy, fx=fx):
                    if T:
                        a = a.T
                    if fy:
                        a = a[::-1, :]
                    if fx:
                        a = a[:, ::-1]
                    return np.ascontiguousarray(a)
                yield g


def _cube_syms():
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((False, True), repeat=3):
            def g(a, perm=perm, flips=flips):
                a = np.transpose(a, perm)
                for ax, fl in enumerate(flips):
                    if fl:
                        a = np.flip(a, ax)
                return np.ascontiguousarray(a)
            yield g


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8), (3, 16)])
def test_cycle_commutes_with_grid_symmetries(orc, dim, n):
    rng = np.random.default_rng(6)
    inner = (slice(1, -1),) * dim
    u = np.zeros((n + 1,) * dim)
    u[inner] = rng.standard_normal((n - 1,) * dim)
    f = rand_f(dim, n, 7)
    base = orc.vcycle(u, f)
    syms = list(_square_syms() if dim == 2 else _cube_syms())
    assert len(syms) == (8 if dim == 2 else 48)
    for g in syms:
        out = orc.vcycle(g(u), g(f))
        np.testing.assert_allclose(out, g(base), rtol=0, atol=1e-13 * np.abs(base).max())


@pytest.mark.parametrize("dim,n", [(2, 64), (3, 16)])
def test_single_precision_cycle_refines_to_1e10(orc, dim, n):
    f = rand_f(dim, n, 30 + n)
    u64 = orc.vcycle(np.zeros_like(f), f, prec=0)
    u32 = orc.vcycle(np.zeros_like(f), f, prec=1)
    # one cycle: single-precision rounding of r, v and every level (relative ~1e-6)
    np.testing.assert_allclose(u32, u64, rtol=0, atol=1e-5 * np.abs(u64).max())
    assert np.abs(u32 - u64).max() > 0  # really computed in single
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), f, prec=1, rtol=1e-10, max_cycles=30)
    assert st == orc.OK and rr <= 1e-10
    ue = dst_solve(f)
    assert np.abs(u - ue).max() <= 1e-9 * np.abs(ue).max()


def test_solve_status_codes(orc):
    n = 16
    f = rand_f(2, n, 1)
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), f, rtol=1e-10, max_cycles=2, check=False)
    assert st == orc.ERR_NOT_CONVERGED and cyc == 2 and len(hist) == 3
    assert hist[0] == pytest.approx(1.0)
    # a strongly over-relaxed cycle diverges
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), f, p=(3.0,), rtol=1e-10, max_cycles=40, check=False)
    assert st == orc.ERR_DIVERGED
    fbad = f.copy()
    fbad[3, 3] = np.nan
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), fbad, rtol=1e-10, max_cycles=5, check=False)
    assert st == orc.ERR_NONFINITE
    # zero right-hand side and zero start: converged before any cycle
    u, cyc, rr, hist, st = orc.solve(np.zeros_like(f), np.zeros_like(f), rtol=1e-10, max_cycles=5)
    assert st == orc.OK and cyc == 0

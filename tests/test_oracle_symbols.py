"""Pins of every oracle step against closed-form sine-mode symbols.

A sine mode prod_i sin(k_i pi x_i) vanishes on the boundary of the unit square
or cube, so each stencil of the paper maps it to itself times a known factor at
every interior point, with no boundary correction.  Points that are not on the
input level are filled with NaN, so a step that reads a wrong neighbour class
produces NaN and fails.  Distinct wavenumbers per axis make a transposed or
wrongly permuted stencil fail too.
"""
import itertools

import numpy as np
import pytest


def mode2(m, k, l):
    a = np.arange(m + 1) / m
    return np.outer(np.sin(l * np.pi * a), np.sin(k * np.pi * a))  # [y, x]


def mode3(m, k, l, q):
    a = np.arange(m + 1) / m
    sx, sy, sz = np.sin(k * np.pi * a), np.sin(l * np.pi * a), np.sin(q * np.pi * a)
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]  # [z, y, x]


def idx2(m):
    b, a = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    inter = (a > 0) & (a < m) & (b > 0) & (b < m)
    return a, b, inter


def idx3(m):
    c, b, a = np.meshgrid(np.arange(m + 1), np.arange(m + 1), np.arange(m + 1), indexing="ij")
    inter = (a > 0) & (a < m) & (b > 0) & (b < m) & (c > 0) & (c < m)
    return a, b, c, inter


def with_nan(arr, member, m, dim):
    out = np.array(arr, dtype=np.float64)
    idx = idx2(m) if dim == 2 else idx3(m)
    inter = idx[-1]
    # boundary values stay (they are zero for a sine mode); interior non-members -> NaN
    out[inter & ~member] = np.nan
    return out


@pytest.mark.parametrize("n,k,l", [(8, 1, 3), (16, 5, 2), (32, 7, 11)])
def test_residual_5pt_symbol(orc, n, k, l):
    h = 1.0 / n
    u = mode2(n, k, l)
    lam = -(4 / h**2) * (np.sin(k * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2)
    r = orc.residual(u, np.zeros_like(u))
    np.testing.assert_allclose(r, -lam * u, rtol=0, atol=1e-12 * abs(lam))


@pytest.mark.parametrize("n,k,l,q", [(8, 1, 3, 2), (16, 5, 2, 7)])
def test_residual_7pt_symbol(orc, n, k, l, q):
    h = 1.0 / n
    u = mode3(n, k, l, q)
    lam = -(4 / h**2) * sum(np.sin(w * np.pi * h / 2) ** 2 for w in (k, l, q))
    r = orc.residual(u, np.zeros_like(u))
    np.testing.assert_allclose(r, -lam * u, rtol=0, atol=1e-12 * abs(lam))


@pytest.mark.parametrize("m,k,l", [(8, 1, 2), (16, 3, 5), (32, 9, 4)])
def test_restrict_2d_symbols(orc, m, k, l):
    ck, cl = np.cos(k * np.pi / m), np.cos(l * np.pi / m)
    a, b, inter = idx2(m)
    md = mode2(m, k, l)
    # Eq. Erest2r: axis grid -> diagonal grid of the same stride
    out = orc.step_restrict(2, 0, md)
    diag = inter & ((a + b) % 2 == 0)
    exp = np.where(diag, md * (0.5 + (ck + cl) / 4), 0.0)
    np.testing.assert_allclose(out, exp, atol=1e-14)
    # Eq. Erest2b: diagonal grid -> axis grid of twice the stride (input: diagonal members only)
    out = orc.step_restrict(2, 1, with_nan(md, (a + b) % 2 == 0, m, 2))
    assert np.isfinite(out).all()
    exp = md[::2, ::2] * (1 + ck * cl) / 2
    exp[[0, -1], :] = 0
    exp[:, [0, -1]] = 0
    np.testing.assert_allclose(out, exp, atol=1e-14)


@pytest.mark.parametrize("m,k,l,q", [(8, 1, 2, 3), (16, 5, 3, 2)])
def test_restrict_3d_symbols(orc, m, k, l, q):
    c1, c2, c3 = (np.cos(w * np.pi / m) for w in (k, l, q))
    a, b, c, inter = idx3(m)
    nodd = (a % 2) + (b % 2) + (c % 2)
    md = mode3(m, k, l, q)
    # Eq. Erred: green -> red
    out = orc.step_restrict(3, 0, md)
    exp = np.where(inter & (nodd % 2 == 0), md * (3 + c1 + c2 + c3) / 6, 0.0)
    np.testing.assert_allclose(out, exp, atol=1e-14)
    # Eqs. Ermagc / Ermagm: red -> magenta (input: red members only)
    out = orc.step_restrict(3, 1, with_nan(md, nodd % 2 == 0, m, 3))
    assert np.isfinite(out).all()
    exp = np.where(inter & (nodd == 0), md * (3 + c1 * c2 + c1 * c3 + c2 * c3) / 6,
                   np.where(inter & (nodd == 3), md * (c1 + c2 + c3) / 3, 0.0))
    np.testing.assert_allclose(out, exp, atol=1e-14)
    # Eq. Erblu: magenta -> blue (input: magenta members only)
    out = orc.step_restrict(3, 2, with_nan(md, (nodd == 0) | (nodd == 3), m, 3))
    assert np.isfinite(out).all()
    exp = md[::2, ::2, ::2] * (1 + c1 * c2 * c3) / 2
    mc = m // 2
    _, _, _, ic = idx3(mc)
    exp[~ic] = 0
    np.testing.assert_allclose(out, exp, atol=1e-14)


@pytest.mark.parametrize("m,k,l,alpha,cc", [(8, 1, 3, 0.7, 0.3), (16, 4, 7, -1.3, 0.05)])
def test_jacobi_2d_symbols(orc, m, k, l, alpha, cc):
    """Eqs. Ejacr/Ejacb with over-relaxation (Eajacr/Eajacb) and the axis-grid analogue."""
    ck, cl = np.cos(k * np.pi / m), np.cos(l * np.pi / m)
    a, b, inter = idx2(m)
    md = mode2(m, k, l)
    r = alpha * md
    # axis grid: coarse input is the diagonal grid of the same stride
    vd = with_nan(md, (a + b) % 2 == 0, m, 2)
    v = orc.step_jacobi(2, 0, cc, r, vd)
    beta = (-cc * alpha + 2 * (ck + cl)) / 4
    gamma = (-cc * alpha + 2 * (ck + cl) * beta) / 4
    exp = np.where(inter & ((a + b) % 2 == 1), beta * md, np.where(inter, gamma * md, 0.0))
    np.testing.assert_allclose(v, exp, atol=1e-14)
    # diagonal grid: coarse input is the axis grid of twice the stride
    va = md[::2, ::2].copy()
    v = orc.step_jacobi(2, 1, cc, with_nan(r, (a + b) % 2 == 0, m, 2), va)
    beta = (-cc * alpha + 4 * ck * cl) / 4
    gamma = (-cc * alpha + 4 * ck * cl * beta) / 4
    odd = inter & (a % 2 == 1) & (b % 2 == 1)
    even = inter & (a % 2 == 0) & (b % 2 == 0)
    exp = np.where(odd, beta * md, np.where(even, gamma * md, 0.0))
    np.testing.assert_allclose(v, exp, atol=1e-14)


@pytest.mark.parametrize("m,k,l,q,alpha", [(8, 1, 2, 3, 0.6), (16, 3, 5, 2, -0.9)])
def test_jacobi_3d_symbols(orc, m, k, l, q, alpha):
    """Eqs. Egprolg/Egprolr, Erprolr/Erprolm (all three face orientations), Emprolm/Emprolb."""
    c1, c2, c3 = (np.cos(w * np.pi / m) for w in (k, l, q))
    a, b, c, inter = idx3(m)
    nodd = (a % 2) + (b % 2) + (c % 2)
    md = mode3(m, k, l, q)
    r = alpha * md
    # green: coarse input red (same side)
    cg = 0.37
    v = orc.step_jacobi(3, 0, cg, r, with_nan(md, nodd % 2 == 0, m, 3))
    beta = (-cg * alpha + 2 * (c1 + c2 + c3)) / 6
    gamma = (-cg * alpha + 2 * (c1 + c2 + c3) * beta) / 6
    exp = np.where(inter & (nodd % 2 == 1), beta * md, np.where(inter, gamma * md, 0.0))
    np.testing.assert_allclose(v, exp, atol=1e-14)
    # red: coarse input magenta (same side); residual only read on red points
    ca, cb = 0.21, 0.44
    v = orc.step_jacobi(3, 1, [ca, cb], with_nan(r, nodd % 2 == 0, m, 3),
                        with_nan(md, (nodd == 0) | (nodd == 3), m, 3))
    bx = (-ca * alpha + 4 * c1 + 4 * c2 * c3) / 8   # even axis x (a even; b, c odd)
    by = (-ca * alpha + 4 * c2 + 4 * c1 * c3) / 8
    bz = (-ca * alpha + 4 * c3 + 4 * c1 * c2) / 8
    ge = (-cb * alpha + 4 * c1 * c2 * bz + 4 * c1 * c3 * by + 4 * c2 * c3 * bx) / 12
    ev = [(a % 2 == 0), (b % 2 == 0), (c % 2 == 0)]
    exp = np.zeros_like(md)
    two = inter & (nodd == 2)
    for e, bb in zip(ev, (bx, by, bz)):
        exp = np.where(two & e, bb * md, exp)
    exp = np.where(inter & (nodd == 0), ge * md, exp)
    np.testing.assert_allclose(v, exp, atol=1e-14)
    # magenta: coarse input blue (side m/2)
    cm = 0.29
    vb = md[::2, ::2, ::2].copy()
    v = orc.step_jacobi(3, 2, cm, with_nan(r, (nodd == 0) | (nodd == 3), m, 3), vb)
    beta = (-cm * alpha + 8 * c1 * c2 * c3) / 8
    gamma = (-cm * alpha + 8 * c1 * c2 * c3 * beta) / 8
    exp = np.where(inter & (nodd == 3), beta * md, np.where(inter & (nodd == 0), gamma * md, 0.0))
    np.testing.assert_allclose(v, exp, atol=1e-14)


def test_single_unknown_cycle_is_exact_jacobi(orc):
    """n = 2: one interior node, so the cycle is one Jacobi step from zero:
    v = -p h^2 r / 4 (2D) and -p_g h^2 r / 6 (3D), h = 1/2."""
    u = np.zeros((3, 3)); f = np.zeros((3, 3)); f[1, 1] = 1.0
    out = orc.vcycle(u, f, (1.052,))
    assert out[1, 1] == pytest.approx(-1.052 * 0.25 / 4, rel=1e-15)
    u = np.zeros((3, 3, 3)); f = np.zeros((3, 3, 3)); f[1, 1, 1] = 1.0
    out = orc.vcycle(u, f, (1.11, 1.42, 1.08, 0.99))
    assert out[1, 1, 1] == pytest.approx(-0.99 * 0.25 / 6, rel=1e-15)

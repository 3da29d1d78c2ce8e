"""Per-step check of a single-precision GPU cycle against the oracle.

Every level of a GPU cycle with single-precision levels is compared with the
oracle's double-precision step (one restriction, or one two-colour Jacobi
step) applied to the GPU's own input levels, read back as doubles.  The only
difference left is the rounding of that one step, so each level is bounded by
a few float ulps of the values it is computed from rather than of anything
else in the cycle:

* restriction into level d (Eqs. Erest2r, Erest2b; Erred, Ermagc, Ermagm,
  Erblu): positive weights summing to 1 over at most 13 terms; the rounding
  of the running sum and of the final scaling is at most ~5 eps32 of the
  largest input value (the 3D corner restriction, 24 terms of weight 1/24),
  bounded here by 16 eps32 * max|r_{d-1}|;
* Jacobi at level d (Eqs. Eajacr/Eajacb and their axis-grid analogue;
  Emprolm .. Egprolr): the first colour is a sum of at most 8 coarse values
  and c*r scaled by 1/4 .. 1/8; the second colour repeats that on the first
  colour's new values, so it inherits the first colour's rounding with
  weight 1 (the weights sum to 1).  The bound is
  16 eps32 * (max|v_{d+1}| + |c| max|r_d| + max|v_d|);
  the coefficient c is the single-precision value the GPU multiplies by;
* the finest residual is computed in double and rounded to single:
  eps32 * max|r_0| plus the double rounding of the stencil,
  64 eps64 * (max|f| + (2 dim + 4) max|u| / h^2);
* the finest correction reaches u in double (u += v): the double rounding of
  that sum, 4 eps64 * max|u_new|, is added to the Jacobi bound.
"""
import numpy as np

EPS32 = float(np.finfo(np.float32).eps)
EPS64 = float(np.finfo(np.float64).eps)


def _f32(x):
    return float(np.float32(x))


def restrict_kind(dim, d):
    """Oracle restriction kind producing depth d from depth d-1."""
    if dim == 2:
        return 0 if d % 2 == 1 else 1
    return {1: 0, 2: 1, 0: 2}[d % 3]


def jacobi_step(dim, n, d, p):
    """(kind, coefficients) of the Jacobi step at depth d, rounded to single."""
    m = n >> (d // dim)
    sh = (n // m) / n                     # sigma * h
    if dim == 2:
        return (0, [_f32(p[0] * sh * sh)]) if d % 2 == 0 else (1, [_f32(2 * p[0] * sh * sh)])
    pm, pr1, pr2, pg = p
    t = d % 3
    if t == 0:
        return 0, [_f32(pg * sh * sh)]
    if t == 1:
        return 1, [_f32(2 * pr1 * sh * sh), _f32(4 * pr2 * sh * sh)]
    return 2, [_f32(4 * pm * sh * sh)]


def check_fp32_cycle(orc, dim, n, p, u0, f, ug, gr, gv, order=2):
    """gr[d]: GPU residual of depth d (d = 0 .. D); gv[d-1]: GPU correction of
    depth d (d = 1 .. D); ug: u after the GPU cycle (u0 before).  Returns the
    largest ratio error / bound seen (every one must be <= 1)."""
    D = len(gr) - 1
    worst = 0.0
    r0 = orc.residual(u0, f, order=order)
    sten = 2 * dim + 4 if order == 2 else (40 if dim == 2 else 60)
    b0 = EPS32 * np.abs(r0).max() + 64 * EPS64 * (np.abs(f).max() + sten * np.abs(u0).max() * n * n)
    e0 = np.abs(gr[0] - r0).max()
    assert e0 <= b0, ("r", 0, e0, b0)
    worst = max(worst, e0 / b0)
    for d in range(1, D + 1):
        ref = orc.step_restrict(dim, restrict_kind(dim, d), gr[d - 1])
        bound = 16 * EPS32 * np.abs(gr[d - 1]).max() + 1e-300
        err = np.abs(gr[d] - ref).max()
        assert err <= bound, ("r", d, err, bound)
        worst = max(worst, err / bound)
    for d in range(D, -1, -1):
        kind, c = jacobi_step(dim, n, d, p)
        m = n >> (d // dim)
        if d == D:
            vc = np.zeros((m + 1,) * dim)
        else:
            vc = gv[d]                                   # depth d+1
        ref = orc.step_jacobi(dim, kind, c, gr[d], vc)
        got = gv[d - 1] if d >= 1 else ug - u0
        bound = 16 * EPS32 * (np.abs(vc).max() + max(abs(x) for x in c) * np.abs(gr[d]).max() + np.abs(ref).max())
        if d == 0:
            bound += 4 * EPS64 * np.abs(ug).max()
        bound += 1e-300
        err = np.abs(got - ref).max()
        assert err <= bound, ("v", d, err, bound)
        worst = max(worst, err / bound)
    return worst


def check_fp32_cycle_usual(orc, dim, n, p, u0, f, ug, gr, gv, order=2):
    """The same per-step check for the conventional cycle (full weighting,
    interpolation plus one red-black Jacobi iteration; levels of side n >> d).
    The bounds are those above: the full weighting has positive weights
    summing to 1 (at most 27 terms; its running sums round to at most ~4 eps32
    of the largest input), and an up step's interpolated values are means of
    coarse values, so they never exceed max|v_{d+1}|."""
    D = len(gr) - 1
    worst = 0.0
    r0 = orc.residual(u0, f, order=order)
    sten = 2 * dim + 4 if order == 2 else (40 if dim == 2 else 60)
    b0 = EPS32 * np.abs(r0).max() + 64 * EPS64 * (np.abs(f).max() + sten * np.abs(u0).max() * n * n)
    e0 = np.abs(gr[0] - r0).max()
    assert e0 <= b0, ("r", 0, e0, b0)
    worst = max(worst, e0 / b0)
    rk = 2 if dim == 2 else 3
    for d in range(1, D + 1):
        ref = orc.step_restrict(dim, rk, gr[d - 1])
        bound = 16 * EPS32 * np.abs(gr[d - 1]).max() + 1e-300
        err = np.abs(gr[d] - ref).max()
        assert err <= bound, ("r", d, err, bound)
        worst = max(worst, err / bound)
    for d in range(D, -1, -1):
        m = n >> d
        c = _f32(p * ((1 << d) / n) ** 2)
        vc = np.zeros((m // 2 + 1,) * dim) if d == D else gv[d]
        ref = orc.step_jacobi(dim, rk, [c], gr[d], vc)
        got = gv[d - 1] if d >= 1 else ug - u0
        bound = 16 * EPS32 * (np.abs(vc).max() + abs(c) * np.abs(gr[d]).max() + np.abs(ref).max())
        if d == 0:
            bound += 4 * EPS64 * np.abs(ug).max()
        bound += 1e-300
        err = np.abs(got - ref).max()
        assert err <= bound, ("v", d, err, bound)
        worst = max(worst, err / bound)
    return worst

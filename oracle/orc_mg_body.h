/*
 * Oracle body: one V-cycle of the diagonally oriented multigrid for the
 * discrete Poisson equation, written as plainly as possible.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU reference that the GPU
 * path is checked against; nothing in the product links it.
 *
 * Included twice by orc_mg.c: with R = double (SFX adds nothing) and with
 * R = float (SFX appends "_f32").  R is the type every level residual and
 * correction is held in; the finest residual r = f - Lap(u) and the update
 * u += v are always computed in double (the f32 instance is the
 * mixed-precision iterative refinement: the cycle in single, the outer
 * residual and the update in double).
 *
 * Storage: every level is a full array of its own stride sigma, natural
 * order with x fastest, indices in units of sigma (the paper indexes every
 * level of a group with the subscripts of that group's finest grid,
 * Section 3.1).  Points of the array that are not on the level, and
 * boundary points, hold 0 (zero Dirichlet data for the correction).
 *
 * 2D (Section 2): n = 2^K, depth d = 0 .. 2(K-1).  Even d: axis grid,
 * sigma = 2^(d/2), spacing sigma*h.  Odd d: diagonal grid of the points
 * with (a+b) even, sigma = 2^((d-1)/2), spacing sqrt2*sigma*h.  Array side
 * m+1 with m = n/sigma.
 *
 * 3D (Section 3): depth d = 3q+t, sigma = 2^q.  t=0 green (cubic), t=1 red
 * (points with a+b+c even: cube corners and face centres), t=2 magenta
 * (points with a,b,c all even or all odd: corners and cube centres).  The
 * blue grid that ends a group is the next group's green grid.
 *
 * Every sum below is evaluated left to right in the order the paper prints
 * its terms; the build uses -ffp-contract=off.
 */

/* ------------------------------------------------------------------ 2D */

#define I2(m, a, b) ((size_t)(b) * (size_t)((m) + 1) + (size_t)(a))

/* Eq. (Erest2r): restriction from an axis grid to the diagonal grid of the
 * same stride; the weights are 1/2 on the point and 1/8 on each of its four
 * axis neighbours (Fig. Erest2).  Coarse side is m as well. */
static void SFX(rs2_axis_to_diag)(int m, const R *r, R *rc)
{
    memset(rc, 0, sizeof(R) * (size_t)(m + 1) * (size_t)(m + 1));
    for (int b = 1; b < m; b++)
        for (int a = 1; a < m; a++) {
            if ((a + b) % 2 != 0) continue;
            rc[I2(m, a, b)] = (R)((4 * r[I2(m, a, b)] + r[I2(m, a - 1, b)] + r[I2(m, a, b - 1)]
                                   + r[I2(m, a + 1, b)] + r[I2(m, a, b + 1)]) / 8);
        }
}

/* Eq. (Erest2b): restriction from a diagonal grid (side m) onto the axis
 * grid of twice the stride (side m/2), weights 1/2 and 1/8 on the four
 * diagonal neighbours. */
static void SFX(rs2_diag_to_axis)(int m, const R *r, R *rc)
{
    int mc = m / 2;
    memset(rc, 0, sizeof(R) * (size_t)(mc + 1) * (size_t)(mc + 1));
    for (int B = 1; B < mc; B++)
        for (int A = 1; A < mc; A++) {
            int a = 2 * A, b = 2 * B;
            rc[I2(mc, A, B)] = (R)((4 * r[I2(m, a, b)] + r[I2(m, a - 1, b - 1)] + r[I2(m, a + 1, b - 1)]
                                    + r[I2(m, a + 1, b + 1)] + r[I2(m, a - 1, b + 1)]) / 8);
        }
}

/* Jacobi prolongation onto an axis grid of side m (Section 2.2, "similarly
 * for a green grid"; over-relaxed form Section 2.4).  c = p*(sigma*h)^2.
 * First the points with (a+b) odd, which are not on the coarser diagonal
 * grid, from the four axis neighbours of vd (the coarser diagonal level,
 * same side m); then the points with (a+b) even from the new odd values. */
static void SFX(jac2_axis)(int m, R c, const R *r, const R *vd, R *v)
{
    memset(v, 0, sizeof(R) * (size_t)(m + 1) * (size_t)(m + 1));
    for (int b = 1; b < m; b++)
        for (int a = 1; a < m; a++) {
            if ((a + b) % 2 != 1) continue;
            v[I2(m, a, b)] = (R)((-c * r[I2(m, a, b)] + vd[I2(m, a - 1, b)] + vd[I2(m, a, b - 1)]
                                  + vd[I2(m, a + 1, b)] + vd[I2(m, a, b + 1)]) / 4);
        }
    for (int b = 1; b < m; b++)
        for (int a = 1; a < m; a++) {
            if ((a + b) % 2 != 0) continue;
            v[I2(m, a, b)] = (R)((-c * r[I2(m, a, b)] + v[I2(m, a - 1, b)] + v[I2(m, a, b - 1)]
                                  + v[I2(m, a + 1, b)] + v[I2(m, a, b + 1)]) / 4);
        }
}

/* Eq. (Eajacr) then Eq. (Eajacb): Jacobi prolongation onto a diagonal grid
 * of side m from the axis grid va of twice the stride (side m/2).
 * c = 2*p*(sigma*h)^2 (the diagonal spacing is sqrt2*sigma*h).  First the
 * points with a,b odd (not on the coarser grid), then the points with a,b
 * even from the new odd values. */
static void SFX(jac2_diag)(int m, R c, const R *r, const R *va, R *v)
{
    int mc = m / 2;
    memset(v, 0, sizeof(R) * (size_t)(m + 1) * (size_t)(m + 1));
    for (int b = 1; b < m; b += 2)
        for (int a = 1; a < m; a += 2) {
            int A0 = (a - 1) / 2, A1 = (a + 1) / 2, B0 = (b - 1) / 2, B1 = (b + 1) / 2;
            v[I2(m, a, b)] = (R)((-c * r[I2(m, a, b)] + va[I2(mc, A0, B0)] + va[I2(mc, A1, B0)]
                                  + va[I2(mc, A1, B1)] + va[I2(mc, A0, B1)]) / 4);
        }
    for (int b = 2; b < m; b += 2)
        for (int a = 2; a < m; a += 2)
            v[I2(m, a, b)] = (R)((-c * r[I2(m, a, b)] + v[I2(m, a - 1, b - 1)] + v[I2(m, a + 1, b - 1)]
                                  + v[I2(m, a + 1, b + 1)] + v[I2(m, a - 1, b + 1)]) / 4);
}

/* ------------------------------------------------------------------ 3D */

#define I3(m, a, b, c) (((size_t)(c) * (size_t)((m) + 1) + (size_t)(b)) * (size_t)((m) + 1) + (size_t)(a))

static size_t SFX(vol3)(int m) { return (size_t)(m + 1) * (size_t)(m + 1) * (size_t)(m + 1); }

/* Eq. (Erred): green -> red (same side m), at the points with a+b+c even. */
static void SFX(rs3_green_to_red)(int m, const R *r, R *rc)
{
    memset(rc, 0, sizeof(R) * SFX(vol3)(m));
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                if ((i + j + k) % 2 != 0) continue;
                rc[I3(m, i, j, k)] = (R)((6 * r[I3(m, i, j, k)]
                    + r[I3(m, i + 1, j, k)] + r[I3(m, i - 1, j, k)] + r[I3(m, i, j + 1, k)] + r[I3(m, i, j - 1, k)]
                    + r[I3(m, i, j, k + 1)] + r[I3(m, i, j, k - 1)]) / 12);
            }
}

/* Eq. (Ermagc) at the magenta corners (all indices even) and Eq. (Ermagm)
 * at the magenta cube centres (all odd, no centre term). */
static void SFX(rs3_red_to_magenta)(int m, const R *r, R *rc)
{
    memset(rc, 0, sizeof(R) * SFX(vol3)(m));
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                int odd = (i & 1) + (j & 1) + (k & 1);
                if (odd == 0)
                    rc[I3(m, i, j, k)] = (R)((12 * r[I3(m, i, j, k)]
                        + r[I3(m, i + 1, j + 1, k)] + r[I3(m, i + 1, j - 1, k)]
                        + r[I3(m, i - 1, j - 1, k)] + r[I3(m, i - 1, j + 1, k)]
                        + r[I3(m, i + 1, j, k + 1)] + r[I3(m, i + 1, j, k - 1)]
                        + r[I3(m, i - 1, j, k - 1)] + r[I3(m, i - 1, j, k + 1)]
                        + r[I3(m, i, j + 1, k + 1)] + r[I3(m, i, j + 1, k - 1)]
                        + r[I3(m, i, j - 1, k - 1)] + r[I3(m, i, j - 1, k + 1)]) / 24);
                else if (odd == 3)
                    rc[I3(m, i, j, k)] = (R)((r[I3(m, i + 1, j, k)] + r[I3(m, i - 1, j, k)]
                        + r[I3(m, i, j + 1, k)] + r[I3(m, i, j - 1, k)]
                        + r[I3(m, i, j, k + 1)] + r[I3(m, i, j, k - 1)]) / 6);
            }
}

/* Eq. (Erblu): magenta (side m) -> blue = green grid of twice the stride
 * (side m/2), at the blue points (all indices even). */
static void SFX(rs3_magenta_to_blue)(int m, const R *r, R *rc)
{
    int mc = m / 2;
    memset(rc, 0, sizeof(R) * SFX(vol3)(mc));
    for (int C = 1; C < mc; C++)
        for (int B = 1; B < mc; B++)
            for (int A = 1; A < mc; A++) {
                int i = 2 * A, j = 2 * B, k = 2 * C;
                rc[I3(mc, A, B, C)] = (R)((8 * r[I3(m, i, j, k)]
                    + r[I3(m, i + 1, j + 1, k + 1)] + r[I3(m, i + 1, j + 1, k - 1)]
                    + r[I3(m, i + 1, j - 1, k + 1)] + r[I3(m, i + 1, j - 1, k - 1)]
                    + r[I3(m, i - 1, j + 1, k + 1)] + r[I3(m, i - 1, j + 1, k - 1)]
                    + r[I3(m, i - 1, j - 1, k + 1)] + r[I3(m, i - 1, j - 1, k - 1)]) / 16);
            }
}

/* Eq. (Emprolm) then Eq. (Emprolb): magenta-blue Jacobi on the magenta grid
 * (side m) from the blue grid vb (side m/2).  c = 4*p_m*(sigma*h)^2.
 * Cube centres (all odd) from their eight blue neighbours, then the corners
 * (all even) from the new centre values. */
static void SFX(jac3_magenta)(int m, R c, const R *r, const R *vb, R *v)
{
    int mc = m / 2;
    memset(v, 0, sizeof(R) * SFX(vol3)(m));
    for (int k = 1; k < m; k += 2)
        for (int j = 1; j < m; j += 2)
            for (int i = 1; i < m; i += 2) {
                int i0 = (i - 1) / 2, i1 = (i + 1) / 2, j0 = (j - 1) / 2, j1 = (j + 1) / 2;
                int k0 = (k - 1) / 2, k1 = (k + 1) / 2;
                v[I3(m, i, j, k)] = (R)((-c * r[I3(m, i, j, k)]
                    + vb[I3(mc, i1, j1, k1)] + vb[I3(mc, i1, j1, k0)]
                    + vb[I3(mc, i1, j0, k1)] + vb[I3(mc, i1, j0, k0)]
                    + vb[I3(mc, i0, j1, k1)] + vb[I3(mc, i0, j1, k0)]
                    + vb[I3(mc, i0, j0, k1)] + vb[I3(mc, i0, j0, k0)]) / 8);
            }
    for (int k = 2; k < m; k += 2)
        for (int j = 2; j < m; j += 2)
            for (int i = 2; i < m; i += 2)
                v[I3(m, i, j, k)] = (R)((-c * r[I3(m, i, j, k)]
                    + v[I3(m, i + 1, j + 1, k + 1)] + v[I3(m, i + 1, j + 1, k - 1)]
                    + v[I3(m, i + 1, j - 1, k + 1)] + v[I3(m, i + 1, j - 1, k - 1)]
                    + v[I3(m, i - 1, j + 1, k + 1)] + v[I3(m, i - 1, j + 1, k - 1)]
                    + v[I3(m, i - 1, j - 1, k + 1)] + v[I3(m, i - 1, j - 1, k - 1)]) / 8);
}

/* Eq. (Erprolr) then Eq. (Erprolm): red-magenta Jacobi on the red grid (side
 * m) from the magenta grid vm (same side).  c1 = 2*p_r1*(sigma*h)^2,
 * c2 = 4*p_r2*(sigma*h)^2.
 * Face centres (two indices odd): the two magenta cube centres along the
 * even axis count twice, plus the four magenta corners in the plane normal
 * to that axis; the paper prints the z-normal case and the x- and y-normal
 * cases are its cyclic permutations (k->i->j).  Then the corners (all even)
 * from their twelve new face-centre neighbours.  The magenta cube centres
 * are not on the red grid and are not carried. */
static void SFX(jac3_red)(int m, R c1, R c2, const R *r, const R *vm, R *v)
{
    memset(v, 0, sizeof(R) * SFX(vol3)(m));
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                int oi = i & 1, oj = j & 1, ok = k & 1;
                if (oi + oj + ok != 2) continue;
                R s;
                if (!ok)        /* face normal to z: i, j odd */
                    s = 2 * (vm[I3(m, i, j, k + 1)] + vm[I3(m, i, j, k - 1)])
                        + vm[I3(m, i + 1, j + 1, k)] + vm[I3(m, i + 1, j - 1, k)]
                        + vm[I3(m, i - 1, j - 1, k)] + vm[I3(m, i - 1, j + 1, k)];
                else if (!oi)   /* face normal to x: j, k odd (z->x, x->y, y->z) */
                    s = 2 * (vm[I3(m, i + 1, j, k)] + vm[I3(m, i - 1, j, k)])
                        + vm[I3(m, i, j + 1, k + 1)] + vm[I3(m, i, j + 1, k - 1)]
                        + vm[I3(m, i, j - 1, k - 1)] + vm[I3(m, i, j - 1, k + 1)];
                else            /* face normal to y: k, i odd */
                    s = 2 * (vm[I3(m, i, j + 1, k)] + vm[I3(m, i, j - 1, k)])
                        + vm[I3(m, i + 1, j, k + 1)] + vm[I3(m, i - 1, j, k + 1)]
                        + vm[I3(m, i - 1, j, k - 1)] + vm[I3(m, i + 1, j, k - 1)];
                v[I3(m, i, j, k)] = (R)((-c1 * r[I3(m, i, j, k)] + s) / 8);
            }
    for (int k = 2; k < m; k += 2)
        for (int j = 2; j < m; j += 2)
            for (int i = 2; i < m; i += 2)
                v[I3(m, i, j, k)] = (R)((-c2 * r[I3(m, i, j, k)]
                    + v[I3(m, i + 1, j + 1, k)] + v[I3(m, i + 1, j - 1, k)]
                    + v[I3(m, i - 1, j - 1, k)] + v[I3(m, i - 1, j + 1, k)]
                    + v[I3(m, i + 1, j, k + 1)] + v[I3(m, i + 1, j, k - 1)]
                    + v[I3(m, i - 1, j, k - 1)] + v[I3(m, i - 1, j, k + 1)]
                    + v[I3(m, i, j + 1, k + 1)] + v[I3(m, i, j + 1, k - 1)]
                    + v[I3(m, i, j - 1, k - 1)] + v[I3(m, i, j - 1, k + 1)]) / 12);
}

/* Eq. (Egprolg) then Eq. (Egprolr): green-red Jacobi on the green grid
 * (side m) from the red grid vr (same side).  c = p_g*(sigma*h)^2.  Points
 * with a+b+c odd (edge midpoints and cube centres) first, then the red
 * points from the new values. */
static void SFX(jac3_green)(int m, R c, const R *r, const R *vr, R *v)
{
    memset(v, 0, sizeof(R) * SFX(vol3)(m));
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                if ((i + j + k) % 2 != 1) continue;
                v[I3(m, i, j, k)] = (R)((-c * r[I3(m, i, j, k)]
                    + vr[I3(m, i + 1, j, k)] + vr[I3(m, i - 1, j, k)] + vr[I3(m, i, j + 1, k)]
                    + vr[I3(m, i, j - 1, k)] + vr[I3(m, i, j, k + 1)] + vr[I3(m, i, j, k - 1)]) / 6);
            }
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                if ((i + j + k) % 2 != 0) continue;
                v[I3(m, i, j, k)] = (R)((-c * r[I3(m, i, j, k)]
                    + v[I3(m, i + 1, j, k)] + v[I3(m, i - 1, j, k)] + v[I3(m, i, j + 1, k)]
                    + v[I3(m, i, j - 1, k)] + v[I3(m, i, j, k + 1)] + v[I3(m, i, j, k - 1)]) / 6);
            }
}

/* ------------------------------------------------------------ V-cycle */

/* One V-cycle (Section 1, Eq. Evpois): r = f - Lap_h(u) on the finest grid
 * (order 4: the fourth-order residual of Sections 2.3 / 3.3 instead),
 * restrict down to the coarsest grid (3x3 or 3x3x3, one interior node),
 * one Jacobi iteration on each grid going back up, the coarsest one starting
 * from zero, then u <- u + v.
 * p: 2D {p}; 3D {p_m, p_r1, p_r2, p_g}.
 * rtrace / vtrace (nullable): every level's residual and correction, in
 * depth order, each level as its full (m+1)^dim array, converted to double. */
static int SFX(vcycle)(int dim, int n, int order, const double *p, double *u, const double *f,
                       double *rtrace, double *vtrace)
{
    int K = orc_log2(n);
    if (K < 1 || (dim != 2 && dim != 3)) return ORC_ERR_SIZE;
    int D = (dim == 2) ? 2 * (K - 1) : 3 * (K - 1);
    double h = 1.0 / n;
    R **rl = (R **)calloc((size_t)D + 1, sizeof(R *));
    R **vl = (R **)calloc((size_t)D + 1, sizeof(R *));
    int *ml = (int *)calloc((size_t)D + 1, sizeof(int));
    if (!rl || !vl || !ml) { free(rl); free(vl); free(ml); return ORC_ERR_ALLOC; }
    int rc = ORC_OK;
    for (int d = 0; d <= D; d++) {
        int sig = (dim == 2) ? (1 << (d / 2)) : (1 << (d / 3));
        ml[d] = n / sig;
        size_t cnt = (dim == 2) ? (size_t)(ml[d] + 1) * (size_t)(ml[d] + 1) : SFX(vol3)(ml[d]);
        rl[d] = (R *)calloc(cnt, sizeof(R));
        vl[d] = (R *)calloc(cnt, sizeof(R));
        if (!rl[d] || !vl[d]) { rc = ORC_ERR_ALLOC; goto done; }
    }
    /* finest residual, computed in double (Eq. Evpois; order 4: Eq. Efos2 / Efos4) */
    {
        size_t cnt = (dim == 2) ? (size_t)(n + 1) * (size_t)(n + 1) : SFX(vol3)(n);
        double *r0 = (double *)malloc(cnt * sizeof(double));
        if (!r0) { rc = ORC_ERR_ALLOC; goto done; }
        orc_residual_ord_core(dim, n, order, u, f, r0);
        for (size_t q = 0; q < cnt; q++) rl[0][q] = (R)r0[q];
        free(r0);
    }
    /* restriction down the hierarchy */
    for (int d = 1; d <= D; d++) {
        if (dim == 2) {
            if (d % 2 == 1) SFX(rs2_axis_to_diag)(ml[d - 1], rl[d - 1], rl[d]);
            else            SFX(rs2_diag_to_axis)(ml[d - 1], rl[d - 1], rl[d]);
        } else {
            if (d % 3 == 1)      SFX(rs3_green_to_red)(ml[d - 1], rl[d - 1], rl[d]);
            else if (d % 3 == 2) SFX(rs3_red_to_magenta)(ml[d - 1], rl[d - 1], rl[d]);
            else                 SFX(rs3_magenta_to_blue)(ml[d - 1], rl[d - 1], rl[d]);
        }
    }
    /* Jacobi back up; the coarsest grid runs its own Jacobi from a zero
     * coarser correction (the zero array vz). */
    {
        size_t cz = (dim == 2) ? 9 : 27;
        R *vz = (R *)calloc(cz, sizeof(R));
        if (!vz) { rc = ORC_ERR_ALLOC; goto done; }
        for (int d = D; d >= 0; d--) {
            const R *vc = (d == D) ? vz : vl[d + 1];
            int m = ml[d];
            if (dim == 2) {
                double sh = (double)(n / m) * h;          /* sigma * h */
                if (d % 2 == 0) SFX(jac2_axis)(m, (R)(p[0] * sh * sh), rl[d], (d == D) ? vz : vc, vl[d]);
                else            SFX(jac2_diag)(m, (R)(2 * p[0] * sh * sh), rl[d], vc, vl[d]);
            } else {
                double sh = (double)(n / m) * h;
                if (d % 3 == 0)      SFX(jac3_green)(m, (R)(p[3] * sh * sh), rl[d], vc, vl[d]);
                else if (d % 3 == 1) SFX(jac3_red)(m, (R)(2 * p[1] * sh * sh), (R)(4 * p[2] * sh * sh), rl[d], vc, vl[d]);
                else                 SFX(jac3_magenta)(m, (R)(4 * p[0] * sh * sh), rl[d], vc, vl[d]);
            }
        }
        free(vz);
    }
    {
        size_t cnt = (dim == 2) ? (size_t)(n + 1) * (size_t)(n + 1) : SFX(vol3)(n);
        for (size_t q = 0; q < cnt; q++) u[q] = u[q] + (double)vl[0][q];
    }
    if (rtrace || vtrace) {
        size_t off = 0;
        for (int d = 0; d <= D; d++) {
            size_t cnt = (dim == 2) ? (size_t)(ml[d] + 1) * (size_t)(ml[d] + 1) : SFX(vol3)(ml[d]);
            for (size_t q = 0; q < cnt; q++) {
                if (rtrace) rtrace[off + q] = (double)rl[d][q];
                if (vtrace) vtrace[off + q] = (double)vl[d][q];
            }
            off += cnt;
        }
    }
done:
    for (int d = 0; d <= D; d++) { free(rl[d]); free(vl[d]); }
    free(rl); free(vl); free(ml);
    return rc;
}

/* ------------------------------------------- the conventional ("usual") cycle
 * The comparison scheme of Sections 2.1-2.3 and 3.1-3.3: the standard
 * hierarchy of axis-aligned (cubic) grids of spacing h, 2h, 4h, ... down to
 * one interior node; the conventional nine-point (2D) or 27-point (3D)
 * full-weighting restriction; bilinear (trilinear) interpolation of the
 * coarse correction followed by one Jacobi iteration on the finer grid
 * (nu1 = 0, nu2 = 1), taken in red-black order as the diagonal scheme's
 * sweeps are: the points with an odd index sum first, then the even ones
 * from the new odd values.  Every level is a full array of side m = n/sigma. */

/* nine-point full weighting: coarse (A,B) from the 3x3 fine block around
 * (2A,2B), weights 4 (centre), 2 (axis neighbours), 1 (diagonal), over 16 */
static void SFX(rs2_full)(int m, const R *r, R *rc)
{
    int mc = m / 2;
    memset(rc, 0, sizeof(R) * (size_t)(mc + 1) * (size_t)(mc + 1));
    for (int B = 1; B < mc; B++)
        for (int A = 1; A < mc; A++) {
            int a = 2 * A, b = 2 * B;
            rc[I2(mc, A, B)] = (R)((4 * r[I2(m, a, b)]
                + 2 * (r[I2(m, a + 1, b)] + r[I2(m, a, b + 1)] + r[I2(m, a - 1, b)] + r[I2(m, a, b - 1)])
                + r[I2(m, a + 1, b + 1)] + r[I2(m, a - 1, b + 1)] + r[I2(m, a - 1, b - 1)] + r[I2(m, a + 1, b - 1)])
                / 16);
        }
}

/* 27-point full weighting: weights 8 (centre), 4 (6 faces), 2 (12 edges),
 * 1 (8 corners), over 64 */
static void SFX(rs3_full)(int m, const R *r, R *rc)
{
    int mc = m / 2;
    memset(rc, 0, sizeof(R) * SFX(vol3)(mc));
    for (int C = 1; C < mc; C++)
        for (int B = 1; B < mc; B++)
            for (int A = 1; A < mc; A++) {
                int i = 2 * A, j = 2 * B, k = 2 * C;
                R faces = r[I3(m, i + 1, j, k)] + r[I3(m, i - 1, j, k)] + r[I3(m, i, j + 1, k)]
                        + r[I3(m, i, j - 1, k)] + r[I3(m, i, j, k + 1)] + r[I3(m, i, j, k - 1)];
                R edges = r[I3(m, i + 1, j + 1, k)] + r[I3(m, i + 1, j - 1, k)] + r[I3(m, i - 1, j + 1, k)]
                        + r[I3(m, i - 1, j - 1, k)] + r[I3(m, i + 1, j, k + 1)] + r[I3(m, i + 1, j, k - 1)]
                        + r[I3(m, i - 1, j, k + 1)] + r[I3(m, i - 1, j, k - 1)] + r[I3(m, i, j + 1, k + 1)]
                        + r[I3(m, i, j + 1, k - 1)] + r[I3(m, i, j - 1, k + 1)] + r[I3(m, i, j - 1, k - 1)];
                R corners = r[I3(m, i + 1, j + 1, k + 1)] + r[I3(m, i + 1, j + 1, k - 1)]
                          + r[I3(m, i + 1, j - 1, k + 1)] + r[I3(m, i + 1, j - 1, k - 1)]
                          + r[I3(m, i - 1, j + 1, k + 1)] + r[I3(m, i - 1, j + 1, k - 1)]
                          + r[I3(m, i - 1, j - 1, k + 1)] + r[I3(m, i - 1, j - 1, k - 1)];
                rc[I3(mc, A, B, C)] = (R)((8 * r[I3(m, i, j, k)] + 4 * faces + 2 * edges + corners) / 64);
            }
}

/* bilinear (2D) / trilinear (3D) interpolation from the grid of side m/2 onto
 * the grid of side m: a fine point with q odd indices is the mean of its 2^q
 * coarse neighbours (boundary values are 0 on both grids) */
static void SFX(interp_lin)(int dim, int m, const R *vc, R *v)
{
    int mc = m / 2;
    if (dim == 2) {
        memset(v, 0, sizeof(R) * (size_t)(m + 1) * (size_t)(m + 1));
        for (int b = 1; b < m; b++)
            for (int a = 1; a < m; a++) {
                int a0 = a / 2, a1 = (a + 1) / 2, b0 = b / 2, b1 = (b + 1) / 2;
                if (a % 2 == 0 && b % 2 == 0) v[I2(m, a, b)] = vc[I2(mc, a0, b0)];
                else if (b % 2 == 0) v[I2(m, a, b)] = (R)((vc[I2(mc, a0, b0)] + vc[I2(mc, a1, b0)]) / 2);
                else if (a % 2 == 0) v[I2(m, a, b)] = (R)((vc[I2(mc, a0, b0)] + vc[I2(mc, a0, b1)]) / 2);
                else v[I2(m, a, b)] = (R)((vc[I2(mc, a0, b0)] + vc[I2(mc, a1, b0)] + vc[I2(mc, a1, b1)]
                                            + vc[I2(mc, a0, b1)]) / 4);
            }
        return;
    }
    memset(v, 0, sizeof(R) * SFX(vol3)(m));
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                /* the mean of the distinct coarse corners: the indices of an
                 * odd axis take both neighbours, an even axis its own */
                int i0 = i / 2, i1 = (i + 1) / 2, j0 = j / 2, j1 = (j + 1) / 2, k0 = k / 2, k1 = (k + 1) / 2;
                int q = (i & 1) + (j & 1) + (k & 1);
                R s = 0;
                for (int kk = k0; kk <= k1; kk++)
                    for (int jj = j0; jj <= j1; jj++)
                        for (int ii = i0; ii <= i1; ii++) s = (R)(s + vc[I3(mc, ii, jj, kk)]);
                s = (R)(s / (R)(1 << q));
                v[I3(m, i, j, k)] = s;
            }
}

/* One red-black Jacobi iteration in place on the cubic grid of side m for
 * Lap v = r with spacing s (c = p s^2): v(x) = (sum of the 2 dim axis
 * neighbours - c r(x)) / (2 dim), first at the points with an odd index sum
 * from the values v holds, then at the even ones from the new odd values. */
static void SFX(rbj_cubic)(int dim, int m, R c, const R *r, R *v)
{
    for (int par = 1; par >= 0; par--) {
        if (dim == 2) {
            for (int b = 1; b < m; b++)
                for (int a = 1; a < m; a++) {
                    if ((a + b) % 2 != par) continue;
                    v[I2(m, a, b)] = (R)((-c * r[I2(m, a, b)] + v[I2(m, a - 1, b)] + v[I2(m, a, b - 1)]
                                          + v[I2(m, a + 1, b)] + v[I2(m, a, b + 1)]) / 4);
                }
        } else {
            for (int k = 1; k < m; k++)
                for (int j = 1; j < m; j++)
                    for (int i = 1; i < m; i++) {
                        if ((i + j + k) % 2 != par) continue;
                        v[I3(m, i, j, k)] = (R)((-c * r[I3(m, i, j, k)]
                            + v[I3(m, i + 1, j, k)] + v[I3(m, i - 1, j, k)] + v[I3(m, i, j + 1, k)]
                            + v[I3(m, i, j - 1, k)] + v[I3(m, i, j, k + 1)] + v[I3(m, i, j, k - 1)]) / 6);
                    }
        }
    }
}

/* One conventional V-cycle: r = f - Lap_h(u) on the finest grid (order 4:
 * Eq. Efos2 / Efos4), full weighting down to side 2, then from a zero
 * correction on the coarsest grid: interpolate, one red-black Jacobi
 * iteration with c = p (sigma h)^2, up to the finest grid; u <- u + v.
 * rtrace / vtrace (nullable): every level's residual and correction, finest
 * first, each as its full (m+1)^dim array. */
static int SFX(vcycle_usual)(int dim, int n, int order, double p, double *u, const double *f, double *rtrace,
                             double *vtrace)
{
    int K = orc_log2(n);
    if (K < 1 || (dim != 2 && dim != 3)) return ORC_ERR_SIZE;
    int D = K - 1;
    double h = 1.0 / n;
    R **rl = (R **)calloc((size_t)D + 1, sizeof(R *));
    R **vl = (R **)calloc((size_t)D + 1, sizeof(R *));
    if (!rl || !vl) { free(rl); free(vl); return ORC_ERR_ALLOC; }
    int rc = ORC_OK;
    for (int d = 0; d <= D; d++) {
        int m = n >> d;
        size_t cnt = (dim == 2) ? (size_t)(m + 1) * (size_t)(m + 1) : SFX(vol3)(m);
        rl[d] = (R *)calloc(cnt, sizeof(R));
        vl[d] = (R *)calloc(cnt, sizeof(R));
        if (!rl[d] || !vl[d]) { rc = ORC_ERR_ALLOC; goto done; }
    }
    {
        size_t cnt = (dim == 2) ? (size_t)(n + 1) * (size_t)(n + 1) : SFX(vol3)(n);
        double *r0 = (double *)malloc(cnt * sizeof(double));
        if (!r0) { rc = ORC_ERR_ALLOC; goto done; }
        orc_residual_ord_core(dim, n, order, u, f, r0);
        for (size_t q = 0; q < cnt; q++) rl[0][q] = (R)r0[q];
        free(r0);
    }
    for (int d = 1; d <= D; d++) {
        if (dim == 2) SFX(rs2_full)(n >> (d - 1), rl[d - 1], rl[d]);
        else SFX(rs3_full)(n >> (d - 1), rl[d - 1], rl[d]);
    }
    for (int d = D; d >= 0; d--) {
        int m = n >> d;
        double sh = (double)(1 << d) * h;    /* sigma * h */
        if (d < D) SFX(interp_lin)(dim, m, vl[d + 1], vl[d]);   /* the coarsest starts from vl[D] = 0 */
        SFX(rbj_cubic)(dim, m, (R)(p * sh * sh), rl[d], vl[d]);
    }
    {
        size_t cnt = (dim == 2) ? (size_t)(n + 1) * (size_t)(n + 1) : SFX(vol3)(n);
        for (size_t q = 0; q < cnt; q++) u[q] = u[q] + (double)vl[0][q];
    }
    if (rtrace || vtrace) {
        size_t off = 0;
        for (int d = 0; d <= D; d++) {
            int m = n >> d;
            size_t cnt = (dim == 2) ? (size_t)(m + 1) * (size_t)(m + 1) : SFX(vol3)(m);
            for (size_t q = 0; q < cnt; q++) {
                if (rtrace) rtrace[off + q] = (double)rl[d][q];
                if (vtrace) vtrace[off + q] = (double)vl[d][q];
            }
            off += cnt;
        }
    }
done:
    for (int d = 0; d <= D; d++) { free(rl[d]); free(vl[d]); }
    free(rl); free(vl);
    return rc;
}

/* ------------------------------------------ more sweeps per level, W-cycles
 * The paper leaves both to further research (Section 4: extra Jacobi
 * iterations on each level of the diagonal hierarchy; W-cycles, with more
 * scope there because the hierarchy has more levels).  Readings:
 *  - nu >= 1 red-black iterations per level on the way up: the first as in
 *    the V-cycle (first colour from the coarser level's values at the points
 *    both levels share), each further one the same step with the level's own
 *    current values at those points.  The red level's first colour also
 *    reads the magenta cube centres, which are not red points: those keep
 *    the values the magenta level handed up.
 *  - gamma visits (1: V-cycle, 2: W-cycle) of the coarse correction per
 *    group of levels (2D: axis -> diagonal -> axis of twice the stride; 3D:
 *    green -> red -> magenta -> blue): after the first visit returns w, the
 *    residual of the coarser axis (green) grid's own equation, r - A w with
 *    the 5-point (7-point) Laplacian of that grid's spacing, goes through a
 *    second visit whose correction is added to w.
 */

/* the coarse input of a further sweep on level d: the level's own values at
 * the points it shares with the level below, in that level's layout */
static void SFX(again_input)(int dim, int d, int m, const R *v, const R *vc_prev, R *out)
{
    if (dim == 2) {
        if (d % 2 == 0) { memcpy(out, v, sizeof(R) * (size_t)(m + 1) * (size_t)(m + 1)); return; }
        int mc = m / 2;
        for (int B = 0; B <= mc; B++)
            for (int A = 0; A <= mc; A++) out[I2(mc, A, B)] = v[I2(m, 2 * A, 2 * B)];
        return;
    }
    int t = d % 3;
    if (t == 0) { memcpy(out, v, sizeof(R) * SFX(vol3)(m)); return; }
    if (t == 1) {   /* the magenta input with its corners replaced by the red level's own */
        memcpy(out, vc_prev, sizeof(R) * SFX(vol3)(m));
        for (int k = 0; k <= m; k += 2)
            for (int j = 0; j <= m; j += 2)
                for (int i = 0; i <= m; i += 2) out[I3(m, i, j, k)] = v[I3(m, i, j, k)];
        return;
    }
    int mc = m / 2;
    for (int C = 0; C <= mc; C++)
        for (int B = 0; B <= mc; B++)
            for (int A = 0; A <= mc; A++) out[I3(mc, A, B, C)] = v[I3(m, 2 * A, 2 * B, 2 * C)];
}

/* one red-black Jacobi step of level d from the coarse input vc */
static void SFX(jac_step)(int dim, int n, int d, const int *ml, const double *p, const R *r, const R *vc, R *v)
{
    int m = ml[d];
    double sh = (double)(n / m) * (1.0 / n);   /* sigma * h */
    if (dim == 2) {
        if (d % 2 == 0) SFX(jac2_axis)(m, (R)(p[0] * sh * sh), r, vc, v);
        else SFX(jac2_diag)(m, (R)(2 * p[0] * sh * sh), r, vc, v);
    } else {
        if (d % 3 == 0) SFX(jac3_green)(m, (R)(p[3] * sh * sh), r, vc, v);
        else if (d % 3 == 1) SFX(jac3_red)(m, (R)(2 * p[1] * sh * sh), (R)(4 * p[2] * sh * sh), r, vc, v);
        else SFX(jac3_magenta)(m, (R)(4 * p[0] * sh * sh), r, vc, v);
    }
}

static void SFX(restrict_step)(int dim, int d, const int *ml, const R *fine, R *coarse)
{
    if (dim == 2) {
        if (d % 2 == 1) SFX(rs2_axis_to_diag)(ml[d - 1], fine, coarse);
        else SFX(rs2_diag_to_axis)(ml[d - 1], fine, coarse);
    } else {
        if (d % 3 == 1) SFX(rs3_green_to_red)(ml[d - 1], fine, coarse);
        else if (d % 3 == 2) SFX(rs3_red_to_magenta)(ml[d - 1], fine, coarse);
        else SFX(rs3_magenta_to_blue)(ml[d - 1], fine, coarse);
    }
}

/* r <- r - A w on the axis (green) grid of side m and spacing s */
static void SFX(coarse_residual)(int dim, int m, double s, R *r, const R *w)
{
    R is2 = (R)(1.0 / (s * s));
    if (dim == 2) {
        for (int b = 1; b < m; b++)
            for (int a = 1; a < m; a++) {
                R lap = (w[I2(m, a - 1, b)] + w[I2(m, a, b - 1)] + w[I2(m, a + 1, b)] + w[I2(m, a, b + 1)]
                         - 4 * w[I2(m, a, b)]) * is2;
                r[I2(m, a, b)] = (R)(r[I2(m, a, b)] - lap);
            }
        return;
    }
    for (int k = 1; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m; i++) {
                R lap = (w[I3(m, i + 1, j, k)] + w[I3(m, i - 1, j, k)] + w[I3(m, i, j + 1, k)]
                         + w[I3(m, i, j - 1, k)] + w[I3(m, i, j, k + 1)] + w[I3(m, i, j, k - 1)]
                         - 6 * w[I3(m, i, j, k)]) * is2;
                r[I3(m, i, j, k)] = (R)(r[I3(m, i, j, k)] - lap);
            }
}

struct SFX(gen_state) {
    int dim, n, D, nu, gamma;
    const int *ml;
    const double *p;
    R **rl, **vl, **tsave_r, **tsave_v, **tq;
    R *vz;
};

static size_t SFX(gen_count)(int dim, int m)
{
    return dim == 2 ? (size_t)(m + 1) * (size_t)(m + 1) : SFX(vol3)(m);
}

/* the correction of level d (an axis / green level) for the residual rl[d] */
static void SFX(gen_group)(const struct SFX(gen_state) *S, int d)
{
    int dim = S->dim, g = dim;
    if (d < S->D) {
        for (int j = d + 1; j <= d + g; j++) SFX(restrict_step)(dim, j, S->ml, S->rl[j - 1], S->rl[j]);
        SFX(gen_group)(S, d + g);
        for (int k = 1; k < S->gamma; k++) {
            int c = d + g;
            size_t cnt = SFX(gen_count)(dim, S->ml[c]);
            memcpy(S->tsave_r[c], S->rl[c], cnt * sizeof(R));
            memcpy(S->tsave_v[c], S->vl[c], cnt * sizeof(R));
            SFX(coarse_residual)(dim, S->ml[c], (double)(S->n / S->ml[c]) / S->n, S->rl[c], S->vl[c]);
            SFX(gen_group)(S, c);
            for (size_t q = 0; q < cnt; q++) S->vl[c][q] = (R)(S->tsave_v[c][q] + S->vl[c][q]);
            memcpy(S->rl[c], S->tsave_r[c], cnt * sizeof(R));
        }
    }
    int top = d < S->D ? d + g - 1 : d;
    for (int j = top; j >= d; j--) {
        const R *vc = (j == S->D) ? S->vz : S->vl[j + 1];
        SFX(jac_step)(dim, S->n, j, S->ml, S->p, S->rl[j], vc, S->vl[j]);
        for (int s = 1; s < S->nu; s++) {
            SFX(again_input)(dim, j, S->ml[j], S->vl[j], vc, S->tq[j]);
            SFX(jac_step)(dim, S->n, j, S->ml, S->p, S->rl[j], S->tq[j], S->vl[j]);
        }
    }
}

/* One cycle with nu sweeps per level and gamma coarse visits per group (nu =
 * gamma = 1: the V-cycle above).  rtrace / vtrace as for the V-cycle (each
 * level's arrays as the cycle leaves them). */
static int SFX(cycle_gen)(int dim, int n, int order, const double *p, int nu, int gamma, double *u, const double *f,
                          double *rtrace, double *vtrace)
{
    int K = orc_log2(n);
    if (K < 1 || (dim != 2 && dim != 3) || nu < 1 || gamma < 1 || gamma > 2) return ORC_ERR_ARG;
    int D = (dim == 2) ? 2 * (K - 1) : 3 * (K - 1);
    R **rl = (R **)calloc((size_t)D + 1, sizeof(R *));
    R **vl = (R **)calloc((size_t)D + 1, sizeof(R *));
    R **t1 = (R **)calloc((size_t)D + 1, sizeof(R *));
    R **t2 = (R **)calloc((size_t)D + 1, sizeof(R *));
    R **tq = (R **)calloc((size_t)D + 1, sizeof(R *));
    int *ml = (int *)calloc((size_t)D + 1, sizeof(int));
    R *vz = (R *)calloc(27, sizeof(R));
    int rc = ORC_OK;
    if (!rl || !vl || !t1 || !t2 || !tq || !ml || !vz) { rc = ORC_ERR_ALLOC; goto done; }
    for (int d = 0; d <= D; d++) {
        ml[d] = n >> (d / dim);
        size_t cnt = SFX(gen_count)(dim, ml[d]);
        rl[d] = (R *)calloc(cnt, sizeof(R));
        vl[d] = (R *)calloc(cnt, sizeof(R));
        t1[d] = (R *)calloc(cnt, sizeof(R));
        t2[d] = (R *)calloc(cnt, sizeof(R));
        tq[d] = (R *)calloc(cnt, sizeof(R));
        if (!rl[d] || !vl[d] || !t1[d] || !t2[d] || !tq[d]) { rc = ORC_ERR_ALLOC; goto done; }
    }
    {
        size_t cnt = SFX(gen_count)(dim, n);
        double *r0 = (double *)malloc(cnt * sizeof(double));
        if (!r0) { rc = ORC_ERR_ALLOC; goto done; }
        orc_residual_ord_core(dim, n, order, u, f, r0);
        for (size_t q = 0; q < cnt; q++) rl[0][q] = (R)r0[q];
        free(r0);
        struct SFX(gen_state) S = {dim, n, D, nu, gamma, ml, p, rl, vl, t1, t2, tq, vz};
        SFX(gen_group)(&S, 0);
        for (size_t q = 0; q < cnt; q++) u[q] = u[q] + (double)vl[0][q];
    }
    if (rtrace || vtrace) {
        size_t off = 0;
        for (int d = 0; d <= D; d++) {
            size_t cnt = SFX(gen_count)(dim, ml[d]);
            for (size_t q = 0; q < cnt; q++) {
                if (rtrace) rtrace[off + q] = (double)rl[d][q];
                if (vtrace) vtrace[off + q] = (double)vl[d][q];
            }
            off += cnt;
        }
    }
done:
    if (rl && vl && t1 && t2 && tq)
        for (int d = 0; d <= D; d++) { free(rl[d]); free(vl[d]); free(t1[d]); free(t2[d]); free(tq[d]); }
    free(rl); free(vl); free(t1); free(t2); free(tq); free(ml); free(vz);
    return rc;
}

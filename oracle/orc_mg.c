/*
 * CPU oracle of the diagonally oriented multigrid V-cycle (A.J. Roberts,
 * "Fast and accurate multigrid solution of Poissons equation using
 * diagonally oriented grids", Sections 1-3).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, obviously correct C, double
 * precision, no blocking, fusion or reordering.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it; the GPU
 * library neither links nor calls it, and it shares no source with it.
 *
 * Interface: host pointers, natural (n+1)^dim arrays with x fastest,
 * zero Dirichlet boundary (boundary entries of u are read and never
 * written; boundary entries of f are ignored).  n = 2^K, K >= 1.
 * Return codes match the GPU library's numbering so tests can compare them.
 *
 * Parity pins live in tests/: closed-form sine-mode symbols of every
 * restriction and Jacobi half-sweep, a dense direct solve as the fixed
 * point, point counts, grid symmetries, and the paper's tabulated
 * convergence factors (Tables tbl:2d, tbl:3d, tbl:3dopt).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_OK = 0,
    ORC_ERR_ARG = -1,
    ORC_ERR_SIZE = -2,
    ORC_ERR_ALLOC = -4,
    ORC_ERR_NONFINITE = -6,
    ORC_ERR_DIVERGED = -7,
    ORC_ERR_NOT_CONVERGED = -8
};

static int orc_log2(int n)
{
    if (n < 2) return -1;
    int k = 0;
    while ((1 << k) < n) k++;
    return ((1 << k) == n) ? k : -1;
}

/* r = f - Lap_h(u) at interior nodes, 0 on the boundary (Eq. Evpois with
 * the 5-point / 7-point second-order Laplacian). */
static void orc_residual_core(int dim, int n, const double *u, const double *f, double *r)
{
    double h2 = (1.0 / n) * (1.0 / n);
    size_t s = (size_t)n + 1;
    if (dim == 2) {
        memset(r, 0, s * s * sizeof(double));
        for (int j = 1; j < n; j++)
            for (int i = 1; i < n; i++) {
                size_t c = (size_t)j * s + (size_t)i;
                double lap = (u[c - 1] + u[c - s] + u[c + 1] + u[c + s] - 4 * u[c]) / h2;
                r[c] = f[c] - lap;
            }
    } else {
        size_t s2 = s * s;
        memset(r, 0, s2 * s * sizeof(double));
        for (int k = 1; k < n; k++)
            for (int j = 1; j < n; j++)
                for (int i = 1; i < n; i++) {
                    size_t c = (size_t)k * s2 + (size_t)j * s + (size_t)i;
                    double lap = (u[c + 1] + u[c - 1] + u[c + s] + u[c - s] + u[c + s2] + u[c - s2]
                                  - 6 * u[c]) / h2;
                    r[c] = f[c] - lap;
                }
    }
}

/* sum of squares over interior nodes, natural order */
static double orc_interior_sumsq(int dim, int n, const double *a)
{
    size_t s = (size_t)n + 1;
    double acc = 0;
    if (dim == 2) {
        for (int j = 1; j < n; j++)
            for (int i = 1; i < n; i++) { double x = a[(size_t)j * s + i]; acc += x * x; }
    } else {
        for (int k = 1; k < n; k++)
            for (int j = 1; j < n; j++)
                for (int i = 1; i < n; i++) { double x = a[((size_t)k * s + j) * s + i]; acc += x * x; }
    }
    return acc;
}

#define R double
#define SFX(x) x
#include "orc_mg_body.h"
#undef R
#undef SFX
#undef I2
#undef I3

#define R float
#define SFX(x) x##_f32
#include "orc_mg_body.h"
#undef R
#undef SFX

static size_t orc_count(int dim, int n)
{
    size_t s = (size_t)n + 1;
    return dim == 2 ? s * s : s * s * s;
}

static int orc_check(int dim, int n)
{
    if (dim != 2 && dim != 3) return ORC_ERR_ARG;
    if (orc_log2(n) < 1) return ORC_ERR_SIZE;
    return ORC_OK;
}

int orc_residual(int dim, int n, const double *u, const double *f, double *r)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!u || !f || !r) return ORC_ERR_ARG;
    orc_residual_core(dim, n, u, f, r);
    return ORC_OK;
}

/* ||f - Lap_h u||_2 / ||f||_2 over interior nodes (||r||_2 when f = 0). */
int orc_relres(int dim, int n, const double *u, const double *f, double *out)
{
    int e = orc_check(dim, n);
    if (e) return e;
    double *r = (double *)malloc(orc_count(dim, n) * sizeof(double));
    if (!r) return ORC_ERR_ALLOC;
    orc_residual_core(dim, n, u, f, r);
    double rn = sqrt(orc_interior_sumsq(dim, n, r));
    double fn = sqrt(orc_interior_sumsq(dim, n, f));
    free(r);
    *out = fn > 0 ? rn / fn : rn;
    return ORC_OK;
}

/* prec 0: every level in double; prec 1: levels in single, the residual
 * and the update in double (iterative refinement). */
int orc_vcycle_trace(int dim, int n, const double *p, int prec, double *u, const double *f,
                     double *rtrace, double *vtrace)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!p || !u || !f || (prec != 0 && prec != 1)) return ORC_ERR_ARG;
    return prec == 0 ? vcycle(dim, n, p, u, f, rtrace, vtrace)
                     : vcycle_f32(dim, n, p, u, f, rtrace, vtrace);
}

int orc_vcycle(int dim, int n, const double *p, int prec, double *u, const double *f)
{
    return orc_vcycle_trace(dim, n, p, prec, u, f, NULL, NULL);
}

/* Outer iteration u <- u + v (Section 1): check the relative residual
 * before each cycle, stop once it is <= rtol or after max_cycles cycles.
 * history (nullable, max_cycles+1 entries): relative residual after
 * 0, 1, ... cycles.  A residual that grows for three cycles in a row and
 * exceeds the starting residual is reported as divergence (growth at the
 * rounding floor is not). */
int orc_solve(int dim, int n, const double *p, int prec, double *u, const double *f,
              double rtol, int max_cycles, int *cycles_out, double *relres_out, double *history)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!p || !u || !f || max_cycles < 0 || !(rtol >= 0)) return ORC_ERR_ARG;
    double rr;
    e = orc_relres(dim, n, u, f, &rr);
    if (e) return e;
    if (history) history[0] = rr;
    int k = 0, grow = 0;
    double prev = rr, rr0 = rr;
    int status = ORC_OK;
    while (!(rr <= rtol) && k < max_cycles) {
        if (!isfinite(rr)) { status = ORC_ERR_NONFINITE; break; }
        e = orc_vcycle(dim, n, p, prec, u, f);
        if (e) return e;
        k++;
        e = orc_relres(dim, n, u, f, &rr);
        if (e) return e;
        if (history) history[k] = rr;
        if (!isfinite(rr)) { status = ORC_ERR_NONFINITE; break; }
        grow = (rr > prev) ? grow + 1 : 0;
        prev = rr;
        if (grow >= 3 && rr > rr0) { status = ORC_ERR_DIVERGED; break; }
    }
    if (status == ORC_OK && !(rr <= rtol)) status = ORC_ERR_NOT_CONVERGED;
    if (cycles_out) *cycles_out = k;
    if (relres_out) *relres_out = rr;
    return status;
}

/* Single steps, for the tests that pin each equation on its own.
 * dim 2 restrict kind: 0 Eq. Erest2r (side m -> m), 1 Eq. Erest2b (m -> m/2).
 * dim 3 restrict kind: 0 Eq. Erred, 1 Eqs. Ermagc/Ermagm, 2 Eq. Erblu (m -> m/2).
 * dim 2 jacobi kind: 0 axis grid (coarse input side m), 1 diagonal grid
 *   (coarse input side m/2); c[0] the residual coefficient.
 * dim 3 jacobi kind: 0 green (input red, side m), 1 red (input magenta, side
 *   m; c[0], c[1]), 2 magenta (input blue, side m/2).  All in double. */
int orc_step_restrict(int dim, int kind, int m, const double *fine, double *coarse)
{
    if (orc_log2(m) < 1 || !fine || !coarse) return ORC_ERR_ARG;
    if (dim == 2 && kind == 0) rs2_axis_to_diag(m, fine, coarse);
    else if (dim == 2 && kind == 1) rs2_diag_to_axis(m, fine, coarse);
    else if (dim == 3 && kind == 0) rs3_green_to_red(m, fine, coarse);
    else if (dim == 3 && kind == 1) rs3_red_to_magenta(m, fine, coarse);
    else if (dim == 3 && kind == 2) rs3_magenta_to_blue(m, fine, coarse);
    else return ORC_ERR_ARG;
    return ORC_OK;
}

int orc_step_jacobi(int dim, int kind, int m, const double *c, const double *r, const double *vc,
                    double *v)
{
    if (orc_log2(m) < 1 || !c || !r || !vc || !v) return ORC_ERR_ARG;
    if (dim == 2 && kind == 0) jac2_axis(m, c[0], r, vc, v);
    else if (dim == 2 && kind == 1) jac2_diag(m, c[0], r, vc, v);
    else if (dim == 3 && kind == 0) jac3_green(m, c[0], r, vc, v);
    else if (dim == 3 && kind == 1) jac3_red(m, c[0], c[1], r, vc, v);
    else if (dim == 3 && kind == 2) jac3_magenta(m, c[0], r, vc, v);
    else return ORC_ERR_ARG;
    return ORC_OK;
}

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
 * restriction and Jacobi half-sweep and of the fourth-order residuals, a
 * dense direct solve as the fixed point, point counts, grid symmetries,
 * polynomial exactness and the fourth-order convergence of the Mehrstellen
 * schemes, and the paper's tabulated convergence factors (Tables tbl:2d,
 * tbl:3d, tbl:3dopt).
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

/* Fourth-order residual at interior nodes, 0 on the boundary: the compact
 * "Mehrstellen" scheme of Section 2.3, Eq. (Efos2), in 2D (the right-hand
 * side combination (8f + 4 neighbours)/12 minus the 9-point operator over
 * 6h^2) and the 19-point scheme of Section 3.3, Eq. (Efos4), in 3D
 * ((6f + 6 face neighbours)/12 minus the operator with weights -24 centre,
 * 2 faces, 1 edges, over 6h^2).  Reads f on boundary nodes too: the
 * right-hand side combination of a node next to the boundary includes them. */
static void orc_residual4_core(int dim, int n, const double *u, const double *f, double *r)
{
    double h2 = (1.0 / n) * (1.0 / n);
    size_t s = (size_t)n + 1;
    if (dim == 2) {
        memset(r, 0, s * s * sizeof(double));
        for (int j = 1; j < n; j++)
            for (int i = 1; i < n; i++) {
                size_t c = (size_t)j * s + (size_t)i;
                double rhs = (8 * f[c] + f[c + 1] + f[c + s] + f[c - 1] + f[c - s]) / 12;
                double op = (-20 * u[c] + 4 * (u[c - s] + u[c + s] + u[c - 1] + u[c + 1])
                             + u[c + 1 + s] + u[c - 1 + s] + u[c - 1 - s] + u[c + 1 - s]) / (6 * h2);
                r[c] = rhs - op;
            }
    } else {
        size_t s2 = s * s;
        memset(r, 0, s2 * s * sizeof(double));
        for (int k = 1; k < n; k++)
            for (int j = 1; j < n; j++)
                for (int i = 1; i < n; i++) {
                    size_t c = (size_t)k * s2 + (size_t)j * s + (size_t)i;
                    double rhs = (6 * f[c] + f[c + 1] + f[c + s] + f[c - 1] + f[c - s] + f[c + s2] + f[c - s2]) / 12;
                    double op = (-24 * u[c]
                                 + 2 * (u[c - s] + u[c + s] + u[c - 1] + u[c + 1] + u[c + s2] + u[c - s2])
                                 + u[c + 1 + s] + u[c - 1 + s] + u[c - 1 - s] + u[c + 1 - s]
                                 + u[c + s + s2] + u[c + s - s2] + u[c - s - s2] + u[c - s + s2]
                                 + u[c + 1 + s2] + u[c - 1 + s2] + u[c - 1 - s2] + u[c + 1 - s2]) / (6 * h2);
                    r[c] = rhs - op;
                }
    }
}

/* the finest residual of a cycle: order 2 (Eq. Evpois) or 4 (Eqs. Efos2 / Efos4) */
static void orc_residual_ord_core(int dim, int n, int order, const double *u, const double *f, double *r)
{
    if (order == 4) orc_residual4_core(dim, n, u, f, r);
    else orc_residual_core(dim, n, u, f, r);
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

int orc_residual_ord(int dim, int n, int order, const double *u, const double *f, double *r)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!u || !f || !r || (order != 2 && order != 4)) return ORC_ERR_ARG;
    orc_residual_ord_core(dim, n, order, u, f, r);
    return ORC_OK;
}

int orc_residual(int dim, int n, const double *u, const double *f, double *r)
{
    return orc_residual_ord(dim, n, 2, u, f, r);
}

/* ||r(u)||_2 / ||r(0)||_2 over interior nodes (||r(u)||_2 when r(0) = 0):
 * order 2, r = f - Lap_h u and r(0) = f; order 4, the residual of Eq. Efos2
 * / Efos4, whose r(0) is the right-hand side combination of f. */
int orc_relres_ord(int dim, int n, int order, const double *u, const double *f, double *out)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (order != 2 && order != 4) return ORC_ERR_ARG;
    size_t cnt = orc_count(dim, n);
    double *r = (double *)malloc(cnt * sizeof(double));
    if (!r) return ORC_ERR_ALLOC;
    orc_residual_ord_core(dim, n, order, u, f, r);
    double rn = sqrt(orc_interior_sumsq(dim, n, r));
    double fn;
    if (order == 2) {
        fn = sqrt(orc_interior_sumsq(dim, n, f));
    } else {
        double *z = (double *)calloc(cnt, sizeof(double));
        if (!z) { free(r); return ORC_ERR_ALLOC; }
        orc_residual4_core(dim, n, z, f, r);
        fn = sqrt(orc_interior_sumsq(dim, n, r));
        free(z);
    }
    free(r);
    *out = fn > 0 ? rn / fn : rn;
    return ORC_OK;
}

int orc_relres(int dim, int n, const double *u, const double *f, double *out)
{
    return orc_relres_ord(dim, n, 2, u, f, out);
}

/* prec 0: every level in double; prec 1: levels in single, the residual
 * and the update in double (iterative refinement).  order: 2, or 4 for the
 * fourth-order residual on the finest grid, the rest of the cycle unchanged
 * (Sections 2.3 and 3.3). */
int orc_vcycle_ord_trace(int dim, int n, const double *p, int prec, int order, double *u, const double *f,
                         double *rtrace, double *vtrace)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!p || !u || !f || (prec != 0 && prec != 1) || (order != 2 && order != 4)) return ORC_ERR_ARG;
    return prec == 0 ? vcycle(dim, n, order, p, u, f, rtrace, vtrace)
                     : vcycle_f32(dim, n, order, p, u, f, rtrace, vtrace);
}

int orc_vcycle_trace(int dim, int n, const double *p, int prec, double *u, const double *f,
                     double *rtrace, double *vtrace)
{
    return orc_vcycle_ord_trace(dim, n, p, prec, 2, u, f, rtrace, vtrace);
}

int orc_vcycle(int dim, int n, const double *p, int prec, double *u, const double *f)
{
    return orc_vcycle_ord_trace(dim, n, p, prec, 2, u, f, NULL, NULL);
}

/* Outer iteration u <- u + v (Section 1): check the relative residual
 * before each cycle, stop once it is <= rtol or after max_cycles cycles.
 * history (nullable, max_cycles+1 entries): relative residual after
 * 0, 1, ... cycles.  A residual that grows for three cycles in a row and
 * exceeds the starting residual is reported as divergence (growth at the
 * rounding floor is not).  `cycle` runs one cycle of the chosen scheme. */
typedef int (*orc_cycle_fn)(const void *ctx, double *u, const double *f);

static int orc_solve_loop(int dim, int n, int order, double *u, const double *f, double rtol, int max_cycles,
                          int *cycles_out, double *relres_out, double *history, orc_cycle_fn cycle, const void *ctx)
{
    double rr;
    int e = orc_relres_ord(dim, n, order, u, f, &rr);
    if (e) return e;
    if (history) history[0] = rr;
    int k = 0, grow = 0;
    double prev = rr, rr0 = rr;
    int status = ORC_OK;
    while (!(rr <= rtol) && k < max_cycles) {
        if (!isfinite(rr)) { status = ORC_ERR_NONFINITE; break; }
        e = cycle(ctx, u, f);
        if (e) return e;
        k++;
        e = orc_relres_ord(dim, n, order, u, f, &rr);
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

struct orc_cycle_args {
    int dim, n, prec, order;
    const double *p;
};

static int orc_diag_cycle(const void *ctx, double *u, const double *f)
{
    const struct orc_cycle_args *a = (const struct orc_cycle_args *)ctx;
    return orc_vcycle_ord_trace(a->dim, a->n, a->p, a->prec, a->order, u, f, NULL, NULL);
}

int orc_solve_ord(int dim, int n, const double *p, int prec, int order, double *u, const double *f,
                  double rtol, int max_cycles, int *cycles_out, double *relres_out, double *history)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!p || !u || !f || max_cycles < 0 || !(rtol >= 0) || (order != 2 && order != 4)) return ORC_ERR_ARG;
    struct orc_cycle_args a = {dim, n, prec, order, p};
    return orc_solve_loop(dim, n, order, u, f, rtol, max_cycles, cycles_out, relres_out, history, orc_diag_cycle, &a);
}

/* The conventional comparison cycle (Sections 2.1-2.3, 3.1-3.3): one
 * parameter p (2D) / p_g (3D) scaling the residual term of every Jacobi
 * iteration; prec and order as for the diagonal cycle. */
int orc_vcycle_usual(int dim, int n, double p, int prec, int order, double *u, const double *f, double *rtrace,
                     double *vtrace)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!u || !f || !(p > 0) || (prec != 0 && prec != 1) || (order != 2 && order != 4)) return ORC_ERR_ARG;
    return prec == 0 ? vcycle_usual(dim, n, order, p, u, f, rtrace, vtrace)
                     : vcycle_usual_f32(dim, n, order, p, u, f, rtrace, vtrace);
}

static int orc_usual_cycle(const void *ctx, double *u, const double *f)
{
    const struct orc_cycle_args *a = (const struct orc_cycle_args *)ctx;
    return orc_vcycle_usual(a->dim, a->n, a->p[0], a->prec, a->order, u, f, NULL, NULL);
}

int orc_solve_usual(int dim, int n, double p, int prec, int order, double *u, const double *f, double rtol,
                    int max_cycles, int *cycles_out, double *relres_out, double *history)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!u || !f || !(p > 0) || max_cycles < 0 || !(rtol >= 0) || (order != 2 && order != 4)) return ORC_ERR_ARG;
    struct orc_cycle_args a = {dim, n, prec, order, &p};
    return orc_solve_loop(dim, n, order, u, f, rtol, max_cycles, cycles_out, relres_out, history, orc_usual_cycle, &a);
}

int orc_solve(int dim, int n, const double *p, int prec, double *u, const double *f,
              double rtol, int max_cycles, int *cycles_out, double *relres_out, double *history)
{
    return orc_solve_ord(dim, n, p, prec, 2, u, f, rtol, max_cycles, cycles_out, relres_out, history);
}

/* More Jacobi sweeps per level (nu >= 1) and W-cycles (gamma = 2) on the
 * diagonal hierarchy, the two directions Section 4 leaves to further
 * research (readings in orc_mg_body.h); nu = gamma = 1 is the V-cycle. */
int orc_cycle_gen(int dim, int n, const double *p, int prec, int order, int nu, int gamma, double *u, const double *f,
                  double *rtrace, double *vtrace)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!p || !u || !f || (prec != 0 && prec != 1) || (order != 2 && order != 4) || nu < 1 || nu > 16 ||
        gamma < 1 || gamma > 2)
        return ORC_ERR_ARG;
    return prec == 0 ? cycle_gen(dim, n, order, p, nu, gamma, u, f, rtrace, vtrace)
                     : cycle_gen_f32(dim, n, order, p, nu, gamma, u, f, rtrace, vtrace);
}

struct orc_gen_args {
    struct orc_cycle_args c;
    int nu, gamma;
};

static int orc_gen_cycle(const void *ctx, double *u, const double *f)
{
    const struct orc_gen_args *a = (const struct orc_gen_args *)ctx;
    return orc_cycle_gen(a->c.dim, a->c.n, a->c.p, a->c.prec, a->c.order, a->nu, a->gamma, u, f, NULL, NULL);
}

int orc_solve_gen(int dim, int n, const double *p, int prec, int order, int nu, int gamma, double *u,
                  const double *f, double rtol, int max_cycles, int *cycles_out, double *relres_out, double *history)
{
    int e = orc_check(dim, n);
    if (e) return e;
    if (!p || !u || !f || max_cycles < 0 || !(rtol >= 0) || (order != 2 && order != 4) || nu < 1 || nu > 16 ||
        gamma < 1 || gamma > 2)
        return ORC_ERR_ARG;
    struct orc_gen_args a = {{dim, n, prec, order, p}, nu, gamma};
    return orc_solve_loop(dim, n, order, u, f, rtol, max_cycles, cycles_out, relres_out, history, orc_gen_cycle, &a);
}

/* Single steps, for the tests that pin each equation on its own.
 * dim 2 restrict kind: 0 Eq. Erest2r (side m -> m), 1 Eq. Erest2b (m -> m/2).
 * dim 3 restrict kind: 0 Eq. Erred, 1 Eqs. Ermagc/Ermagm, 2 Eq. Erblu (m -> m/2).
 * dim 2 jacobi kind: 0 axis grid (coarse input side m), 1 diagonal grid
 *   (coarse input side m/2); c[0] the residual coefficient.
 * dim 3 jacobi kind: 0 green (input red, side m), 1 red (input magenta, side
 *   m; c[0], c[1]), 2 magenta (input blue, side m/2).
 * The conventional cycle: restrict kind 2 (dim 2) / 3 (dim 3) is the full
 *   weighting (m -> m/2); jacobi kind 2 (dim 2) / 3 (dim 3) interpolates the
 *   coarse correction (side m/2) and runs one red-black iteration.
 * All in double. */
int orc_step_restrict(int dim, int kind, int m, const double *fine, double *coarse)
{
    if (orc_log2(m) < 1 || !fine || !coarse) return ORC_ERR_ARG;
    if (dim == 2 && kind == 0) rs2_axis_to_diag(m, fine, coarse);
    else if (dim == 2 && kind == 1) rs2_diag_to_axis(m, fine, coarse);
    else if (dim == 3 && kind == 0) rs3_green_to_red(m, fine, coarse);
    else if (dim == 3 && kind == 1) rs3_red_to_magenta(m, fine, coarse);
    else if (dim == 3 && kind == 2) rs3_magenta_to_blue(m, fine, coarse);
    else if (dim == 2 && kind == 2) rs2_full(m, fine, coarse);
    else if (dim == 3 && kind == 3) rs3_full(m, fine, coarse);
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
    else if ((dim == 2 && kind == 2) || (dim == 3 && kind == 3)) {
        interp_lin(dim, m, vc, v);
        rbj_cubic(dim, m, c[0], r, v);
    }
    else return ORC_ERR_ARG;
    return ORC_OK;
}

/*
 * dmg.h -- C ABI of libdmg, a diagonally oriented multigrid V-cycle for the
 * discrete Poisson equation on MI355X (gfx950).
 *
 * Method: A.J. Roberts, "Fast and accurate multigrid solution of Poissons
 * equation using diagonally oriented grids" (arXiv math/9907190).
 *   2D (Section 2): grids alternate between axis-aligned and 45-degree
 *   rotated (spacings h, sqrt2 h, 2h, ...); restriction Eqs. (Erest2r),
 *   (Erest2b); red-black Jacobi prolongation with over-relaxation p,
 *   Eqs. (Eajacr), (Eajacb) (Section 2.4).
 *   3D (Section 3): cubic -> FCC -> BCC -> cubic of twice the spacing;
 *   restrictions Eqs. (Erred), (Ermagc), (Ermagm), (Erblu); Jacobi steps
 *   Eqs. (Emprolm)-(Egprolr) with parameters p_m, p_r1, p_r2, p_g.
 *   One V-cycle (Section 1, Eq. Evpois): r = f - Lap_h(u) with the 5-point or
 *   7-point Laplacian, restrict down to the coarsest grid (3^dim nodes, one
 *   interior node), one Jacobi iteration per level back up (the coarsest one
 *   from a zero correction), u <- u + v.
 *
 * Problem: Lap_h u = f on the unit square / cube, n intervals per side
 * (h = 1/n, n = 2^K, 2 <= n <= 2^15 in 2D, 2^11 in 3D), zero Dirichlet data.
 *
 * Memory: u and f are DEVICE pointers to (n+1)^dim doubles in natural order,
 * x fastest (index ((z*(n+1) + y)*(n+1) + x)).  Boundary entries of u are
 * read and never written (the iteration keeps them); boundary entries of f
 * are ignored.  The caller owns u, f and the device workspace; the library
 * allocates no device memory.  An mg_plan is host memory owned by the
 * library (mg_setup allocates it, mg_destroy frees it).
 *
 * Streams: every call enqueues its work on the HIP stream given to
 * mg_setup (NULL = the default stream) and returns once that work is
 * enqueued, except mg_solve, which synchronises that stream to read the
 * residual history.  A plan is bound to one stream and one device and is
 * not thread-safe; distinct plans with distinct workspaces are independent.
 *
 * Errors: every function returns MG_OK (0) or a negative MG_ERR_* code;
 * mg_strerror names it.  On an argument error nothing is enqueued.
 */
#ifndef DMG_H
#define DMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MG_OK = 0,
    MG_ERR_ARG = -1,            /* null pointer, bad dim / precision / parameter count */
    MG_ERR_SIZE = -2,           /* n not a power of two in the supported range */
    MG_ERR_WS = -3,             /* workspace null, misaligned (256 B) or too small */
    MG_ERR_ALLOC = -4,          /* host allocation failed */
    MG_ERR_HIP = -5,            /* a HIP runtime call failed */
    MG_ERR_NONFINITE = -6,      /* residual norm became NaN or Inf */
    MG_ERR_DIVERGED = -7,       /* residual grew 3 cycles in a row and exceeds the initial one */
    MG_ERR_NOT_CONVERGED = -8,  /* max_cycles reached; cycles and residual still returned */
    MG_ERR_SCRATCH = -9         /* mg_vcycle_static: the problem needs more than MG_STATIC_SCRATCH_BYTES */
};

enum {
    MG_FP64 = 0,          /* every level in double */
    MG_FP32_REFINED = 1   /* levels in single; r = f - Lap_h(u) and u += v in double
                             (iterative refinement, u and f stay double) */
};

/* Flag OR-ed into `precision` of mg_workspace_bytes / mg_setup (a batch of
 * one in mg_setup_batched): the finest residual is the fourth-order compact
 * ("Mehrstellen") scheme, and the rest of the cycle is unchanged.
 *   2D, Section 2.3, Eq. (Efos2):
 *     r = (8f + f_E + f_N + f_W + f_S)/12
 *         - (-20u + 4(u_S + u_N + u_W + u_E) + u_NE + u_NW + u_SW + u_SE)/(6h^2);
 *   3D, Section 3.3, Eq. (Efos4): r = (6f + the 6 face neighbours of f)/12
 *     - (-24u + 2 (the 6 face neighbours) + the 12 edge neighbours)/(6h^2).
 * The right-hand side combination is made once per mg_solve / mg_vcycle call
 * into the workspace (which grows by (n+1)^dim doubles); boundary entries of
 * f are then read too.  The relative residual becomes ||r(u)||_2 / ||r(0)||_2.
 * The paper tunes p = 1.20 (2D, Section 2.4) and (p_m, p_r1, p_r2, p_g) =
 * (0.91, 0.80, 0.70, 1.77) (3D, Section 3.4) for this residual; a
 * fourth-order solution is reached fastest after second-order cycles (two
 * plans on the same u, Sections 2.3 and 3.3).  Another precision value with
 * this flag, or a batch of more than one problem: MG_ERR_ARG. */
enum { MG_ORDER4 = 0x100 };

/* Flag OR-ed into `precision` of mg_workspace_bytes / mg_setup: the
 * conventional V-cycle the paper compares its diagonal grids with (Sections
 * 2.1-2.3 and 3.1-3.3; Tables tbl:2d, tbl:3d, tbl:3dopt, rows "usual") on
 * the standard hierarchy of grids of spacing h, 2h, 4h, ... down to one
 * interior node: the nine-point (2D) / 27-point (3D) full-weighting
 * restriction (weights 4, 2, 1 over 16; 8, 4, 2, 1 over 64), and on the way
 * up bilinear / trilinear interpolation of the coarse correction followed
 * by one Jacobi iteration of Lap v = r in red-black order (the points with
 * an odd index sum first, then the even ones from the new odd values), with
 * one parameter on the residual term: np = 1 in 2D and 3D (p; the paper
 * tunes 1.121 in 2D and p_g = 1.30 in 3D, 1.216 / 1.70 with MG_ORDER4).
 * Levels: depth d = 0 .. log2(n) - 1 of side n >> d, natural arrays (for
 * mg_level_get).  Combines with MG_FP64 / MG_FP32_REFINED and MG_ORDER4;
 * single problems only (mg_setup), no learned correction, no two-stage
 * solve (MG_ERR_ARG). */
enum { MG_USUAL = 0x200 };

typedef struct mg_plan mg_plan;

/* Bytes of device workspace mg_setup needs for (dim, n, precision). */
int mg_workspace_bytes(int dim, int n, int precision, size_t *bytes);

/* Build a plan.  p: over-relaxation parameters, np = 1 in 2D (p, Section
 * 2.4; the paper's tuned value is 1.052) and np = 4 in 3D (p_m, p_r1, p_r2,
 * p_g, Section 3.4; tuned 1.11, 1.42, 1.08, 0.99).  workspace: device
 * memory of at least mg_workspace_bytes bytes, 256-byte aligned, used only
 * by this plan until mg_destroy.  hip_stream: a hipStream_t or NULL.
 * Enqueues the zeroing of the workspace on the stream. */
int mg_setup(mg_plan **out, int dim, int n, int precision, const double *p, int np,
             void *workspace, size_t ws_bytes, void *hip_stream);

/* One V-cycle in place on u (Section 1).  rel_res_before (host, nullable):
 * receives ||f - Lap_h u||_2 / ||f||_2 over interior nodes for the u on
 * entry (||r||_2 if f = 0); passing it synchronises the stream. */
int mg_vcycle(mg_plan *plan, double *u, const double *f, double *rel_res_before);

/* Solve of Lap_h u = f (Section 1, Eq. Evpois: each cycle computes the
 * correction v of the residual equation Lap_h v = f - Lap_h u and sets
 * u <- u + v).  Outer iteration u <- u + v until the relative residual is <= rtol or
 * max_cycles (0 .. 1000) cycles have run; the residual is checked before
 * every cycle.  cycles_out, rel_res_out (host, nullable).  history (host,
 * nullable, max_cycles+1 doubles): relative residual after 0, 1, ...
 * cycles.  Returns MG_OK, MG_ERR_NOT_CONVERGED, MG_ERR_NONFINITE or
 * MG_ERR_DIVERGED (the last three still fill the outputs).  Synchronises
 * the stream.  A 2D second-order plan of one problem, n >= 128, FP64 or
 * MG_FP32_REFINED (mg_setup), runs the cycles out of place: the iterates
 * alternate between u and a workspace array, u holds the result when the call
 * returns, and u's boundary values are read, never written.  Its finest
 * kernel also forms the next residual evaluation (the relative residuals then
 * equal the in-place path's to rounding: the norm's partial sums are grouped
 * differently); with the environment variable DMG_NO_FUSED_RESIDUAL=1 at
 * mg_setup the residual kernel runs after each cycle instead. */
int mg_solve(mg_plan *plan, double *u, const double *f, double rtol, int max_cycles,
             int *cycles_out, double *rel_res_out, double *history);

/* Fourth-order solution in two stages (Sections 2.3 and 3.3): mg_solve on
 * `first` (a plan without MG_ORDER4) until its relative residual is <= rtol1,
 * then mg_solve on `second` (the same dim and n, with MG_ORDER4) on the same u
 * until the fourth-order relative residual is <= rtol; each stage at most
 * max_cycles cycles.  cycles1, cycles2, rel_res_out (host, nullable): the
 * cycles of each stage and the final fourth-order relative residual (the
 * first stage's if it failed).  Returns the second stage's status, or the
 * first stage's if that one failed with another code than
 * MG_ERR_NOT_CONVERGED (the second stage then does not run).  Mismatched or
 * batched plans: MG_ERR_ARG.  Synchronises both plans' streams. */
int mg_solve_two_stage(mg_plan *first, mg_plan *second, double *u, const double *f, double rtol1, double rtol,
                       int max_cycles, int *cycles1, int *cycles2, double *rel_res_out);

/* Cycles with more Jacobi sweeps per level and W-cycles on the diagonal
 * hierarchy, the two directions the paper leaves to further research
 * (Section 4).  nu (1 .. 8): red-black iterations per level on the way up,
 * the first as in the V-cycle, each further one the same step with the
 * level's own values, at the points it shares with the level below, as the
 * coarse input (the red level's step keeps the magenta cube centres).
 * gamma (1 or 2): visits of each group's coarse correction (2D: axis ->
 * diagonal -> axis of twice the stride; 3D: green -> red -> magenta ->
 * blue); the second visit corrects the residual of the coarse axis (green)
 * grid's own equation, r - A w with its 5-/7-point Laplacian, and its
 * correction is added to w.  nu = gamma = 1 is the V-cycle (with one launch
 * per level step instead of the fused kernels of mg_setup).  Other
 * arguments, the use with mg_vcycle / mg_solve / mg_level_get /
 * mg_timing_*, and mg_destroy as for mg_setup; no learned correction, no
 * batching, no two-stage solve (MG_ERR_ARG).  Extra workspace: each level's
 * further-sweep input (nu > 1), a finest-size correction array (nu > 1),
 * and a saved residual and correction per coarse axis / green level
 * (gamma = 2). */
int mg_cycle_workspace_bytes(int dim, int n, int precision, int nu, int gamma, size_t *bytes);
int mg_setup_cycle(mg_plan **out, int dim, int n, int precision, const double *p, int np, int nu, int gamma,
                   void *workspace, size_t ws_bytes, void *hip_stream);

/* Copy level `depth` of the last cycle into dst (device, (m+1)^dim doubles,
 * natural order, m = the level's side in units of its stride; points not on
 * the level and boundary points read 0).  which = 0: restricted residual
 * r (depth 0 .. D); which = 1: correction v (depth 1 .. D; the finest
 * correction is added to u and not kept).  Some diagonal levels' Jacobi runs
 * inside the kernel of the axis level above them, which does not store their
 * correction (2D: depth 1 for finest sides >= 128; in a single-problem plan
 * also the odd depths whose aligned level is >= 15).  which = 1 recomputes
 * such a level (same arithmetic, same values) from its residual and the
 * next coarser correction, so it is the last cycle's only right after
 * mg_vcycle (mg_solve ends with a fresh residual).  After an out-of-place
 * mg_solve (see there) the finest residual is not stored: depths 0 and 1
 * return MG_ERR_ARG until the next mg_vcycle.  For parity tests. */
int mg_level_get(mg_plan *plan, int depth, int which, double *dst);

/* Number of levels D+1 and the side m of level `depth` (host-only). */
int mg_level_info(int dim, int n, int depth, int *num_levels, int *side);

/* Batched 2D solve.  nprob independent problems on the unit square, problem
 * i with n[i] intervals per side (a power of two, 2 .. 2^15), all with the
 * same over-relaxation p (Section 2.4).  The hierarchies are aligned from the
 * coarsest grid, where every level of the same aligned index has the same
 * side whatever the problem's size, so one kernel launch per level serves the
 * whole batch; a converged problem's work returns at once.  One outer
 * iteration is captured in a hipGraph and replayed.  u and f are HOST arrays
 * of nprob DEVICE pointers, each to (n[i]+1)^2 doubles laid out as for
 * mg_solve.  The plan is used with mg_solve_batched / mg_vcycle_batched (and
 * with mg_solve / mg_vcycle when nprob = 1), mg_autotune, mg_destroy. */
int mg_batch_workspace_bytes(int nprob, const int *n, int precision, size_t *bytes);
int mg_setup_batched(mg_plan **out, int nprob, const int *n, int precision, double p,
                     void *workspace, size_t ws_bytes, void *hip_stream);
/* Per problem (host arrays of nprob, nullable): cycles run, final relative
 * residual, status (MG_OK / MG_ERR_NOT_CONVERGED / MG_ERR_NONFINITE /
 * MG_ERR_DIVERGED).  Returns MG_OK when every problem converged, else the
 * most negative per-problem status.  Synchronises the stream. */
int mg_solve_batched(mg_plan *plan, double *const *u, const double *const *f, double rtol,
                     int max_cycles, int *cycles, double *rel_res, int *status);
/* One V-cycle of every problem; rel_res_before (host, nprob, nullable). */
int mg_vcycle_batched(mg_plan *plan, double *const *u, const double *const *f, double *rel_res_before);

/* Tile autotuner (2D plans): times every candidate launch shape (one thread
 * per point, or row strips of 4..32 rows per wavefront) of every level
 * launch of the cycle on the plan's own arrays and keeps the fastest.  If
 * the environment variable DMG_TUNE_CACHE names a file, results are appended
 * to it and later plans read them at setup.  Enqueues and synchronises work
 * on the plan's stream; the workspace's level arrays are overwritten. */
int mg_autotune(mg_plan *plan);

/* Measurement.  Kernel families of one cycle: */
enum {
    MG_K_RESIDUAL = 0,  /* finest residual r = f - Lap_h(u) and its norm partials */
    MG_K_RESTRICT = 1,  /* one restriction step per launch (all levels above the coarse part) */
    MG_K_JACOBI = 2,    /* one Jacobi step per launch (levels between the finest and the coarse part) */
    MG_K_FINEST = 3,    /* finest Jacobi step fused with u += v */
    MG_K_COARSE = 4,    /* persistent kernel running every coarse level */
    MG_K_NORM = 5,      /* norm finalisation and the stopping decision */
    MG_K_FAMILIES = 6
};
/* Bracket every later launch of kernel family `family` (-1: none) on the
 * plan's stream with HIP events.  mg_timing_read synchronises those events
 * and returns, since the previous read: the summed kernel duration in ms,
 * the number of launches, and their summed algorithmic HBM bytes (each
 * array element a launch must read or write, counted once). */
int mg_timing_enable(mg_plan *plan, int family);
int mg_timing_read(mg_plan *plan, double *ms, long long *launches, double *bytes);

/* ------------------------------------------------------------------------
 * Learned coarse correction (an extension; the paper has no learned part).
 *
 * A network of four convolutions with 16 channels, 3x3 taps in 2D and 3x3x3
 * in 3D, ReLU after the first three, no bias, zero padding, acting on one
 * grid of the cut level: aligned level MG_NET_CUT, the axis grid of side 16
 * (17 x 17 points) in 2D and the cubic grid of side 8 (9^3 points) in 3D.
 * It maps the cut level's restricted residual r_c to an estimate of the
 * exact correction e_c = A_c^{-1} r_c (A_c: the 5-point / 7-point Laplacian
 * of that level, the equation Section 1 solves for v), replacing the
 * restrictions and Jacobi steps of every coarser level.  bf16 weights and
 * activations with fp32 accumulation; FP32 master weights.
 *
 * Weights: host float arrays of mg_net_weight_count(dim) entries, layout
 * [layer 4][tap][c_in 16][c_out 16], tap = (dy+1)*3 + (dx+1) in 2D and
 * ((dz+1)*3 + (dy+1))*3 + (dx+1) in 3D; layer 0 reads channel 0 only and
 * layer 3 writes channel 0 only (the other entries are forced to 0).
 *
 * Normalisation: with s = rms of r_c over interior points and H = 1/(G-1)
 * the cut level's spacing, the network sees r_c / s and its output y
 * stands for the correction y s H^2.
 */
#define MG_NET_CUT 6

typedef struct mg_net mg_net;

int mg_net_weight_count(int dim);  /* 9216 (2D) or 27648 (3D); 0 for another dim */

/* Trainer state: master weights, Adam moments, bf16 copies and the
 * per-sample gradient buffers of up to max_batch samples, all in the
 * caller's device workspace (256-byte aligned). */
int mg_net_workspace_bytes(int dim, int max_batch, size_t *bytes);
int mg_net_create(mg_net **out, int dim, int max_batch, void *workspace, size_t ws_bytes,
                  void *hip_stream);
/* Set (host array; resets Adam) / read the FP32 master weights; He-normal
 * initialisation from a seed.  Synchronise the stream. */
int mg_net_set_weights(mg_net *net, const float *w);
int mg_net_get_weights(mg_net *net, float *w);
int mg_net_init(mg_net *net, unsigned long long seed);
/* Inference on `batch` grids (device, batch x G^dim doubles each, natural
 * order, boundary ignored; out's boundary is written 0).  normalize = 1
 * applies the normalisation above (out = the correction estimate);
 * normalize = 0 returns the raw network output for the raw input. */
int mg_net_forward(mg_net *net, const double *in, double *out, int batch, int normalize);
/* Mean-squared-error loss over the interior points of `batch` samples
 * (batch <= max_batch) and its gradient with respect to the weights (host,
 * nullable, mg_net_weight_count floats; the padded entries are 0), from the
 * bf16 forward and backward kernels.  With normalize = 1 the target is
 * scaled like the output.  Synchronises the stream. */
int mg_net_loss_grad(mg_net *net, const double *in, const double *target, int batch, int normalize,
                     float *grad, double *loss);
/* Training objective of mg_net_loss_grad and mg_net_train.
 * MG_NET_LOSS_MSE (the default): the mean squared error above.
 * MG_NET_LOSS_CUT: what the plan's judge compares.  The output at the cut
 * level's points with even index sum (those it shares with the level below)
 * goes through the cut level's red-black Jacobi step for Lap v = x
 * (Section 2.2; over-relaxed form of Section 2.4 with parameter pj, the
 * cut level's p: 2D p, 3D p_g), odd points first, in the normalised units
 * (x = r_c / s, spacing 1); the loss is the mean over interior points of
 * (x - Lap v)^2, the square of the cut level's residual reduction.  The
 * target is not read and may be NULL.  pj in (0, 1000); MG_ERR_ARG
 * otherwise.  The setting stays until changed. */
#define MG_NET_LOSS_MSE 0
#define MG_NET_LOSS_CUT 1
int mg_net_set_loss(mg_net *net, int kind, double pj);
/* Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) on npairs normalised
 * (r_c, e_c) pairs (device, npairs x G^dim doubles each), `epochs` passes
 * of npairs / batch steps; the order of every pass is a seeded permutation.
 * epoch_loss (host, nullable, `epochs` doubles): mean batch loss of each
 * pass.  Synchronises the stream. */
int mg_net_train(mg_net *net, const double *r, const double *e, int npairs, int epochs, int batch,
                 float lr, unsigned long long seed, double *epoch_loss);
int mg_net_destroy(mg_net *net);

/* Use a trained network in a plan's cycles (w: host weights as above, NULL
 * removes it; cut_level must be MG_NET_CUT).  Every problem that has the
 * cut level below its finest grid then runs, per cycle, the network
 * instead of the levels below the cut.  The plain sub-cycle is the judge:
 * on the first cycle of a solve both run and the plain one's reduction of
 * the cut level's residual, ||r_c - A_c v_c|| / ||r_c||, becomes the bar;
 * a cycle where the network does worse than the bar (or worse than the
 * plain sub-cycle on the first cycle) takes the plain correction instead,
 * and the network stays off for the rest of that solve. */
int mg_set_coarse_net(mg_plan *plan, const float *w, int cut_level);
/* Per problem, for the last solve or cycle (host arrays of nprob,
 * nullable): cycles whose coarse correction came from the network; 1 where
 * the judge switched the network off; and the first cycle's cut-level
 * residual reductions ||r_c - A_c v_c|| / ||r_c|| with the network's and
 * with the plain sub-cycle's correction (0 where the problem has no level
 * below the cut or no network is set).  Synchronises the stream. */
int mg_net_stats(mg_plan *plan, int *net_cycles, int *fell_back, double *q_net, double *q_plain);
/* Copy the restricted residual of aligned level `level` (0 .. the cut
 * level) of every problem, as left by the last cycle, into dst (device,
 * nprob x G^dim doubles, G = the level's side + 1; problems without that
 * level read 0).  For generating training pairs. */
int mg_coarse_export(mg_plan *plan, int level, double *dst);

int mg_destroy(mg_plan *plan);
const char *mg_strerror(int code);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * V-cycle in place on u, as mg_setup + mg_vcycle would run it, with the
 * workspace taken from a device array inside the library instead of the
 * caller's memory.  The call allocates nothing: no hipMalloc, hipHostMalloc
 * or hipFree, no event, stream or graph; the array is zeroed and the plan's
 * tables are written into it by kernels on hip_stream (host bookkeeping for
 * the call is a few hundred bytes of ordinary host memory).
 *
 * dim, n, precision (MG_FP64 or MG_FP32_REFINED, optionally | MG_ORDER4),
 * p, np, u, f, rel_res_before: as for mg_setup and mg_vcycle (u, f device
 * pointers on the current device; rel_res_before host, nullable, and when
 * given the call synchronises hip_stream).  hip_stream: a stream of the
 * current device, or NULL.
 *
 * The array holds MG_STATIC_SCRATCH_BYTES (64 MiB) on every device the
 * library runs on, from the first call there until the process ends.
 * Problems whose workspace is larger return MG_ERR_SCRATCH and enqueue
 * nothing.  That workspace is mg_workspace_bytes, except for 2D
 * MG_FP32_REFINED, where it is (n+1)^2 * 4 bytes less: the cycle here runs
 * in place, without the second double iterate of mg_solve's out-of-place
 * cycles; 64 MiB covers 2D n <= 1024 in every
 * precision (n = 2048 with single-precision levels) and 3D n <= 128
 * (second-order residual).  Every call on one device uses the same array
 * and leaves its contents behind; the next call zeroes it first.  Calls
 * that overlap on one device (two host threads, or two streams whose work
 * runs concurrently) race on the array and give wrong results: serialise
 * them. */
#define MG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int mg_vcycle_static(int dim, int n, int precision, const double *p, int np, double *u, const double *f,
                     double *rel_res_before, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* DMG_H */

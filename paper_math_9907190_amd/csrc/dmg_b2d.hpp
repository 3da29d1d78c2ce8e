// Work items of the 2D kernels.  Every 2D launch processes a list of
// independent problems: blockIdx.y (point kernels: blockIdx.z) selects the
// item, so one launch per level serves a whole batch, and a single problem
// is a batch of one.  Levels are aligned from the coarsest grid: at aligned
// level lambda every problem's grid has the same side and kind, whatever its
// finest size.
#pragma once
#include "dmg_common.hpp"

namespace dmg {

// one problem's arrays at one level
template <typename T>
struct Item2 {
    T* r;          // residual of this level (restriction output, Jacobi input)
    T* v;          // correction of this level (Jacobi output)
    const T* in;   // restriction: residual of the finer level; Jacobi: correction of the coarser level
    int prob;      // problem index: ctl[prob].done skips the item
    int pad;
};

// one problem's arrays for the Jacobi of an axis level L run together with
// that of the diagonal level L-1 below it
template <typename T>
struct JPair2 {
    const T* rA;   // residual of level L (level L-1's is restricted from it on the fly)
    const T* v2;   // correction of level L-2
    T* vA;         // correction of level L (output; level L-1's is not stored)
    int prob;
    int pad;
};

// one problem's arrays for the restrictions from an axis level L to L-1
// and on to L-2 in one launch
template <typename T>
struct RsPair2 {
    const T* rA;   // residual of level L
    T* r2;         // residual of level L-2 (output; level L-1's is not stored)
    int prob;
    int pad;
};

// one problem's finest-level arrays
template <typename T>
struct Fin2 {
    double* u;
    const double* f;
    T* r0;         // finest residual (natural layout)
    T* r1;         // residual of the first diagonal level (written by the unfused residual only)
    const T* v1;   // correction of the first diagonal level (or a zero array)
    const T* v2;   // correction of the level below it (read when the finest kernel runs its Jacobi)
    T* r2;         // residual of that level (written by the residual kernel when fused)
    double* part;  // norm partial sums of this problem
    double* partf; // partial sums of f^2 (first evaluation of a solve, made by the residual kernel)
    double* ub;    // out-of-place solves: the second iterate buffer ((n+1)^2 doubles), else null
    int prob;
    int pad;
};

// one problem's coarse levels (aligned levels 0 .. top, side <= the coarse limit)
constexpr int kCoarseLevels = 12;
template <typename T>
struct Coarse2B {
    T* r[kCoarseLevels];
    T* v[kCoarseLevels];
    int top;       // highest aligned level run by the coarse kernel (-1: none)
    int prob;
};

// per aligned level (the same for every problem at that level)
template <typename T>
struct LevInfo {
    int m;
    int diag;
    T c;
};

// fused = 1: the kernel also restricts r1 onto the axis level below it (r2)
// withf: also the partial sums of f^2 (into partf), for finalize kind 2
// oop (fused FP64 single problems with ub set): out-of-place solve step: the
// residual of the iterate of evaluation k (the control block's count: u for
// even k, ub for odd k) is formed, restricted and summed but not stored
template <typename T>
void launch_b_resid(int n, int fused, int order, const Fin2<T>* items, int nitems, const Ctl* ctls, hipStream_t s,
                    int withf = 0, int oop = 0);
// order 4: f of the items is the right-hand side combination made by launch_b_rhs4
void launch_b_rhs4(int n, const double* f, double* g, hipStream_t s);
int b_resid_parts(int n);
// fused = 1: the kernel also runs the Jacobi of the first diagonal level
// (coefficient c1) from r1 and v2 instead of reading v1
// oop (fused, FP64, one item with ub set): the kernel of cycle k forms the
// finest residual from the iterate of cycle k-1 and f itself and writes the
// new iterate into the other buffer (cycle k writes u for even k, ub for odd k)
template <typename T>
void launch_b_finest(int n, T c, T c1, int fused, const Fin2<T>* items, int nitems, const Ctl* ctls, hipStream_t s,
                     int oop = 0);
// The out-of-place step (one problem, fused, n >= 8) that also forms
// the residual of the iterate it writes, its norm partials (nparts of them,
// as the residual kernel's) and its restriction onto the level below the
// first diagonal one, as the residual kernel would for the next evaluation.
// b_finest_res_fits: whether its grid has at most nparts blocks (else the
// separate residual kernel stays in use).
template <typename T>
bool b_finest_res_fits(int n, int nparts);
template <typename T>
void launch_b_finest_res(int n, T c, T c1, const Fin2<T>* items, const Ctl* ctls, int nparts, hipStream_t s);
// the boundary entries of an (n+1)^2 array: dst <- src (src null: zeros)
void launch_b_copy_ring(int n, const double* src, double* dst, hipStream_t s);
// end of an out-of-place solve (ctl: the problem's control block, done set)
void launch_b_oop_finish(int n, const Ctl* ctl, double* ub, double* u, hipStream_t s);
// does a problem with finest level D run the first diagonal level's Jacobi in
// the finest kernel, and the restriction into the level below it (D-2) in
// the residual kernel (when both levels are above the coarse kernel's top lamc)
inline bool fin_fused(int D, int lamc) { return D - 2 >= lamc; }
// In single-problem plans (pairs = true), axis levels L = kPairLow,
// kPairLow+2, ... below the finest (L <= D-2) run their Jacobi together with
// that of level L-1 (launch_b_jac_pair), and the restrictions from L into L-1
// and L-2 run in one launch (launch_b_rs_pair).  Batches keep the autotuned
// per-level launches there (measured faster for the Jacobi steps).
constexpr int kPairLow = 16;
inline bool pair_level(int L, int D, bool pairs) { return pairs && !(L & 1) && L >= kPairLow && L <= D - 2; }
template <typename T>
void launch_b_jac_pair(int m, T cc, T cd, const JPair2<T>* items, int nitems, const Ctl* ctls, hipStream_t s);
template <typename T>
void launch_b_rs_pair(int m, const RsPair2<T>* items, int nitems, const Ctl* ctls, hipStream_t s);
template <typename T>
void launch_b_restrict(int diag_in, int m, int rows, const Item2<T>* items, int nitems, const Ctl* ctls,
                       hipStream_t s);
template <typename T>
void launch_b_jacobi(int diag, int m, int rows, T c, const Item2<T>* items, int nitems, const Ctl* ctls,
                     hipStream_t s);
template <typename T>
// top_cap: highest level the coarse kernel runs (below each item's top)
void launch_b_coarse(const LevInfo<T>* lev, const Coarse2B<T>* items, int nitems, const T* zero, const Ctl* ctls,
                     hipStream_t s, int top_cap = kCoarseLevels);
// sum of f^2 over interior nodes per problem, into the problem's partials (b_resid_parts(n) of them)
template <typename T>
void launch_b_sumsq(int n, const Fin2<T>* items, int nitems, const Ctl* ctls, hipStream_t s);
// host (pinned host memory, single-item launches only): receives, for kind
// 1 and 2 in a solve, the decision (done, status, cycles), the relative
// residual (last) and its entry of hist
template <typename T>
void launch_b_finalize(int kind, const Fin2<T>* items, int nitems, int nparts, Ctl* ctls, int* nactive,
                       hipStream_t s, Ctl* host = nullptr);
void launch_b_ctl_reset(Ctl* ctls, int nprob, int mode, int max_cycles, double rtol, int* nactive, int net,
                        hipStream_t s);
// the coarse kernel with the learned correction at the cut level (wf: packed forward weights)
template <typename T>
void launch_b_coarse_net(const LevInfo<T>* lev, const Coarse2B<T>* items, int nitems, const T* zero, Ctl* ctls,
                         const unsigned short* wf, hipStream_t s, int top_cap = kCoarseLevels);
// A single problem's aligned levels 14 .. 9 (sides 256 .. 64) in one launch
// each way: restriction r14 -> r13 .. r8 (r[k]: level 8 + k); Jacobi from
// v8 up to v9 .. v14 (r[k], v[k], c[k]: level 9 + k).  The coarse kernel
// then runs levels 8 .. 0 only.  Needs n >= 512.
constexpr int kMidTop = 14, kMidLow = 10, kMidCoarseTop = 8;
static_assert(kPairLow == kMidTop + 2, "Jacobi pairs start right above the fused mid levels");
template <typename T>
void launch_b_mid_down(const T* r14, T* const* r, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_b_mid_up(const T* v8, const T* const* r, T* const* v, const T* c, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_b_coarse_export(int lam, int diag, int m, const Coarse2B<T>* items, int nitems, double* dst, hipStream_t s);
template <typename T>
void launch_b_level_get(int diag, int m, const T* src, double* dst, hipStream_t s);
// default strip length of a row-marching launch (0: use the one-thread-per-point kernel)
int b_default_rows(int kind, int m);

}  // namespace dmg

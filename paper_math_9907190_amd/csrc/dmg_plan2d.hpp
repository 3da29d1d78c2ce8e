// The 2D plan (a batch of independent problems; one problem is a batch of one).
#pragma once
#include "dmg_host.hpp"

#include <vector>

namespace dmg {

struct Plan2 {
    int nprob = 0, prec = 0;
    int rorder = 2;           // finest residual: 2 (Eq. Evpois) or 4 (Eq. Efos2; single problem)
    size_t off_g = 0;         // order 4: the right-hand side combination of f, (n+1)^2 doubles
    double p = 1.0;
    std::vector<int> n, D;    // per problem: intervals per side, finest depth (= its finest aligned level)
    int Dmax = 0, lamc = 0;   // highest aligned level; highest level run by the coarse kernel
    // size classes (distinct n, ascending); the finest-item table is grouped by class
    std::vector<int> order, cls_n, cls_first, cls_count, nparts;
    // workspace offsets
    size_t off_ctl = 0, off_nactive = 0, off_zero = 0, off_fin = 0, off_coarse = 0, off_net = 0, off_lg_item = 0, total = 0;
    bool has_net = false;     // learned coarse correction set (packed bf16 weights at off_net)
    // single FP64 second-order problem with the fused finest kernels: solves
    // update u out of place, alternating between u and the finest residual's
    // array (which they then do not store); r0_stale: it holds an iterate
    bool oop = false, r0_stale = false;
    std::vector<size_t> off_r0, off_part, off_partf;
    std::vector<std::vector<size_t>> off_r, off_v;   // [problem][aligned level]
    std::vector<size_t> off_rs_items, off_jac_items; // [aligned level]
    std::vector<int> n_rs_items, n_jac_items;
    bool pairs = false;                              // Jacobi pairs in use (single problem)
    std::vector<size_t> off_pair_items;              // [aligned level L]: Jacobi pairs (L, L-1)
    std::vector<int> n_pair_items;
    std::vector<size_t> off_rsp_items;               // [aligned level L]: restrictions L -> L-1 -> L-2
    std::vector<int> n_rsp_items;
    int n_coarse_items = 0;
    std::vector<int> rows_rs, rows_jac;              // launch shape per level (0: one thread per point)
    // runtime
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    void* hfin = nullptr;     // pinned host image of the finest-item table
    Ctl* hctl = nullptr;      // pinned: problem 0's control block (a single problem's solve: written by its finalize kernel)
    int* hact = nullptr;      // pinned: active-problem counts of two iterations
    char* hres = nullptr;     // pinned: the first kCtlHead bytes of every control block
    hipEvent_t ev[2];
    hipEvent_t evu;           // completion of the last finest-table upload (hfin is then free to rewrite)
    bool evs = false, fin_valid = false;
    std::vector<const void*> last_u, last_f;
    Timing tm;
    hipGraphExec_t gexec = nullptr;
    bool gready = false, use_graph = true;
    bool res = false;   // out of place: the finest kernel also forms the next residual
    hipStream_t cap = nullptr;
    // bound by plan2_bind_static: no pinned host memory, events or graph; the
    // tables are written by stream-ordered kernels
    bool stat = false;
    std::vector<unsigned char> stage;   // static binding: host image of the tables, by workspace offset
    size_t stage_lo = 0;                // lowest offset written into stage
};

// allow_oop = false: no out-of-place solves (plans that only run cycles)
int plan2_layout(Plan2& P, int nprob, const int* n, int prec, double p, bool allow_oop = true);
int plan2_setup(Plan2& P, void* ws, size_t ws_bytes, hipStream_t stream);
void plan2_destroy(Plan2& P);
// Single problem: bind the laid-out plan to workspace ws (P.total bytes,
// 256-byte aligned) on `stream` without allocating anything: the workspace
// is zeroed by a fill kernel and the item tables are written by kernels, all
// in stream order.  Then only plan2_vcycle may be called; nothing to destroy.
int plan2_bind_static(Plan2& P, void* ws, hipStream_t stream);
int plan2_vcycle(Plan2& P, double* const* u, const double* const* f, double* relres);
int plan2_solve(Plan2& P, double* const* u, const double* const* f, double rtol, int max_cycles, int* cycles,
                double* relres, int* status, double* history0);
int plan2_level_get(Plan2& P, int depth, int which, double* dst);
int plan2_tune_load(Plan2& P);
int plan2_autotune(Plan2& P);
int plan2_set_net(Plan2& P, const float* w, int cut_level);
int plan2_net_stats(Plan2& P, int* net_cycles, int* fell_back, double* q_net, double* q_plain);
int plan2_coarse_export(Plan2& P, int level, double* dst);

}  // namespace dmg

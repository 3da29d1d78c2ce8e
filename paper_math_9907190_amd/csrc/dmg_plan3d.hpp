// The 3D plan (one problem).
#pragma once
#include "dmg_host.hpp"

namespace dmg {

constexpr int kMaxLev3 = 32;  // 3D n <= 2^11 has 31 levels

struct Level3 {
    int m = 0;
    int kind = 0;           // 0 green, 1 red, 2 magenta
    size_t r = 0, v = 0;    // byte offsets; magenta: corner (E) arrays
    size_t r2 = 0, v2 = 0;  // magenta: cube-centre (O) arrays
    double c = 0, c2 = 0;   // Jacobi residual coefficients
};

struct Plan3 {
    int n = 0, prec = 0, D = 0, dc = 0;
    int rorder = 2;           // finest residual: 2 (Eq. Evpois) or 4 (Eq. Efos4)
    size_t g = 0;             // order 4: the right-hand side combination of f, (n+1)^3 doubles
    double p[4] = {1, 1, 1, 1};
    size_t ctl = 0, partial = 0, zero = 0, r0 = 0, net = 0, total = 0;
    bool has_net = false;   // learned coarse correction set (packed bf16 weights at net)
    int nparts = 0;         // norm partials of ||f|| (and of the residual when not fused)
    int nparts_res = 0;     // norm partials of the residual
    bool fused_resid = false;   // residual fused with the first restriction (n >= 128)
    Level3 lev[kMaxLev3];
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    Ctl* hctl = nullptr;
    HostState* hstate = nullptr;   // pinned: written by the finalize kernel of a solve
    bool live = false;   // set up: destroy synchronises the stream before freeing the pinned state
    Timing tm;
};

int plan3_layout(Plan3& P, int n, int prec, const double* p);
int plan3_setup(Plan3& P, void* ws, size_t ws_bytes, hipStream_t stream);
void plan3_destroy(Plan3& P);
// Bind the laid-out plan to workspace ws (P.total bytes, 256-byte aligned) on
// `stream` without allocating anything (the workspace is zeroed by a fill
// kernel in stream order).  Then only plan3_vcycle may be called; nothing to
// destroy.
int plan3_bind_static(Plan3& P, void* ws, hipStream_t stream);
int plan3_vcycle(Plan3& P, double* u, const double* f, double* relres);
int plan3_solve(Plan3& P, double* u, const double* f, double rtol, int max_cycles, int* cycles, double* relres,
                double* history);
int plan3_level_get(Plan3& P, int depth, int which, double* dst);
int plan3_set_net(Plan3& P, const float* w, int cut_level);
int plan3_net_stats(Plan3& P, int* net_cycles, int* fell_back, double* q_net, double* q_plain);
int plan3_coarse_export(Plan3& P, int level, double* dst);

}  // namespace dmg

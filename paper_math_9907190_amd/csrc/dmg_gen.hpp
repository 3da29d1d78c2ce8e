// The generalised diagonal cycle: nu red-black sweeps per level and gamma
// visits of the coarse correction per group of levels (gamma = 2: W-cycle),
// the directions Section 4 leaves to further research.  Plan and entry points.
#pragma once
#include "dmg_host.hpp"

namespace dmg {

constexpr int kMaxLevG = 32;   // 2D n <= 2^15: 29 levels; 3D n <= 2^11: 31

struct LevelG {
    int m = 0;
    size_t r = 0, v = 0;      // residual and correction (2D: A or D layout; 3D: G, R, or magenta corners)
    size_t r2 = 0, v2 = 0;    // 3D magenta cube centres
    size_t tq = 0, tq2 = 0;   // the coarse input of a further sweep on this level (the next level's layout)
    size_t sr = 0, sv = 0;    // W-cycle: saved residual and correction of a group's coarse axis / green level
    double c = 0, c2 = 0;     // Jacobi coefficients as in the V-cycle
};

struct PlanG {
    int dim = 2, n = 0, prec = 0, rorder = 2, D = 0, nu = 1, gamma = 1;
    double p[4] = {1, 1, 1, 1};
    size_t ctl = 0, partial = 0, zero = 0, r0 = 0, g = 0, v0 = 0, total = 0;
    int nparts = 0;
    LevelG lev[kMaxLevG];
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    Ctl* hctl = nullptr;
    HostState* hstate = nullptr;
    bool live = false;   // set up: destroy synchronises the stream before freeing the pinned state
    Timing tm;
};

int plang_layout(PlanG& P, int dim, int n, int prec, const double* p, int nu, int gamma);
int plang_setup(PlanG& P, void* ws, size_t ws_bytes, hipStream_t stream);
void plang_destroy(PlanG& P);
int plang_vcycle(PlanG& P, double* u, const double* f, double* relres);
int plang_solve(PlanG& P, double* u, const double* f, double rtol, int max_cycles, int* cycles, double* relres,
                double* history);
int plang_level_get(PlanG& P, int depth, int which, double* dst);

}  // namespace dmg

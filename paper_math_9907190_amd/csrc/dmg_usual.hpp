// The conventional comparison V-cycle (Roberts, Sections 2.1-2.3 and 3.1-3.3)
// on the standard hierarchy of axis-aligned grids: plan and launchers.
#pragma once
#include "dmg_host.hpp"

namespace dmg {

constexpr int kMaxLevU = 16;   // n <= 2^15: levels of side n, n/2, ..., 2

struct PlanU {
    int dim = 2, n = 0, prec = 0, rorder = 2, D = 0;   // levels d = 0 .. D, side n >> d
    double p = 1.0;
    size_t ctl = 0, partial = 0, zero = 0, r0 = 0, g = 0, total = 0;
    size_t r[kMaxLevU] = {}, v[kMaxLevU] = {};          // d >= 1 (the finest correction goes into u)
    double c[kMaxLevU] = {};                             // Jacobi coefficient p (2^d h)^2
    int nparts = 0;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    Ctl* hctl = nullptr;
    HostState* hstate = nullptr;
    bool live = false;   // set up: destroy synchronises the stream before freeing the pinned state
    Timing tm;
};

int planu_layout(PlanU& P, int dim, int n, int prec, double p);
int planu_setup(PlanU& P, void* ws, size_t ws_bytes, hipStream_t stream);
void planu_destroy(PlanU& P);
int planu_vcycle(PlanU& P, double* u, const double* f, double* relres);
int planu_solve(PlanU& P, double* u, const double* f, double rtol, int max_cycles, int* cycles, double* relres,
                double* history);
int planu_level_get(PlanU& P, int depth, int which, double* dst);

}  // namespace dmg

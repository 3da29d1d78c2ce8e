// Host-side launchers of the libdmg kernels (one declaration per kernel
// family; definitions and explicit instantiations live in the .hip files).
#pragma once
#include "dmg_common.hpp"

namespace dmg {

constexpr int kMaxLev = 32;  // 2D n <= 2^15 has 29 levels, 3D n <= 2^11 has 31

// One 2D level as the coarse persistent kernel sees it.
template <typename T>
struct Lev2 {
    int m;      // side in units of the level's stride
    int diag;   // 1: diagonal grid (D layout), 0: axis grid (A layout)
    T* r;
    T* v;
    T c;        // Jacobi residual coefficient: p*(sigma h)^2 (axis) or 2p*(sigma h)^2 (diagonal)
};

template <typename T>
struct Coarse2 {
    int first, last;      // depths handled: restriction first+1..last, Jacobi last..first
    Lev2<T> lev[kMaxLev]; // indexed by depth
    T* zeroD;             // zero coarse correction for the coarsest Jacobi
};

// residual r = f - Lap_h u on the finest grid (5- or 7-point), written as T
// into r0 (natural layout), per-block partial sums of r^2 (double) in partial.
template <typename T>
void launch_residual(int dim, int n, const double* u, const double* f, T* r0, double* partial, int nparts,
                     const Ctl* ctl, hipStream_t s);
int residual_parts(int dim, int n);

void launch_sumsq(int dim, int n, const double* a, double* partial, int nparts, const Ctl* ctl, hipStream_t s);
// finalize: kind 0 -> ||f|| into ctl->fnorm; kind 1 -> relative residual of evaluation k
void launch_finalize(int kind, int k, const double* partial, int nparts, Ctl* ctl, hipStream_t s);
void launch_ctl_reset(Ctl* ctl, int mode, int max_cycles, double rtol, hipStream_t s);

template <typename T>
void launch_rs2(int diag_in, int m, const T* in, T* out, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_jac2(int diag, int m, T c, const T* r, const T* vc, T* v, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_jac2_finest(int n, T c, const T* r0, const T* vD, double* u, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_coarse2(const Coarse2<T>& a, const Ctl* ctl, hipStream_t s);

// level -> natural double array (parity tests)
template <typename T>
void launch_level_get2(int diag, int m, const T* src, double* dst, hipStream_t s);

}  // namespace dmg

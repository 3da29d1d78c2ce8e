// Host-side launchers of the single-problem residual / norm kernels (used
// by the 3D plan); definitions in dmg_util.hip.
#pragma once
#include "dmg_common.hpp"

namespace dmg {

// residual r = f - Lap_h u on the finest grid (5- or 7-point), written as T
// into r0 (natural layout), per-block partial sums of r^2 (double) in partial.
// order 4: f holds the right-hand side combination of the fourth-order scheme
// (Eqs. Efos2 / Efos4) and the operator is the 9- / 19-point one.
template <typename T>
void launch_residual(int dim, int n, const double* u, const double* f, T* r0, double* partial, int nparts,
                     const Ctl* ctl, hipStream_t s, int order = 2);
int residual_parts(int dim, int n);

void launch_sumsq(int dim, int n, const double* a, double* partial, int nparts, const Ctl* ctl, hipStream_t s);
// finalize: kind 0 -> ||f|| into ctl->fnorm; kind 1 -> relative residual of evaluation k
// host (pinned, nullable): receives done and the relative residual after each kind-1 evaluation
void launch_finalize(int kind, const double* partial, int nparts, Ctl* ctl, hipStream_t s, HostState* host = nullptr);
void launch_ctl_reset(Ctl* ctl, int mode, int max_cycles, double rtol, hipStream_t s, int net = 0);

// Stream-ordered set-up of a workspace without host copies: zero `bytes`
// (a multiple of 16) at dst; copy `bytes` (a multiple of 4) of host data to
// dst through the arguments of small kernels (the host data may be reused
// as soon as the call returns).
struct PutWords {
    unsigned w[960];   // 3840 bytes per launch, inside the kernel-argument limit
};
void launch_zero(void* dst, size_t bytes, hipStream_t s);
void launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace dmg

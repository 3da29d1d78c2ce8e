// The generalised diagonal cycle (2D and 3D, one problem): nu red-black
// sweeps per level on the way up and gamma visits of the coarse correction
// per group of levels (2D: axis -> diagonal -> axis of twice the stride; 3D:
// green -> red -> magenta -> blue), the two directions Section 4 of the paper
// leaves to further research.  Readings:
//  * a further sweep on a level is the same two-colour step with the
//    level's own values, at the points it shares with the level below, as
//    the coarse input (the red level keeps the magenta cube centres, which
//    are not red points);
//  * after the first visit of a group's coarse correction returns w, the
//    second visit solves for the residual of the coarse axis (green) grid's
//    own equation, r - A w (5-/7-point Laplacian of that grid's spacing),
//    and its correction is added to w.
// nu = gamma = 1 is the V-cycle.  Every level step is one launch (no fused
// levels): the point arithmetic is the V-cycle's (the 2D point functions of
// dmg_common.hpp, the 3D level kernels of dmg_k3d.hip), so a level gets the
// same values as in the V-cycle kernels; the coarse input of a further sweep
// is copied into a buffer of its own, so every level's arrays end the cycle
// as the CPU reference leaves them.
#include "dmg_b2d.hpp"
#include "dmg_gen.hpp"
#include "dmg_launch.hpp"
#include "dmg_launch3.hpp"

#include <algorithm>
#include <string.h>

namespace dmg {

namespace {

// --------------------------------------------------------------- 2D kernels
// one thread per point of a row, one row per blockIdx.y

template <typename T>
__global__ void __launch_bounds__(256) kg2_rs_a2d(int m, const T* __restrict__ rA, T* __restrict__ rD,
                                                  const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int b = blockIdx.y + 1;
    const int a = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x) + (b & 1);
    if (a < 1 || a > m - 1) return;
    rD[idxD(m, a, b)] = rs2_a2d(rA, m, a, b);
}

template <typename T>
__global__ void __launch_bounds__(256) kg2_rs_d2a(int m, const T* __restrict__ rD, T* __restrict__ rA2,
                                                  const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int B = blockIdx.y + 1, A = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (A > m / 2 - 1) return;
    rA2[idxA(m / 2, A, B)] = rs2_d2a(rD, m, A, B);
}

// axis level of side m from the diagonal level of the same side (vD); both
// colours in one launch (the second colour recomputes its four first-colour
// neighbours).  FINEST: u += v.
template <typename T, bool FINEST>
__global__ void __launch_bounds__(256) kg2_jac_axis(int m, T c, const T* __restrict__ rA, const T* __restrict__ vD,
                                                    T* __restrict__ vA, double* __restrict__ u,
                                                    const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int b = blockIdx.y + 1, a = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (a > m - 1) return;
    const T val = ((a + b) & 1) ? jac2_axisF(rA, vD, m, c, a, b) : jac2_axisC(rA, vD, m, c, a, b);
    const size_t o = idxA(m, a, b);
    if constexpr (FINEST) u[o] = u[o] + (double)val;
    else vA[o] = val;
}

// diagonal level of side m from the axis level of side m/2 (vA2)
template <typename T>
__global__ void __launch_bounds__(256) kg2_jac_diag(int m, T c, const T* __restrict__ rD, const T* __restrict__ vA2,
                                                    T* __restrict__ vD, const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int b = blockIdx.y + 1;
    const int a = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x) + (b & 1);
    if (a < 1 || a > m - 1) return;
    vD[idxD(m, a, b)] = (b & 1) ? jac2_diagF(rD, vA2, m, c, a, b) : jac2_diagC(rD, vA2, m, c, a, b);
}

// the coarse input of a further sweep: an axis level's even points in the
// diagonal layout; a diagonal level's (even, even) points as the axis level
// of half the side (boundary entries included: they are 0 on both)
template <typename T>
__global__ void __launch_bounds__(256) kg2_again_axis(int m, const T* __restrict__ vA, T* __restrict__ vD,
                                                      const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int b = blockIdx.y;
    const int a = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x) + (b & 1);
    if (a > m) return;
    vD[idxD(m, a, b)] = vA[idxA(m, a, b)];
}

template <typename T>
__global__ void __launch_bounds__(256) kg2_again_diag(int m, const T* __restrict__ vD, T* __restrict__ vA2,
                                                      const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int B = blockIdx.y, A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A > m / 2) return;
    vA2[idxA(m / 2, A, B)] = vD[idxD(m, 2 * A, 2 * B)];
}

// --------------------------------------------------------------- 3D copies

// a green level's red points (a+b+c even) in the red layout of the same side
template <typename T>
__global__ void __launch_bounds__(256) kg3_again_green(int m, const T* __restrict__ vG, T* __restrict__ vR,
                                                       const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int b = blockIdx.y, c = blockIdx.z;
    const int a = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x) + ((b + c) & 1);
    if (a > m) return;
    vR[idxR(m, a, b, c)] = vG[idxG(m, a, b, c)];
}

// a red level's corners (all indices even) as the magenta corner array
template <typename T>
__global__ void __launch_bounds__(256) kg3_again_red(int m, const T* __restrict__ vR, T* __restrict__ vE,
                                                     const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int B = blockIdx.y, C = blockIdx.z, A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A > m / 2) return;
    vE[idxME(m, 2 * A, 2 * B, 2 * C)] = vR[idxR(m, 2 * A, 2 * B, 2 * C)];
}

// ------------------------------------------------------------ W-cycle steps

// r <- r - A w on the axis (green) grid of side m, is2 = 1 / (sigma h)^2, in
// the CPU reference's order
template <typename T>
__global__ void __launch_bounds__(256) kg_wres(int dim, int m, T is2, T* __restrict__ r, const T* __restrict__ w,
                                               const Ctl* __restrict__ ctl)
{
#pragma clang fp contract(off)
    if (ctl->done) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x + 1, b = blockIdx.y + 1, c = blockIdx.z + 1;
    if (a > m - 1) return;
    const size_t s = (size_t)m + 1;
    if (dim == 2) {
        const size_t o = (size_t)b * s + a;
        const T lap = (w[o - 1] + w[o - s] + w[o + 1] + w[o + s] - 4 * w[o]) * is2;
        r[o] = r[o] - lap;
        return;
    }
    const size_t s2 = s * s, o = (size_t)c * s2 + (size_t)b * s + a;
    const T lap = (w[o + 1] + w[o - 1] + w[o + s] + w[o - s] + w[o + s2] + w[o - s2] - 6 * w[o]) * is2;
    r[o] = r[o] - lap;
}

// v <- save + v (the first visit's correction plus the second's)
template <typename T>
__global__ void __launch_bounds__(256) kg_add(size_t count, const T* __restrict__ save, T* __restrict__ v,
                                              const Ctl* __restrict__ ctl)
{
#pragma clang fp contract(off)
    if (ctl->done) return;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (size_t)gridDim.x * blockDim.x)
        v[q] = save[q] + v[q];
}

// ------------------------------------------------------------------- plan

template <typename T>
T* at(PlanG& P, size_t off) { return reinterpret_cast<T*>(P.ws + off); }

size_t cnt2(int m, bool diag) { return diag ? sizeD(m) : sizeA(m); }

size_t level_elems(const PlanG& P, int d)
{
    const int m = P.lev[d].m;
    if (P.dim == 2) return cnt2(m, d & 1);
    const int t = d % 3;
    return t == 0 ? sizeG(m) : t == 1 ? sizeR(m) : sizeME(m);
}

template <typename T>
struct CycleG {
    PlanG& P;
    const Ctl* ctl;
    hipStream_t s;
    size_t es = sizeof(T);

    T* R(int d) { return d == 0 ? at<T>(P, P.r0) : at<T>(P, P.lev[d].r); }
    T* V(int d) { return at<T>(P, P.lev[d].v); }

    Lev3<T> lv(int d, bool again = false)
    {
        const LevelG& q = P.lev[d];
        Lev3<T> x;
        x.m = q.m;
        x.kind = d % 3;
        x.r = R(d);
        x.v = d == 0 ? at<T>(P, P.v0) : V(d);
        x.r2 = x.kind == 2 ? at<T>(P, q.r2) : nullptr;
        x.v2 = x.kind == 2 ? at<T>(P, q.v2) : nullptr;
        x.c = (T)q.c;
        x.c2 = (T)q.c2;
        (void)again;
        return x;
    }

    void restrict_into(int d)   // level d-1 -> level d
    {
        Timed t(&P.tm, MG_K_RESTRICT, es * (double)(level_elems(P, d - 1) + level_elems(P, d)));
        const int mf = P.lev[d - 1].m;
        if (P.dim == 2) {
            if (d & 1)
                hipLaunchKernelGGL(kg2_rs_a2d<T>, dim3((mf / 2 + 1 + 255) / 256, mf - 1), dim3(256), 0, s, mf, R(d - 1),
                                   R(d), ctl);
            else if (mf / 2 >= 2)
                hipLaunchKernelGGL(kg2_rs_d2a<T>, dim3((mf / 2 - 1 + 255) / 256, mf / 2 - 1), dim3(256), 0, s, mf,
                                   R(d - 1), R(d), ctl);
            return;
        }
        launch_rs3<T>(lv(d - 1), lv(d), ctl, s);
    }

    // one sweep of level d with coarse input (2D: vc; 3D: Lev3 whose v / v2 are read); last: the final sweep
    // of the finest level, which adds into u
    void sweep(int d, const T* vc, const Lev3<T>& cr, double* u, bool finest_last)
    {
        const LevelG& q = P.lev[d];
        const int m = q.m;
        Timed t(&P.tm, d == 0 && finest_last ? MG_K_FINEST : MG_K_JACOBI, es * 3.0 * (double)level_elems(P, d));
        if (P.dim == 2) {
            if (d & 1) {
                hipLaunchKernelGGL(kg2_jac_diag<T>, dim3((m / 2 + 1 + 255) / 256, m - 1), dim3(256), 0, s, m, (T)q.c,
                                   R(d), vc, V(d), ctl);
            } else if (d == 0 && finest_last) {
                hipLaunchKernelGGL((kg2_jac_axis<T, true>), dim3((m - 1 + 255) / 256, m - 1), dim3(256), 0, s, m,
                                   (T)q.c, R(0), vc, (T*)nullptr, u, ctl);
            } else {
                hipLaunchKernelGGL((kg2_jac_axis<T, false>), dim3((m - 1 + 255) / 256, m - 1), dim3(256), 0, s, m,
                                   (T)q.c, R(d), vc, d == 0 ? at<T>(P, P.v0) : V(d), (double*)nullptr, ctl);
            }
            return;
        }
        if (d == 0 && finest_last) {
            launch_jac3_finest<T>(P.n, (T)q.c, R(0), cr.v ? cr.v : at<T>(P, P.zero), u, ctl, s);
            return;
        }
        launch_jac3<T>(lv(d), cr, at<T>(P, P.zero), ctl, s);
    }

    // the coarse input of a further sweep of level d, into its tq buffers
    void again_input(int d)
    {
        const LevelG& q = P.lev[d];
        const int m = q.m;
        T* v = d == 0 ? at<T>(P, P.v0) : V(d);
        Timed t(&P.tm, MG_K_JACOBI, es * 2.0 * (double)level_elems(P, d + 1));
        if (P.dim == 2) {
            if (d & 1)
                hipLaunchKernelGGL(kg2_again_diag<T>, dim3((m / 2 + 1 + 255) / 256, m / 2 + 1), dim3(256), 0, s, m, v,
                                   at<T>(P, q.tq), ctl);
            else
                hipLaunchKernelGGL(kg2_again_axis<T>, dim3((m / 2 + 1 + 255) / 256, m + 1), dim3(256), 0, s, m, v,
                                   at<T>(P, q.tq), ctl);
            return;
        }
        const int k = d % 3;
        if (k == 0) {
            hipLaunchKernelGGL(kg3_again_green<T>, dim3((m / 2 + 1 + 255) / 256, m + 1, m + 1), dim3(256), 0, s, m, v,
                               at<T>(P, q.tq), ctl);
        } else if (k == 1) {   // the magenta centres as handed up, the red level's corners
            const LevelG& mg = P.lev[d + 1];
            (void)hipMemcpyAsync(at<T>(P, q.tq2), at<T>(P, mg.v2), es * sizeMO(m), hipMemcpyDeviceToDevice, s);
            hipLaunchKernelGGL(kg3_again_red<T>, dim3((m / 2 + 1 + 255) / 256, m / 2 + 1, m / 2 + 1), dim3(256), 0, s,
                               m, v, at<T>(P, q.tq), ctl);
        } else {               // the magenta corners are the blue grid's layout
            (void)hipMemcpyAsync(at<T>(P, q.tq), v, es * sizeME(m), hipMemcpyDeviceToDevice, s);
        }
    }

    Lev3<T> tq_lev(int d)
    {
        Lev3<T> x;
        x.v = at<T>(P, P.lev[d].tq);
        x.v2 = P.lev[d].tq2 ? at<T>(P, P.lev[d].tq2) : nullptr;
        return x;
    }

    // the correction of level d (an axis / green level) for its residual
    void group(int d, double* u)
    {
        const int g = P.dim;
        if (d < P.D) {
            for (int j = d + 1; j <= d + g; j++) restrict_into(j);
            group(d + g, nullptr);
            for (int k = 1; k < P.gamma; k++) {
                const int c = d + g;
                const LevelG& q = P.lev[c];
                const size_t cnt = level_elems(P, c);
                (void)hipMemcpyAsync(at<T>(P, q.sr), R(c), es * cnt, hipMemcpyDeviceToDevice, s);
                (void)hipMemcpyAsync(at<T>(P, q.sv), V(c), es * cnt, hipMemcpyDeviceToDevice, s);
                {
                    Timed t(&P.tm, MG_K_RESTRICT, es * 3.0 * (double)cnt);
                    const double sh = 1.0 / q.m;   // sigma h
                    hipLaunchKernelGGL(kg_wres<T>, dim3((q.m - 1 + 255) / 256, q.m - 1, g == 3 ? q.m - 1 : 1), dim3(256),
                                       0, s, g, q.m, (T)(1.0 / (sh * sh)), R(c), V(c), ctl);
                }
                group(c, nullptr);
                hipLaunchKernelGGL(kg_add<T>, dim3((unsigned)std::min<size_t>((cnt + 255) / 256, 4096)), dim3(256), 0, s,
                                   cnt, at<T>(P, q.sv), V(c), ctl);
                (void)hipMemcpyAsync(R(c), at<T>(P, q.sr), es * cnt, hipMemcpyDeviceToDevice, s);
            }
        }
        const int top = d < P.D ? d + g - 1 : d;
        for (int j = top; j >= d; j--) {
            const bool coarsest = j == P.D;
            Lev3<T> cr = coarsest ? Lev3<T>{} : lv(j + 1);
            const T* vc = coarsest ? at<T>(P, P.zero) : V(j + 1);
            // further sweeps on the single-node coarsest grid repeat the first exactly (its neighbours are
            // boundary points): they are skipped
            const int sweeps = coarsest ? 1 : P.nu;
            for (int k = 0; k < sweeps; k++) {
                if (k > 0) again_input(j);
                const bool last = k == sweeps - 1;
                if (k == 0) sweep(j, vc, cr, u, j == 0 && last);
                else sweep(j, at<T>(P, P.lev[j].tq), tq_lev(j), u, j == 0 && last);
            }
        }
    }
};

template <typename T>
void enq_cycle(PlanG& P, double* u, const Ctl* ctl)
{
    CycleG<T> C{P, ctl, P.stream};
    C.group(0, u);
}

void enq_cycle_any(PlanG& P, double* u, const Ctl* ctl)
{
    if (P.prec == MG_FP64) enq_cycle<double>(P, u, ctl);
    else enq_cycle<float>(P, u, ctl);
}

double inner(int dim, int n) { return dim == 2 ? (double)(n - 1) * (n - 1) : (double)(n - 1) * (n - 1) * (n - 1); }

void enq_residual(PlanG& P, const double* u, const double* f, const Ctl* ctl)
{
    const double es = P.prec == MG_FP64 ? 8 : 4;
    Timed t(&P.tm, MG_K_RESIDUAL, (16 + es) * inner(P.dim, P.n));
    if (P.prec == MG_FP64)
        launch_residual<double>(P.dim, P.n, u, f, at<double>(P, P.r0), at<double>(P, P.partial), P.nparts, ctl,
                                P.stream, P.rorder);
    else
        launch_residual<float>(P.dim, P.n, u, f, at<float>(P, P.r0), at<double>(P, P.partial), P.nparts, ctl,
                               P.stream, P.rorder);
}

void enq_finalize(PlanG& P, int kind, Ctl* ctl, HostState* host = nullptr)
{
    Timed t(&P.tm, MG_K_NORM, 8.0 * P.nparts);
    launch_finalize(kind, at<double>(P, P.partial), P.nparts, ctl, P.stream, host);
}

const double* rhs(PlanG& P, const double* f)
{
    if (P.rorder != 4) return f;
    double* g = at<double>(P, P.g);
    if (P.dim == 2) launch_b_rhs4(P.n, f, g, P.stream);
    else launch_rhs4_3d(P.n, f, g, P.stream);
    return g;
}

}  // namespace

int plang_layout(PlanG& P, int dim, int n, int prec, const double* p, int nu, int gamma)
{
    if (dim != 2 && dim != 3) return MG_ERR_ARG;
    if (nu < 1 || nu > 8 || gamma < 1 || gamma > 2) return MG_ERR_ARG;
    const int K = ilog2(n);
    if (K < 1 || K > (dim == 2 ? 15 : 11)) return MG_ERR_SIZE;
    P.rorder = (prec & MG_ORDER4) ? 4 : 2;
    prec &= ~MG_ORDER4;
    if (prec != MG_FP64 && prec != MG_FP32_REFINED) return MG_ERR_ARG;
    P.dim = dim;
    P.n = n;
    P.prec = prec;
    P.nu = nu;
    P.gamma = gamma;
    P.D = dim * (K - 1);
    if (p)
        for (int i = 0; i < (dim == 2 ? 1 : 4); i++) P.p[i] = p[i];
    const size_t es = prec == MG_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = alignUp(off + bytes);
        return o;
    };
    P.ctl = take(sizeof(Ctl));
    P.nparts = residual_parts(dim, n);
    P.partial = take(sizeof(double) * (size_t)P.nparts);
    P.zero = take(sizeof(double) * 64);
    const double h = 1.0 / n;
    for (int d = 0; d <= P.D; d++) {
        LevelG& q = P.lev[d];
        q = LevelG{};
        q.m = n >> (d / dim);
        const double sh = (double)(n / q.m) * h;   // sigma * h
        if (dim == 2) {
            q.c = (d & 1) ? 2 * P.p[0] * sh * sh : P.p[0] * sh * sh;
        } else {
            const int t = d % 3;
            if (t == 0) q.c = P.p[3] * sh * sh;
            else if (t == 1) { q.c = 2 * P.p[1] * sh * sh; q.c2 = 4 * P.p[2] * sh * sh; }
            else q.c = 4 * P.p[0] * sh * sh;
        }
    }
    P.r0 = take(es * level_elems(P, 0));
    if (P.rorder == 4) P.g = take(sizeof(double) * level_elems(P, 0));
    if (nu > 1) P.v0 = take(es * level_elems(P, 0));
    for (int d = 1; d <= P.D; d++) {
        LevelG& q = P.lev[d];
        const size_t cnt = level_elems(P, d);
        q.r = take(es * cnt);
        q.v = take(es * cnt);
        if (dim == 3 && d % 3 == 2) {
            q.r2 = take(es * sizeMO(q.m));
            q.v2 = take(es * sizeMO(q.m));
        }
        if (gamma > 1 && d % dim == 0) {
            q.sr = take(es * cnt);
            q.sv = take(es * cnt);
        }
    }
    // the coarse input of a further sweep of level d has the layout of level d+1
    for (int d = 0; d < P.D && nu > 1; d++) {
        LevelG& q = P.lev[d];
        q.tq = take(es * level_elems(P, d + 1));
        if (dim == 3 && d % 3 == 1) q.tq2 = take(es * sizeMO(P.lev[d + 1].m));
    }
    P.total = off;
    return MG_OK;
}

int plang_setup(PlanG& P, void* ws, size_t ws_bytes, hipStream_t stream)
{
    if (!ws || ((uintptr_t)ws % kAlign) != 0 || ws_bytes < P.total) return MG_ERR_WS;
    P.ws = (char*)ws;
    P.stream = stream;
    P.tm.stream = stream;
    if (hipGetDevice(&P.device) != hipSuccess) return MG_ERR_HIP;
    if (hipHostMalloc((void**)&P.hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) return MG_ERR_HIP;
    // coherent: the finalize kernel's writes reach the polling host without a release
    if (hipHostMalloc((void**)&P.hstate, sizeof(HostState), hipHostMallocCoherent) != hipSuccess) return MG_ERR_HIP;
    P.live = true;
    return hip_status(hipMemsetAsync(P.ws, 0, P.total, P.stream));
}

void plang_destroy(PlanG& P)
{
    P.tm.destroy();
    if (P.live) (void)hipStreamSynchronize(P.stream);
    if (P.hctl) (void)hipHostFree(P.hctl);
    if (P.hstate) (void)hipHostFree(P.hstate);
}

int plang_vcycle(PlanG& P, double* u, const double* f, double* relres)
{
    Ctl* ctl = at<Ctl>(P, P.ctl);
    f = rhs(P, f);
    launch_ctl_reset(ctl, 0, 0, 0.0, P.stream);
    if (relres) {
        launch_sumsq(P.dim, P.n, f, at<double>(P, P.partial), P.nparts, ctl, P.stream);
        enq_finalize(P, 0, ctl);
    }
    enq_residual(P, u, f, ctl);
    if (relres) enq_finalize(P, 1, ctl);
    enq_cycle_any(P, u, ctl);
    int e = last_launch();
    if (e) return e;
    if (relres) {
        if (hipMemcpyAsync(P.hctl, ctl, kCtlHead, hipMemcpyDeviceToHost, P.stream) != hipSuccess ||
            hipStreamSynchronize(P.stream) != hipSuccess)
            return MG_ERR_HIP;
        *relres = P.hctl->last;
    }
    return MG_OK;
}

int plang_solve(PlanG& P, double* u, const double* f, double rtol, int max_cycles, int* cycles_out, double* rel_res_out,
                double* history)
{
    Ctl* ctl = at<Ctl>(P, P.ctl);
    hipStream_t s = P.stream;
    f = rhs(P, f);
    P.hstate->k = 0;   // the pinned evaluation count the loop polls, fresh before any kernel
    P.hstate->done = 0;
    launch_ctl_reset(ctl, 1, max_cycles, rtol, s);
    launch_sumsq(P.dim, P.n, f, at<double>(P, P.partial), P.nparts, ctl, s);
    enq_finalize(P, 0, ctl);
    enq_residual(P, u, f, ctl);
    enq_finalize(P, 1, ctl, P.hstate);
    auto launch = [&](int it1) -> int {
        enq_cycle_any(P, u, ctl);
        enq_residual(P, u, f, ctl);
        enq_finalize(P, 1, ctl, P.hstate);
        (void)it1;
        return last_launch();
    };
    double rr1 = -1, rr2 = -1;
    for (int it = 0;; it++) {
        const bool likely_last = rr1 > 0 && rr2 > 0 && rr1 * (rr1 / rr2) <= 2 * rtol;
        bool ahead = false;
        if (it < max_cycles && !likely_last) {
            int e = launch(it + 1);
            if (e) return e;
            ahead = true;
        }
        if (int e = wait_evaluation(P.hstate, it, s)) return e;
        const volatile HostState* h = P.hstate;
        if (h->done || it >= max_cycles) break;
        rr2 = rr1;
        rr1 = h->last;
        if (!ahead) {
            int e = launch(it + 1);
            if (e) return e;
        }
    }
    if (hipMemcpyAsync(P.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess) return MG_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
    const Ctl& H = *P.hctl;
    const int cyc = H.done ? H.cycles : max_cycles;
    if (cycles_out) *cycles_out = cyc;
    if (rel_res_out) *rel_res_out = H.last;
    if (history)
        for (int k = 0; k <= cyc; k++) history[k] = H.hist[k];
    return H.done ? H.status : MG_ERR_NOT_CONVERGED;
}

int plang_level_get(PlanG& P, int depth, int which, double* dst)
{
    if (depth < 0 || depth > P.D || (which != 0 && which != 1) || (which == 1 && depth == 0)) return MG_ERR_ARG;
    const LevelG& q = P.lev[depth];
    const size_t src = which == 0 ? (depth == 0 ? P.r0 : q.r) : q.v;
    const size_t src2 = which == 0 ? q.r2 : q.v2;
    if (P.dim == 2) {
        if (P.prec == MG_FP64) launch_b_level_get<double>(depth & 1, q.m, at<double>(P, src), dst, P.stream);
        else launch_b_level_get<float>(depth & 1, q.m, at<float>(P, src), dst, P.stream);
    } else {
        const int kind = depth % 3;
        if (P.prec == MG_FP64)
            launch_level_get3<double>(kind, q.m, at<double>(P, src), kind == 2 ? at<double>(P, src2) : nullptr, dst,
                                      P.stream);
        else
            launch_level_get3<float>(kind, q.m, at<float>(P, src), kind == 2 ? at<float>(P, src2) : nullptr, dst,
                                     P.stream);
    }
    return last_launch();
}

}  // namespace dmg

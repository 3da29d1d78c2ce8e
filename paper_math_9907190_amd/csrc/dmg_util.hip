// Residual, norms and the on-device stopping decision of libdmg.
//
// r = f - Lap_h(u) (Eq. Evpois) with the 5-point (2D) or 7-point (3D)
// second-order Laplacian, computed in double from double u and f and stored
// as T (double, or float for the single-precision cycle).  The squared norm
// is accumulated from the double residual: per block by a wavefront
// shuffle reduction, then across blocks in one fixed-order pass, so the
// result is deterministic for a given n.
#include "dmg_launch.hpp"

#include <math.h>
#include <string.h>

namespace dmg {

constexpr int kMaxParts = 16384;
constexpr int kRowThreads = 256;

__device__ inline double block_sum(double x)
{
    __shared__ double red[kRowThreads / 64];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = x;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += red[i];
    return s;  // valid in thread 0
}

static void row_grid(int dim, int n, dim3& g)
{
    long rows = (dim == 2) ? (long)(n - 1) : (long)(n - 1) * (n - 1);
    int gx = (n - 1 + kRowThreads - 1) / kRowThreads;
    long gy = rows;
    long cap = kMaxParts / gx;
    if (gy > cap) gy = cap;
    if (gy < 1) gy = 1;
    g = dim3(gx, (unsigned)gy);
}

int residual_parts(int dim, int n)
{
    dim3 g;
    row_grid(dim, n, g);
    return (int)(g.x * g.y);
}

template <typename T>
__global__ void __launch_bounds__(kRowThreads) k_residual(int dim, int n, double inv_h2,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ f, T* __restrict__ r0,
                                                          double* __restrict__ partial, const Ctl* ctl, int m4)
{
    if (ctl && ctl->done) return;
    int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
    long rows = (dim == 2) ? (long)(n - 1) : (long)(n - 1) * (n - 1);
    size_t s = (size_t)n + 1, s2 = s * s;
    double acc = 0;
    for (long q = blockIdx.y; q < rows; q += gridDim.y) {
        if (a >= n) continue;
        if (dim == 2) {
            size_t c = (size_t)(q + 1) * s + a;
            double lap = m4 ? (-20 * u[c] + 4 * (u[c - s] + u[c + s] + u[c - 1] + u[c + 1]) + u[c + 1 + s] +
                               u[c - 1 + s] + u[c - 1 - s] + u[c + 1 - s]) * inv_h2
                            : (u[c - 1] + u[c - s] + u[c + 1] + u[c + s] - 4 * u[c]) * inv_h2;
            double r = f[c] - lap;
            r0[c] = (T)r;
            acc += r * r;
        } else {
            long b = q % (n - 1) + 1, cz = q / (n - 1) + 1;
            size_t c = (size_t)cz * s2 + (size_t)b * s + a;
            double lap = m4 ? (-24 * u[c] + 2 * (u[c - s] + u[c + s] + u[c - 1] + u[c + 1] + u[c + s2] + u[c - s2]) +
                               u[c + 1 + s] + u[c - 1 + s] + u[c - 1 - s] + u[c + 1 - s] + u[c + s + s2] +
                               u[c + s - s2] + u[c - s - s2] + u[c - s + s2] + u[c + 1 + s2] + u[c - 1 + s2] +
                               u[c - 1 - s2] + u[c + 1 - s2]) * inv_h2
                            : (u[c + 1] + u[c - 1] + u[c + s] + u[c - s] + u[c + s2] + u[c - s2] - 6 * u[c]) * inv_h2;
            double r = f[c] - lap;
            r0[c] = (T)r;
            acc += r * r;
        }
    }
    double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = t;
}

template <typename T>
void launch_residual(int dim, int n, const double* u, const double* f, T* r0, double* partial, int nparts,
                     const Ctl* ctl, hipStream_t s, int order)
{
    dim3 g;
    row_grid(dim, n, g);
    (void)nparts;
    const int m4 = order == 4 ? 1 : 0;
    double inv_h2 = m4 ? (double)n * (double)n / 6 : (double)n * (double)n;
    hipLaunchKernelGGL(k_residual<T>, g, dim3(kRowThreads), 0, s, dim, n, inv_h2, u, f, r0, partial, ctl, m4);
}

__global__ void __launch_bounds__(kRowThreads) k_sumsq(int dim, int n, const double* __restrict__ a_,
                                                       double* __restrict__ partial, const Ctl* ctl)
{
    if (ctl && ctl->done) return;
    int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
    long rows = (dim == 2) ? (long)(n - 1) : (long)(n - 1) * (n - 1);
    size_t s = (size_t)n + 1, s2 = s * s;
    double acc = 0;
    for (long q = blockIdx.y; q < rows; q += gridDim.y) {
        if (a >= n) continue;
        size_t c = (dim == 2) ? (size_t)(q + 1) * s + a
                              : (size_t)(q / (n - 1) + 1) * s2 + (size_t)(q % (n - 1) + 1) * s + a;
        double x = a_[c];
        acc += x * x;
    }
    double t = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = t;
}

void launch_sumsq(int dim, int n, const double* a, double* partial, int nparts, const Ctl* ctl, hipStream_t s)
{
    dim3 g;
    row_grid(dim, n, g);
    (void)nparts;
    hipLaunchKernelGGL(k_sumsq, g, dim3(kRowThreads), 0, s, dim, n, a, partial, ctl);
}

// kind 0: ctl->fnorm = sqrt(sum).  kind 1: relative residual after k cycles
// and the outer iteration's decision (Section 1): stop when it is <= rtol,
// when it is not finite, when it grew three cycles in a row above the
// starting value, or after max_cycles cycles.
__global__ void __launch_bounds__(1024) k_finalize(int kind, const double* __restrict__ partial, int nparts,
                                                   Ctl* ctl, HostState* host)
{
    if (ctl->done) return;
    __shared__ double red[1024];
    double s = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double tot = red[0];
    if (kind == 0) {
        ctl->fnorm = sqrt(tot);
        return;
    }
    const int k = ctl->k;   // evaluation index = cycles run so far
    ctl->k = k + 1;
    double rn = sqrt(tot);
    double rr = ctl->fnorm > 0 ? rn / ctl->fnorm : rn;
    ctl->last = rr;
    if (k <= kMaxCycles) ctl->hist[k] = rr;
    if (ctl->mode == 0) return;
    int finite = isfinite(rr);
    if (k == 0) {
        ctl->rr0 = rr;
        ctl->prev = rr;
        ctl->grow = 0;
        if (rr <= ctl->rtol) { ctl->status = 0; ctl->done = 1; }
        else if (ctl->max_cycles == 0) { ctl->status = -8; ctl->done = 1; }
        else if (!finite) { ctl->status = -6; ctl->done = 1; }
    } else {
        if (!finite) { ctl->status = -6; ctl->done = 1; }
        else {
            ctl->grow = (rr > ctl->prev) ? ctl->grow + 1 : 0;
            ctl->prev = rr;
            if (ctl->grow >= 3 && rr > ctl->rr0) { ctl->status = -7; ctl->done = 1; }
            else if (rr <= ctl->rtol) { ctl->status = 0; ctl->done = 1; }
            else if (k >= ctl->max_cycles) { ctl->status = -8; ctl->done = 1; }
        }
    }
    if (ctl->done) ctl->cycles = k;
    if (host) {   // pinned host memory, read by the host after an event that follows this kernel
        host->last = rr;
        host->done = ctl->done;
        host->k = k + 1;   // written last: what the host loop polls
    }
}

void launch_finalize(int kind, const double* partial, int nparts, Ctl* ctl, hipStream_t s, HostState* host)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, kind, partial, nparts, ctl, host);
}

__global__ void k_ctl_reset(Ctl* ctl, int mode, int max_cycles, double rtol, int net)
{
    if (threadIdx.x != 0) return;
    ctl->done = 0;
    ctl->status = 0;
    ctl->cycles = 0;
    ctl->k = 0;
    ctl->grow = 0;
    ctl->mode = mode;
    ctl->max_cycles = max_cycles;
    ctl->rtol = rtol;
    ctl->fnorm = 0;
    ctl->rr0 = ctl->prev = ctl->last = 0;
    ctl->net = net;
    ctl->theta = 0;
    ctl->q_net = 0;
    ctl->net_used = 0;
    ctl->net_off = 0;
}

void launch_ctl_reset(Ctl* ctl, int mode, int max_cycles, double rtol, hipStream_t s, int net)
{
    hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, s, ctl, mode, max_cycles, rtol, net);
}

// ------------------------------------------------ stream-ordered workspace set-up
// Zero `bytes` (a multiple of 16) at dst: a fill kernel rather than a
// memset, so the set-up stays a kernel on the caller's stream.
__global__ void __launch_bounds__(256) k_zero16(uint4* __restrict__ dst, size_t n16)
{
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = z;
}

void launch_zero(void* dst, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    const size_t want = (n16 + 255) / 256;
    const int blocks = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(256), 0, s, (uint4*)dst, n16);
}

// Copy words carried in the kernel arguments to dst: host data reaches the
// device in stream order without a host buffer that must outlive the call.
__global__ void __launch_bounds__(256) k_put_words(unsigned* __restrict__ dst, PutWords c, int nw)
{
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = c.w[i];
}

void launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const unsigned char* p = (const unsigned char*)src;
    unsigned char* d = (unsigned char*)dst;
    while (bytes > 0) {
        const size_t chunk = bytes < sizeof(PutWords) ? bytes : sizeof(PutWords);
        PutWords c;
        memcpy(c.w, p, chunk);
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, (unsigned*)d, c, (int)(chunk / 4));
        p += chunk;
        d += chunk;
        bytes -= chunk;
    }
}

template void launch_residual<double>(int, int, const double*, const double*, double*, double*, int, const Ctl*,
                                      hipStream_t, int);
template void launch_residual<float>(int, int, const double*, const double*, float*, double*, int, const Ctl*,
                                     hipStream_t, int);

}  // namespace dmg

// 2D kernels of libdmg: restriction (Eqs. Erest2r, Erest2b) and the
// over-relaxed red-black Jacobi prolongation (Eqs. Eajacr, Eajacb and the
// axis-grid analogue) of Roberts, Section 2.
//
// Jacobi kernels give each thread one (C, F) pair: the point that is also on
// the coarser level (C) and a neighbour that is not (F).  The F value is
// computed from the coarser correction; the C value needs the new values of
// its four F neighbours, which the thread recomputes from the coarser
// correction instead of waiting for the threads that own them, so one launch
// does both half-sweeps with no grid-wide barrier.
#include "dmg_launch.hpp"

namespace dmg {

#define DMG_GATE(ctl) \
    if ((ctl) != nullptr && (ctl)->done) return

// ------------------------------------------------------------ restriction

// axis grid (side m) -> diagonal grid (side m): one thread per D-layout slot.
template <typename T>
__global__ void __launch_bounds__(256) k2_rs_a2d(int m, const T* __restrict__ rA, T* __restrict__ rD,
                                                 const Ctl* ctl)
{
    DMG_GATE(ctl);
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1;
    if (col > m / 2 || b >= m) return;
    int a = 2 * col + (b & 1);
    if (a < 1 || a >= m) return;
    rD[idxD(m, a, b)] = rs2_a2d(rA, m, a, b);
}

// diagonal grid (side m) -> axis grid (side m/2): one thread per coarse point.
template <typename T>
__global__ void __launch_bounds__(256) k2_rs_d2a(int m, const T* __restrict__ rD, T* __restrict__ rA2,
                                                 const Ctl* ctl)
{
    DMG_GATE(ctl);
    int mc = m / 2;
    int A = blockIdx.x * blockDim.x + threadIdx.x + 1;
    int B = blockIdx.y + 1;
    if (A >= mc || B >= mc) return;
    rA2[idxA(mc, A, B)] = rs2_d2a(rD, m, A, B);
}

template <typename T>
void launch_rs2(int diag_in, int m, const T* in, T* out, const Ctl* ctl, hipStream_t s)
{
    if (!diag_in) {
        dim3 g((m / 2 + 1 + 255) / 256, m - 1);
        hipLaunchKernelGGL(k2_rs_a2d<T>, g, dim3(256), 0, s, m, in, out, ctl);
    } else {
        int mc = m / 2;
        if (mc < 2) return;
        dim3 g((mc - 1 + 255) / 256, mc - 1);
        hipLaunchKernelGGL(k2_rs_d2a<T>, g, dim3(256), 0, s, m, in, out, ctl);
    }
}

// ----------------------------------------------------------------- Jacobi

// diagonal grid of side m: thread (A, B) owns F = (2A+1, 2B+1) and C = (2A, 2B).
template <typename T>
__global__ void __launch_bounds__(256) k2_jac_diag(int m, T cc, const T* __restrict__ rD,
                                                   const T* __restrict__ vA2, T* __restrict__ vD,
                                                   const Ctl* ctl)
{
    DMG_GATE(ctl);
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    int B = blockIdx.y;
    int h = m / 2;
    if (A >= h || B >= h) return;
    int a = 2 * A + 1, b = 2 * B + 1;
    vD[idxD(m, a, b)] = jac2_diagF(rD, vA2, m, cc, a, b);
    if (A >= 1 && B >= 1) vD[idxD(m, 2 * A, 2 * B)] = jac2_diagC(rD, vA2, m, cc, 2 * A, 2 * B);
}

// axis grid of side m: thread (t, b) owns columns 2t and 2t+1 of row b.
template <typename T>
__global__ void __launch_bounds__(256) k2_jac_axis(int m, T cc, const T* __restrict__ rA,
                                                   const T* __restrict__ vD, T* __restrict__ vA,
                                                   const Ctl* ctl)
{
    DMG_GATE(ctl);
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1;
    if (t > m / 2 || b >= m) return;
    int aC = 2 * t + (b & 1);      // a + b even: also on the coarser diagonal grid
    int aF = 2 * t + 1 - (b & 1);  // a + b odd
    if (aF >= 1 && aF < m) vA[idxA(m, aF, b)] = jac2_axisF(rA, vD, m, cc, aF, b);
    if (aC >= 1 && aC < m) vA[idxA(m, aC, b)] = jac2_axisC(rA, vD, m, cc, aC, b);
}

// finest axis grid: the same pair sweep, then u <- u + v (Section 1).
template <typename T>
__global__ void __launch_bounds__(256) k2_jac_finest(int n, T cc, const T* __restrict__ r0,
                                                     const T* __restrict__ vD, double* __restrict__ u,
                                                     const Ctl* ctl)
{
    DMG_GATE(ctl);
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1;
    if (t > n / 2 || b >= n) return;
    int aC = 2 * t + (b & 1);
    int aF = 2 * t + 1 - (b & 1);
    if (aF >= 1 && aF < n) {
        size_t q = idxA(n, aF, b);
        u[q] = u[q] + (double)jac2_axisF(r0, vD, n, cc, aF, b);
    }
    if (aC >= 1 && aC < n) {
        size_t q = idxA(n, aC, b);
        u[q] = u[q] + (double)jac2_axisC(r0, vD, n, cc, aC, b);
    }
}

template <typename T>
void launch_jac2(int diag, int m, T c, const T* r, const T* vc, T* v, const Ctl* ctl, hipStream_t s)
{
    if (diag) {
        dim3 g((m / 2 + 255) / 256, m / 2);
        hipLaunchKernelGGL(k2_jac_diag<T>, g, dim3(256), 0, s, m, c, r, vc, v, ctl);
    } else {
        dim3 g((m / 2 + 1 + 255) / 256, m - 1);
        hipLaunchKernelGGL(k2_jac_axis<T>, g, dim3(256), 0, s, m, c, r, vc, v, ctl);
    }
}

template <typename T>
void launch_jac2_finest(int n, T c, const T* r0, const T* vD, double* u, const Ctl* ctl, hipStream_t s)
{
    dim3 g((n / 2 + 1 + 255) / 256, n - 1);
    hipLaunchKernelGGL(k2_jac_finest<T>, g, dim3(256), 0, s, n, c, r0, vD, u, ctl);
}

// ------------------------------------------------- coarse persistent kernel
// All levels from depth `first` down to the coarsest in one workgroup:
// restriction first+1 .. last, the coarsest Jacobi from zero, then Jacobi
// back up to `first`.  Levels this small live in L2; the point of the
// kernel is to replace ~2 launches per level by one.
constexpr int kCoarseThreads = 1024;

template <typename T>
__global__ void __launch_bounds__(kCoarseThreads) k2_coarse(Coarse2<T> a, const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int d = a.first + 1; d <= a.last; d++) {
        const Lev2<T>& F = a.lev[d - 1];
        const Lev2<T>& C = a.lev[d];
        int m = F.m;
        if (!F.diag) {  // axis -> diagonal, same side
            int w = m / 2 + 1;
            for (int q = tid; q < w * (m - 1); q += nt) {
                int col = q % w, b = q / w + 1;
                int aa = 2 * col + (b & 1);
                if (aa >= 1 && aa < m) C.r[idxD(m, aa, b)] = rs2_a2d(F.r, m, aa, b);
            }
        } else {        // diagonal -> axis of side m/2
            int mc = m / 2;
            for (int q = tid; q < (mc - 1) * (mc - 1); q += nt) {
                int A = q % (mc - 1) + 1, B = q / (mc - 1) + 1;
                C.r[idxA(mc, A, B)] = rs2_d2a(F.r, m, A, B);
            }
        }
        __syncthreads();
    }
    for (int d = a.last; d >= a.first; d--) {
        const Lev2<T>& L = a.lev[d];
        const T* vc = (d == a.last) ? a.zeroD : a.lev[d + 1].v;
        int m = L.m;
        if (L.diag) {
            int h = m / 2;
            for (int q = tid; q < h * h; q += nt) {
                int A = q % h, B = q / h;
                L.v[idxD(m, 2 * A + 1, 2 * B + 1)] = jac2_diagF(L.r, vc, m, L.c, 2 * A + 1, 2 * B + 1);
                if (A >= 1 && B >= 1) L.v[idxD(m, 2 * A, 2 * B)] = jac2_diagC(L.r, vc, m, L.c, 2 * A, 2 * B);
            }
        } else {
            int w = m / 2 + 1;
            for (int q = tid; q < w * (m - 1); q += nt) {
                int t = q % w, b = q / w + 1;
                int aC = 2 * t + (b & 1), aF = 2 * t + 1 - (b & 1);
                if (aF >= 1 && aF < m) L.v[idxA(m, aF, b)] = jac2_axisF(L.r, vc, m, L.c, aF, b);
                if (aC >= 1 && aC < m) L.v[idxA(m, aC, b)] = jac2_axisC(L.r, vc, m, L.c, aC, b);
            }
        }
        __syncthreads();
    }
}

template <typename T>
void launch_coarse2(const Coarse2<T>& a, const Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k2_coarse<T>, dim3(1), dim3(kCoarseThreads), 0, s, a, ctl);
}

// ------------------------------------------------------------ level export
template <typename T>
__global__ void k2_level_get(int diag, int m, const T* __restrict__ src, double* __restrict__ dst)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y;
    if (a > m || b > m) return;
    double x = 0;
    if (!diag) x = (double)src[idxA(m, a, b)];
    else if (((a + b) & 1) == 0) x = (double)src[idxD(m, a, b)];
    dst[idxA(m, a, b)] = x;
}

template <typename T>
void launch_level_get2(int diag, int m, const T* src, double* dst, hipStream_t s)
{
    dim3 g((m + 1 + 255) / 256, m + 1);
    hipLaunchKernelGGL(k2_level_get<T>, g, dim3(256), 0, s, diag, m, src, dst);
}

#define DMG_INST2(T)                                                                                   \
    template void launch_rs2<T>(int, int, const T*, T*, const Ctl*, hipStream_t);                      \
    template void launch_jac2<T>(int, int, T, const T*, const T*, T*, const Ctl*, hipStream_t);         \
    template void launch_jac2_finest<T>(int, T, const T*, const T*, double*, const Ctl*, hipStream_t); \
    template void launch_coarse2<T>(const Coarse2<T>&, const Ctl*, hipStream_t);                        \
    template void launch_level_get2<T>(int, int, const T*, double*, hipStream_t);
DMG_INST2(double)
DMG_INST2(float)

}  // namespace dmg

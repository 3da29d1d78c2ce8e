// 3D kernels of libdmg: restrictions Eqs. (Erred), (Ermagc), (Ermagm),
// (Erblu) and the Jacobi steps Eqs. (Emprolm)-(Egprolr) of Roberts,
// Section 3.  As in 2D, each Jacobi thread owns the points of one cell and
// recomputes the first-half-sweep values its second-half-sweep point needs,
// so both half-sweeps run in one launch.
#include "dmg_launch.hpp"
#include "dmg_launch3.hpp"

namespace dmg {

#define DMG_GATE(ctl) \
    if ((ctl) != nullptr && (ctl)->done) return

// ------------------------------------------------------------ restriction

// green (side m) -> red (side m): one thread per R-layout slot
template <typename T>
__global__ void __launch_bounds__(256) k3_rs_g2r(int m, const T* __restrict__ rG, T* __restrict__ rR, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1, c = blockIdx.z + 1;
    if (col > m / 2) return;
    int a = 2 * col + ((b + c) & 1);
    if (a < 1 || a >= m) return;
    rR[idxR(m, a, b, c)] = rs3_g2r(rG, m, a, b, c);
}

// red (side m) -> magenta (side m): thread (A,B,C) owns centre (2A+1,2B+1,2C+1) and corner (2A,2B,2C)
template <typename T>
__global__ void __launch_bounds__(256) k3_rs_r2m(int m, const T* __restrict__ rR, T* __restrict__ rE,
                                                 T* __restrict__ rO, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int h = m / 2;
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    int B = blockIdx.y, C = blockIdx.z;
    if (A >= h) return;
    rO[idxMO(m, 2 * A + 1, 2 * B + 1, 2 * C + 1)] = rs3_r2mO(rR, m, 2 * A + 1, 2 * B + 1, 2 * C + 1);
    if (A >= 1 && B >= 1 && C >= 1) rE[idxME(m, 2 * A, 2 * B, 2 * C)] = rs3_r2mE(rR, m, 2 * A, 2 * B, 2 * C);
}

// magenta (side m) -> blue = green of side m/2
template <typename T>
__global__ void __launch_bounds__(256) k3_rs_m2b(int m, const T* __restrict__ rE, const T* __restrict__ rO,
                                                 T* __restrict__ rB, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int mc = m / 2;
    int A = blockIdx.x * blockDim.x + threadIdx.x + 1;
    int B = blockIdx.y + 1, C = blockIdx.z + 1;
    if (A >= mc) return;
    rB[idxG(mc, A, B, C)] = rs3_m2b(rE, rO, m, A, B, C);
}

template <typename T>
void launch_rs3(const Lev3<T>& F, const Lev3<T>& Cc, const Ctl* ctl, hipStream_t s)
{
    int m = F.m;
    if (Cc.kind == 1) {
        dim3 g((m / 2 + 1 + 255) / 256, m - 1, m - 1);
        hipLaunchKernelGGL(k3_rs_g2r<T>, g, dim3(256), 0, s, m, F.r, Cc.r, ctl);
    } else if (Cc.kind == 2) {
        dim3 g((m / 2 + 255) / 256, m / 2, m / 2);
        hipLaunchKernelGGL(k3_rs_r2m<T>, g, dim3(256), 0, s, m, F.r, Cc.r, Cc.r2, ctl);
    } else {
        int mc = m / 2;
        if (mc < 2) return;
        dim3 g((mc - 1 + 255) / 256, mc - 1, mc - 1);
        hipLaunchKernelGGL(k3_rs_m2b<T>, g, dim3(256), 0, s, m, F.r, F.r2, Cc.r, ctl);
    }
}

// ----------------------------------------------------------------- Jacobi

template <typename T>
__global__ void __launch_bounds__(256) k3_jac_mag(int m, T cc, const T* __restrict__ rE, const T* __restrict__ rO,
                                                  const T* __restrict__ vB, T* __restrict__ vE, T* __restrict__ vO,
                                                  const Ctl* ctl)
{
    DMG_GATE(ctl);
    int h = m / 2;
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    int B = blockIdx.y, C = blockIdx.z;
    if (A >= h) return;
    int a = 2 * A + 1, b = 2 * B + 1, c = 2 * C + 1;
    vO[idxMO(m, a, b, c)] = jac3_magF(rO, vB, m, cc, a, b, c);
    if (A >= 1 && B >= 1 && C >= 1) vE[idxME(m, a - 1, b - 1, c - 1)] = jac3_magC(rE, rO, vB, m, cc, a - 1, b - 1, c - 1);
}

// thread (A,B,C) owns the cell's face centres (2A+1,2B+1,2C), (2A,2B+1,2C+1),
// (2A+1,2B,2C+1) and its corner (2A,2B,2C)
template <typename T>
__global__ void __launch_bounds__(256) k3_jac_red(int m, T c1, T c2, const T* __restrict__ rR,
                                                  const T* __restrict__ vE, const T* __restrict__ vO,
                                                  T* __restrict__ vR, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int h = m / 2;
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    int B = blockIdx.y, C = blockIdx.z;
    if (A >= h) return;
    int a = 2 * A, b = 2 * B, c = 2 * C;
    if (C >= 1) vR[idxR(m, a + 1, b + 1, c)] = jac3_redF(rR, vE, vO, m, c1, a + 1, b + 1, c);
    if (A >= 1) vR[idxR(m, a, b + 1, c + 1)] = jac3_redF(rR, vE, vO, m, c1, a, b + 1, c + 1);
    if (B >= 1) vR[idxR(m, a + 1, b, c + 1)] = jac3_redF(rR, vE, vO, m, c1, a + 1, b, c + 1);
    if (A >= 1 && B >= 1 && C >= 1) vR[idxR(m, a, b, c)] = jac3_redC(rR, vE, vO, m, c1, c2, a, b, c);
}

// green grid: thread (t, b, c) owns x = 2t and 2t+1 of row (b, c)
template <typename T>
__global__ void __launch_bounds__(256) k3_jac_green(int m, T cc, const T* __restrict__ rG, const T* __restrict__ vR,
                                                    T* __restrict__ vG, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1, c = blockIdx.z + 1;
    if (t > m / 2) return;
    int par = (b + c) & 1;
    int aC = 2 * t + par, aF = 2 * t + 1 - par;
    if (aF >= 1 && aF < m) vG[idxG(m, aF, b, c)] = jac3_greenF(rG, vR, m, cc, aF, b, c);
    if (aC >= 1 && aC < m) vG[idxG(m, aC, b, c)] = jac3_greenC(rG, vR, m, cc, aC, b, c);
}

template <typename T>
__global__ void __launch_bounds__(256) k3_jac_finest(int n, T cc, const T* __restrict__ r0, const T* __restrict__ vR,
                                                     double* __restrict__ u, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1, c = blockIdx.z + 1;
    if (t > n / 2) return;
    int par = (b + c) & 1;
    int aC = 2 * t + par, aF = 2 * t + 1 - par;
    if (aF >= 1 && aF < n) {
        size_t q = idxG(n, aF, b, c);
        u[q] = u[q] + (double)jac3_greenF(r0, vR, n, cc, aF, b, c);
    }
    if (aC >= 1 && aC < n) {
        size_t q = idxG(n, aC, b, c);
        u[q] = u[q] + (double)jac3_greenC(r0, vR, n, cc, aC, b, c);
    }
}

template <typename T>
void launch_jac3(const Lev3<T>& L, const Lev3<T>& Cr, T* zero, const Ctl* ctl, hipStream_t s)
{
    int m = L.m;
    const T* vc = Cr.v ? Cr.v : zero;
    if (L.kind == 2) {
        dim3 g((m / 2 + 255) / 256, m / 2, m / 2);
        hipLaunchKernelGGL(k3_jac_mag<T>, g, dim3(256), 0, s, m, L.c, L.r, L.r2, vc, L.v, L.v2, ctl);
    } else if (L.kind == 1) {
        dim3 g((m / 2 + 255) / 256, m / 2, m / 2);
        hipLaunchKernelGGL(k3_jac_red<T>, g, dim3(256), 0, s, m, L.c, L.c2, L.r, Cr.v, Cr.v2, L.v, ctl);
    } else {
        dim3 g((m / 2 + 1 + 255) / 256, m - 1, m - 1);
        hipLaunchKernelGGL(k3_jac_green<T>, g, dim3(256), 0, s, m, L.c, L.r, vc, L.v, ctl);
    }
}

template <typename T>
void launch_jac3_finest(int n, T c, const T* r0, const T* vR, double* u, const Ctl* ctl, hipStream_t s)
{
    dim3 g((n / 2 + 1 + 255) / 256, n - 1, n - 1);
    hipLaunchKernelGGL(k3_jac_finest<T>, g, dim3(256), 0, s, n, c, r0, vR, u, ctl);
}

// ------------------------------------------------- coarse persistent kernel
constexpr int kCoarse3Threads = 1024;

template <typename T>
__global__ void __launch_bounds__(kCoarse3Threads) k3_coarse(Coarse3<T> a, const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int d = a.first + 1; d <= a.last; d++) {
        const Lev3<T>& F = a.lev[d - 1];
        const Lev3<T>& C = a.lev[d];
        int m = F.m;
        if (C.kind == 1) {
            int w = m / 2 + 1;
            int tot = w * (m - 1) * (m - 1);
            for (int q = tid; q < tot; q += nt) {
                int col = q % w, b = (q / w) % (m - 1) + 1, c = q / (w * (m - 1)) + 1;
                int aa = 2 * col + ((b + c) & 1);
                if (aa >= 1 && aa < m) C.r[idxR(m, aa, b, c)] = rs3_g2r(F.r, m, aa, b, c);
            }
        } else if (C.kind == 2) {
            int h = m / 2;
            for (int q = tid; q < h * h * h; q += nt) {
                int A = q % h, B = (q / h) % h, Cc = q / (h * h);
                C.r2[idxMO(m, 2 * A + 1, 2 * B + 1, 2 * Cc + 1)] = rs3_r2mO(F.r, m, 2 * A + 1, 2 * B + 1, 2 * Cc + 1);
                if (A >= 1 && B >= 1 && Cc >= 1) C.r[idxME(m, 2 * A, 2 * B, 2 * Cc)] = rs3_r2mE(F.r, m, 2 * A, 2 * B, 2 * Cc);
            }
        } else {
            int mc = m / 2, k = mc - 1;
            for (int q = tid; q < k * k * k; q += nt) {
                int A = q % k + 1, B = (q / k) % k + 1, Cc = q / (k * k) + 1;
                C.r[idxG(mc, A, B, Cc)] = rs3_m2b(F.r, F.r2, m, A, B, Cc);
            }
        }
        __syncthreads();
    }
    for (int d = a.last; d >= a.first; d--) {
        const Lev3<T>& L = a.lev[d];
        int m = L.m;
        if (L.kind == 2) {
            const T* vB = a.lev[d + 1].v;
            int h = m / 2;
            for (int q = tid; q < h * h * h; q += nt) {
                int A = q % h, B = (q / h) % h, Cc = q / (h * h);
                int x = 2 * A + 1, y = 2 * B + 1, z = 2 * Cc + 1;
                L.v2[idxMO(m, x, y, z)] = jac3_magF(L.r2, vB, m, L.c, x, y, z);
                if (A >= 1 && B >= 1 && Cc >= 1) L.v[idxME(m, x - 1, y - 1, z - 1)] = jac3_magC(L.r, L.r2, vB, m, L.c, x - 1, y - 1, z - 1);
            }
        } else if (L.kind == 1) {
            const Lev3<T>& M = a.lev[d + 1];
            int h = m / 2;
            for (int q = tid; q < h * h * h; q += nt) {
                int A = q % h, B = (q / h) % h, Cc = q / (h * h);
                int x = 2 * A, y = 2 * B, z = 2 * Cc;
                if (Cc >= 1) L.v[idxR(m, x + 1, y + 1, z)] = jac3_redF(L.r, M.v, M.v2, m, L.c, x + 1, y + 1, z);
                if (A >= 1) L.v[idxR(m, x, y + 1, z + 1)] = jac3_redF(L.r, M.v, M.v2, m, L.c, x, y + 1, z + 1);
                if (B >= 1) L.v[idxR(m, x + 1, y, z + 1)] = jac3_redF(L.r, M.v, M.v2, m, L.c, x + 1, y, z + 1);
                if (A >= 1 && B >= 1 && Cc >= 1) L.v[idxR(m, x, y, z)] = jac3_redC(L.r, M.v, M.v2, m, L.c, L.c2, x, y, z);
            }
        } else {
            const T* vR = (d == a.last) ? a.zero : a.lev[d + 1].v;
            int w = m / 2 + 1;
            int tot = w * (m - 1) * (m - 1);
            for (int q = tid; q < tot; q += nt) {
                int t = q % w, b = (q / w) % (m - 1) + 1, c = q / (w * (m - 1)) + 1;
                int par = (b + c) & 1;
                int aC = 2 * t + par, aF = 2 * t + 1 - par;
                if (aF >= 1 && aF < m) L.v[idxG(m, aF, b, c)] = jac3_greenF(L.r, vR, m, L.c, aF, b, c);
                if (aC >= 1 && aC < m) L.v[idxG(m, aC, b, c)] = jac3_greenC(L.r, vR, m, L.c, aC, b, c);
            }
        }
        __syncthreads();
    }
}

template <typename T>
void launch_coarse3(const Coarse3<T>& a, const Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k3_coarse<T>, dim3(1), dim3(kCoarse3Threads), 0, s, a, ctl);
}

// ------------------------------------------------------------ level export
template <typename T>
__global__ void k3_level_get(int kind, int m, const T* __restrict__ src, const T* __restrict__ src2,
                             double* __restrict__ dst)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y, c = blockIdx.z;
    if (a > m) return;
    double x = 0;
    int nodd = (a & 1) + (b & 1) + (c & 1);
    if (kind == 0) x = (double)src[idxG(m, a, b, c)];
    else if (kind == 1) { if ((nodd & 1) == 0) x = (double)src[idxR(m, a, b, c)]; }
    else {
        if (nodd == 0) x = (double)src[idxME(m, a, b, c)];
        else if (nodd == 3) x = (double)src2[idxMO(m, a, b, c)];
    }
    dst[idxG(m, a, b, c)] = x;
}

template <typename T>
void launch_level_get3(int kind, int m, const T* src, const T* src2, double* dst, hipStream_t s)
{
    dim3 g((m + 1 + 255) / 256, m + 1, m + 1);
    hipLaunchKernelGGL(k3_level_get<T>, g, dim3(256), 0, s, kind, m, src, src2, dst);
}

#define DMG_INST3(T)                                                                                      \
    template void launch_rs3<T>(const Lev3<T>&, const Lev3<T>&, const Ctl*, hipStream_t);                 \
    template void launch_jac3<T>(const Lev3<T>&, const Lev3<T>&, T*, const Ctl*, hipStream_t);            \
    template void launch_jac3_finest<T>(int, T, const T*, const T*, double*, const Ctl*, hipStream_t);    \
    template void launch_coarse3<T>(const Coarse3<T>&, const Ctl*, hipStream_t);                          \
    template void launch_level_get3<T>(int, int, const T*, const T*, double*, hipStream_t);
DMG_INST3(double)
DMG_INST3(float)

}  // namespace dmg

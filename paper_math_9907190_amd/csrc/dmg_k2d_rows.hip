// Row-marching 2D kernels of libdmg for the large levels.
//
// A wavefront owns a band of columns and marches down a strip of kRows rows,
// holding a three-row window of its inputs in registers.  On an axis grid
// each lane owns the column pair (2t, 2t+1), so in every row it holds one
// point of each colour; the one value it needs from the neighbouring pair
// comes across lanes by shuffle.  The first and last lane of a wave are halo
// lanes: they compute but do not write, so a wave covers 62 pairs and no
// value ever has to cross a wave.  Every HBM element is read once (plus the
// strip's halo rows), in full coalesced rows.
//
// Arithmetic per point is the paper's (Eqs. Erest2r, Erest2b, Eajacr,
// Eajacb and the axis-grid Jacobi, Section 2), terms summed in the printed
// order.
#include "dmg_launch.hpp"
#include "dmg_rows.hpp"

namespace dmg {

#define DMG_GATE(ctl) \
    if ((ctl) != nullptr && (ctl)->done) return

// -------------------------------------------- finest residual + Eq. Erest2r
// r = f - Lap_h(u) on rows [y0, y1) (written to r0 as T, squared norm
// accumulated in double), then the restriction of r onto the diagonal grid
// at the same rows.  r is formed on rows y0-1 .. y1 (halo) for the
// restriction, from u on rows y0-2 .. y1+1.
template <typename T, int CH = kChunk>
__global__ void __launch_bounds__(kRowBlock) k2_resid_a2d(int m, double inv_h2, const double* __restrict__ u,
                                                          const double* __restrict__ f, T* __restrict__ r0,
                                                          T* __restrict__ rD, double* __restrict__ partial,
                                                          int nwx, int nwaves, int rows, const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    const bool live = wv < nwaves;
    const int wx = wv % nwx, sy = wv / nwx;
    const int t = wx * kPairsPerWave - 1 + lane;
    const int y0 = 1 + sy * rows;
    const int y1 = min(y0 + rows, m);
    const bool useful = lane >= 1 && lane <= kPairsPerWave && t >= 0 && t <= m / 2;
    const size_t w = (size_t)(m + 1);
    const int W = m / 2 + 1;
    const bool c0 = t >= 1 && 2 * t <= m - 1, c1 = t >= 0 && 2 * t + 1 <= m - 1;  // columns 2t, 2t+1 interior
    const bool colok = live && t >= 0 && t <= m / 2;
    // u at columns 2t, 2t+1 of row j (column m+1 does not exist)
    auto ldu = [&](int j, double& x, double& y) {
        x = y = 0;
        if (!colok || j < 0 || j > m) return;
        const double* p = u + (size_t)j * w + 2 * t;
        if (t < m / 2) { P2<double> v = *reinterpret_cast<const P2<double>*>(p); x = v.x; y = v.y; }
        else x = p[0];
    };
    auto ldf = [&](int j, double& x, double& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        P2<double> v = *reinterpret_cast<const P2<double>*>(f + (size_t)j * w + 2 * t);
        x = v.x; y = v.y;
    };
    struct Ck { double ux[CH], uy[CH], fx[CH], fy[CH]; };
    auto load = [&](int jb, Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int j = jb + i;
            c.ux[i] = c.uy[i] = c.fx[i] = c.fy[i] = 0;
            if (j <= y1) { ldu(j + 2, c.ux[i], c.uy[i]); ldf(j, c.fx[i], c.fy[i]); }
        }
    };
    double acc = 0;
    // u rows j-1, j, j+1 of the lane's pair; r rows j-2, j-1 (as stored)
    double um0, um1, uc0, uc1, up0, up1;
    ldu(y0 - 2, um0, um1);
    ldu(y0 - 1, uc0, uc1);
    ldu(y0, up0, up1);
    T rm2_0 = 0, rm2_1 = 0, rm1_0 = 0, rm1_1 = 0;
    auto proc = [&](int jb, const Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int j = jb + i;
            if (j > y1) break;
            bool rowin = j >= 1 && j <= m - 1;
            double uW = __shfl_up(uc1, 1);   // u(2t-1, j)
            double uE = __shfl_down(uc0, 1); // u(2t+2, j)
            double x0 = c.fx[i] - (uW + um0 + uc1 + up0 - 4 * uc0) * inv_h2;
            double x1 = c.fy[i] - (uc0 + um1 + uE + up1 - 4 * uc1) * inv_h2;
            T r0j = (rowin && c0) ? (T)x0 : T(0);
            T r1j = (rowin && c1) ? (T)x1 : T(0);
            if (j >= y0 && j < y1 && useful) {
                T* p = r0 + (size_t)j * w + 2 * t;
                if (c0 && c1) { *reinterpret_cast<P2<T>*>(p) = P2<T>{r0j, r1j}; acc += x0 * x0 + x1 * x1; }
                else if (c1) { p[1] = r1j; acc += x1 * x1; }
                else if (c0) { p[0] = r0j; acc += x0 * x0; }
            }
            if (j - 1 >= y0) {
                // Eq. Erest2r at the diagonal point of row j-1 (a + j-1 even)
                int q = (j - 1) & 1;
                T sh = q ? __shfl_down(rm1_0, 1) : __shfl_up(rm1_1, 1);
                T rc = q ? rm1_1 : rm1_0;
                T rw = q ? rm1_0 : sh;
                T re = q ? sh : rm1_1;
                T rs = q ? rm2_1 : rm2_0;
                T rn = q ? r1j : r0j;
                int a = 2 * t + q;
                if (useful && a >= 1 && a <= m - 1)
                    rD[(size_t)(j - 1) * W + t] = (4 * rc + rw + rs + re + rn) * T(0.125);
            }
            rm2_0 = rm1_0; rm2_1 = rm1_1; rm1_0 = r0j; rm1_1 = r1j;
            um0 = uc0; um1 = uc1; uc0 = up0; uc1 = up1; up0 = c.ux[i]; up1 = c.uy[i];
        }
    };
    rows_march<CH, Ck>(y0 - 1, y1, load, proc);
    double sum = rows_block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}

// -------------------------------------------------- Eq. Erest2r, coarser axis grids
template <typename T, int CH = kChunk>
__global__ void __launch_bounds__(kRowBlock) k2_a2d_rows(int m, const T* __restrict__ rA, T* __restrict__ rD,
                                                         int nwx, int nwaves, int rows, const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int wx = wv % nwx, sy = wv / nwx;
    const int t = wx * kPairsPerWave - 1 + lane;
    const int y0 = 1 + sy * rows;
    const int y1 = min(y0 + rows, m);
    const bool useful = lane >= 1 && lane <= kPairsPerWave && t >= 0 && t <= m / 2;
    const bool colok = t >= 0 && t <= m / 2;
    const bool c0 = t >= 1 && 2 * t <= m - 1, c1 = t >= 0 && 2 * t + 1 <= m - 1;
    const size_t w = (size_t)(m + 1);
    const int W = m / 2 + 1;
    auto ldr = [&](int j, T& x, T& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        P2<T> v = *reinterpret_cast<const P2<T>*>(rA + (size_t)j * w + 2 * t);
        x = c0 ? v.x : T(0);
        y = c1 ? v.y : T(0);
    };
    struct Ck { T x[CH], y[CH]; };
    auto load = [&](int jb, Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            c.x[i] = c.y[i] = 0;
            if (jb + i < y1) ldr(jb + i + 1, c.x[i], c.y[i]);
        }
    };
    T rm0, rm1, rc0, rc1;
    ldr(y0 - 1, rm0, rm1);
    ldr(y0, rc0, rc1);
    auto proc = [&](int jb, const Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int j = jb + i;
            if (j >= y1) break;
            int q = j & 1;
            T sh = q ? __shfl_down(rc0, 1) : __shfl_up(rc1, 1);
            T rc = q ? rc1 : rc0;
            T rw = q ? rc0 : sh;
            T re = q ? sh : rc1;
            T rs = q ? rm1 : rm0;
            T rn = q ? c.y[i] : c.x[i];
            int a = 2 * t + q;
            if (useful && a >= 1 && a <= m - 1) rD[(size_t)j * W + t] = (4 * rc + rw + rs + re + rn) * T(0.125);
            rm0 = rc0; rm1 = rc1; rc0 = c.x[i]; rc1 = c.y[i];
        }
    };
    rows_march<CH, Ck>(y0, y1 - 1, load, proc);
}

// -------------------------------------------------- Eq. Erest2b
// diagonal grid (side m) -> axis grid (side m/2).  Lane owns coarse column A
// (lane 0 is a halo lane), marches over coarse rows B.
template <typename T, int CH = kChunk>
__global__ void __launch_bounds__(kRowBlock) k2_d2a_rows(int m, const T* __restrict__ rD, T* __restrict__ rA2,
                                                         int nwx, int nwaves, int rows, const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int mc = m / 2;
    const int wx = wv % nwx, sy = wv / nwx;
    const int A = wx * kColsPerWave - 1 + lane;
    const int B0 = 1 + sy * rows;
    const int B1 = min(B0 + rows, mc);
    const bool useful = lane >= 1 && A >= 1 && A <= mc - 1;
    const bool colok = A >= 0 && A <= mc;
    const int W = m / 2 + 1;
    auto ld = [&](int row, bool ok) -> T { return (ok && colok && row >= 0 && row <= m) ? rD[(size_t)row * W + A] : T(0); };
    struct Ck { T c[CH], h[CH]; };
    auto load = [&](int Bb, Ck& q) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int B = Bb + i;
            q.c[i] = ld(2 * B, B < B1);
            q.h[i] = ld(2 * B + 1, B < B1);
        }
    };
    T lo = ld(2 * B0 - 1, true);
    auto proc = [&](int Bb, const Ck& q) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int B = Bb + i;
            if (B >= B1) break;
            T hi = q.h[i];
            T lo_w = __shfl_up(lo, 1), hi_w = __shfl_up(hi, 1);
            // 4 r(2A,2B) + r(2A-1,2B-1) + r(2A+1,2B-1) + r(2A+1,2B+1) + r(2A-1,2B+1)
            if (useful) rA2[(size_t)B * (mc + 1) + A] = (4 * q.c[i] + lo_w + lo + hi + hi_w) * T(0.125);
            lo = hi;
        }
    };
    rows_march<CH, Ck>(B0, B1 - 1, load, proc);
}

// -------------------------------------------------- Eqs. Eajacr, Eajacb
// Jacobi on a diagonal grid (side m) from the axis grid vA2 (side m/2).
// Lane owns column A of the compacted rows: F = (2A+1, 2B+1) and C = (2A, 2B).
template <typename T, int CH = kChunk>
__global__ void __launch_bounds__(kRowBlock) k2_jdiag_rows(int m, T cc, const T* __restrict__ rD,
                                                           const T* __restrict__ vA2, T* __restrict__ vD, int nwx,
                                                           int nwaves, int rows, const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int h = m / 2;
    const int wx = wv % nwx, sy = wv / nwx;
    const int A = wx * kPairsPerWave - 1 + lane;
    const int B0 = sy * rows;          // coarse rows B: F row 2B+1 (B in [0,h-1]), C row 2B (B in [1,h-1])
    const int B1 = min(B0 + rows, h);
    const bool useful = lane >= 1 && lane <= kPairsPerWave && A >= 0 && A <= h - 1;
    const bool colok = A >= 0 && A <= h;
    const int W = m / 2 + 1;
    const size_t wc = (size_t)(h + 1);
    auto ldv = [&](int B, bool ok) -> T { return (ok && colok && B >= 0 && B <= h) ? vA2[(size_t)B * wc + A] : T(0); };
    auto ldr = [&](int row, bool ok) -> T {
        return (ok && colok && A <= h - 1 + ((row & 1) ? 0 : 1) && row >= 0 && row <= m) ? rD[(size_t)row * W + A] : T(0);
    };
    // F of the odd row 2B0-1 (needed by the C point of row 2B0)
    T vb = ldv(B0 >= 1 ? B0 - 1 : 0, true);
    T Fprev = 0;
    if (B0 >= 1) {
        T vn = ldv(B0, true);
        T rf = ldr(2 * B0 - 1, true);
        T vb_e = __shfl_down(vb, 1), vn_e = __shfl_down(vn, 1);
        Fprev = (-cc * rf + vb + vb_e + vn_e + vn) * T(0.25);
        vb = vn;
    }
    struct Ck { T v[CH], rf[CH], rc[CH]; };
    auto load = [&](int Bb, Ck& q) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int B = Bb + i;
            bool in = B < B1;
            q.v[i] = ldv(B + 1, in);
            q.rf[i] = ldr(2 * B + 1, in);
            q.rc[i] = ldr(2 * B, in);
        }
    };
    auto proc = [&](int Bb, const Ck& q) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int B = Bb + i;
            if (B >= B1) break;
            T vn = q.v[i];
            T vb_e = __shfl_down(vb, 1), vn_e = __shfl_down(vn, 1);
            // v_{i-1,j-1} + v_{i+1,j-1} + v_{i+1,j+1} + v_{i-1,j+1} on the coarse grid
            T F = (-cc * q.rf[i] + vb + vb_e + vn_e + vn) * T(0.25);
            T Fw = __shfl_up(F, 1), Fpw = __shfl_up(Fprev, 1);
            if (useful) {
                vD[(size_t)(2 * B + 1) * W + A] = F;
                if (B >= 1 && A >= 1) vD[(size_t)(2 * B) * W + A] = (-cc * q.rc[i] + Fpw + Fprev + F + Fw) * T(0.25);
            }
            Fprev = F;
            vb = vn;
        }
    };
    rows_march<CH, Ck>(B0, B1 - 1, load, proc);
}

// ---------------------------------------- axis-grid Jacobi (+ u update on the finest)
// F points (a+b odd) from the diagonal grid vD of the same side, then C
// points (a+b even) from the new F values.  FINEST: u <- u + v instead of
// storing v.
template <typename T, bool FINEST, int CH = kChunk>
__global__ void __launch_bounds__(kRowBlock) k2_jaxis_rows(int m, T cc, const T* __restrict__ rA,
                                                           const T* __restrict__ vD, T* __restrict__ vA,
                                                           double* __restrict__ u, int nwx, int nwaves, int rows,
                                                           const Ctl* ctl)
{
    DMG_GATE(ctl);
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int wx = wv % nwx, sy = wv / nwx;
    const int t = wx * kPairsPerWave - 1 + lane;
    const int y0 = 1 + sy * rows;
    const int y1 = min(y0 + rows, m);
    const bool useful = lane >= 1 && lane <= kPairsPerWave && t >= 0 && t <= m / 2;
    const bool colok = t >= 0 && t <= m / 2;
    const bool c0 = t >= 1 && 2 * t <= m - 1, c1 = t >= 0 && 2 * t + 1 <= m - 1;  // columns 2t, 2t+1 interior
    const size_t w = (size_t)(m + 1);
    const int W = m / 2 + 1;
    auto ldD = [&](int j) -> T { return (colok && j >= 0 && j <= m) ? vD[(size_t)j * W + t] : T(0); };
    // a pair of an interior row: columns 2t, 2t+1 exist for t <= m/2 (column m+1
    // is the next row's column 0 and is never used)
    auto ldR = [&](int j, T& x, T& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        P2<T> v = *reinterpret_cast<const P2<T>*>(rA + (size_t)j * w + 2 * t);
        x = c0 ? v.x : T(0);
        y = c1 ? v.y : T(0);
    };
    struct Ck { T d[CH], rx[CH], ry[CH]; double ux[CH], uy[CH]; };
    auto load = [&](int jb, Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int j = jb + i;
            c.d[i] = c.rx[i] = c.ry[i] = 0;
            c.ux[i] = c.uy[i] = 0;
            if (j <= y1) {
                c.d[i] = ldD(j + 1);
                ldR(j, c.rx[i], c.ry[i]);
                if (FINEST && useful && j >= y0 && j < y1 && (c0 || c1)) {
                    P2<double> v = *reinterpret_cast<const P2<double>*>(u + (size_t)j * w + 2 * t);
                    c.ux[i] = v.x;
                    c.uy[i] = v.y;
                }
            }
        }
    };
    // window entering row j: vD rows j-1, j; F rows j-2, j-1; r at the C point
    // of row j-1; u pair of row j-1
    T dm = ldD(y0 - 2), d0 = ldD(y0 - 1);
    T Fm2 = 0, Fm1 = 0, rCm1 = 0;
    double uxm1 = 0, uym1 = 0;
    auto proc = [&](int jb, const Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int j = jb + i;
            if (j > y1) break;
            T dp = c.d[i];
            int q = j & 1;
            T rF = q ? c.rx[i] : c.ry[i];   // F column 2t+1-q
            T rC = q ? c.ry[i] : c.rx[i];   // C column 2t+q
            // F at row j: vd[a-1,b] + vd[a,b-1] + vd[a+1,b] + vd[a,b+1]
            T nb = q ? __shfl_up(d0, 1) : __shfl_down(d0, 1);
            T vw = q ? nb : d0;
            T ve = q ? d0 : nb;
            int aF = 2 * t + 1 - q;
            T Fj = (aF >= 1 && aF <= m - 1 && j >= 1 && j <= m - 1) ? (-cc * rF + vw + dm + ve + dp) * T(0.25) : T(0);
            if (j - 1 >= y0) {
                int qq = (j - 1) & 1;
                T sb = qq ? __shfl_down(Fm1, 1) : __shfl_up(Fm1, 1);
                T cw = qq ? Fm1 : sb;
                T ce = qq ? sb : Fm1;
                T C = (-cc * rCm1 + cw + Fm2 + ce + Fj) * T(0.25);
                T vx = qq ? Fm1 : C;   // column 2t
                T vy = qq ? C : Fm1;   // column 2t+1
                size_t o = (size_t)(j - 1) * w + 2 * t;
                if (useful) {
                    if (FINEST) {
                        if (c0 && c1) *reinterpret_cast<P2<double>*>(u + o) = P2<double>{uxm1 + (double)vx, uym1 + (double)vy};
                        else if (c1) u[o + 1] = uym1 + (double)vy;
                        else if (c0) u[o] = uxm1 + (double)vx;
                    } else {
                        if (c0 && c1) *reinterpret_cast<P2<T>*>(vA + o) = P2<T>{vx, vy};
                        else if (c1) vA[o + 1] = vy;
                        else if (c0) vA[o] = vx;
                    }
                }
            }
            Fm2 = Fm1; Fm1 = Fj; rCm1 = rC;
            dm = d0; d0 = dp;
            uxm1 = c.ux[i]; uym1 = c.uy[i];
        }
    };
    rows_march<CH, Ck>(y0 - 1, y1, load, proc);
}

// ------------------------------------------------------------- launchers
// Strip length: the longest (fewest halo rows) that still gives the grid
// about `target` waves, so every wave is resident in one round.  Chunk depth
// per kernel from a sweep on MI355X at the 4097^2 level sizes.
constexpr int kChunkResid = 2, kChunkA2D = 1, kChunkD2A = 4, kChunkJDiag = 2, kChunkJAxis = 1;
constexpr int kTargetWavesResid = 8192;  // ~120 VGPRs: 16 waves per CU

static inline int pick_rows(int ncols_units, int per_wave, int nrows, int target = kTargetWaves)
{
    int nwx = (ncols_units + per_wave - 1) / per_wave;
    int r = kMaxRows;
    while (r > 4 && (long)nwx * ((nrows + r - 1) / r) < target) r >>= 1;
    return r;
}

static inline void rows_grid(int ncols_units, int per_wave, int nrows, int rows, int& nwx, int& nwaves, int& nblocks)
{
    nwx = (ncols_units + per_wave - 1) / per_wave;
    int nsy = (nrows + rows - 1) / rows;
    nwaves = nwx * nsy;
    nblocks = (nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
}

int rows_resid_parts(int n)
{
    int nwx, nw, nb;
    rows_grid(n / 2 + 1, kPairsPerWave, n - 1, pick_rows(n / 2 + 1, kPairsPerWave, n - 1, kTargetWavesResid), nwx,
              nw, nb);
    return nb;
}

template <typename T>
void launch_resid_a2d(int n, const double* u, const double* f, T* r0, T* rD, double* partial, const Ctl* ctl,
                      hipStream_t s)
{
    int nwx, nw, nb;
    int rows = pick_rows(n / 2 + 1, kPairsPerWave, n - 1, kTargetWavesResid);
    rows_grid(n / 2 + 1, kPairsPerWave, n - 1, rows, nwx, nw, nb);
    hipLaunchKernelGGL((k2_resid_a2d<T, kChunkResid>), dim3(nb), dim3(kRowBlock), 0, s, n, (double)n * (double)n,
                       u, f, r0, rD, partial, nwx, nw, rows, ctl);
}

template <typename T>
void launch_rs2_rows(int diag_in, int m, const T* in, T* out, const Ctl* ctl, hipStream_t s)
{
    int nwx, nw, nb;
    if (!diag_in) {
        int rows = pick_rows(m / 2 + 1, kPairsPerWave, m - 1);
        rows_grid(m / 2 + 1, kPairsPerWave, m - 1, rows, nwx, nw, nb);
        hipLaunchKernelGGL((k2_a2d_rows<T, kChunkA2D>), dim3(nb), dim3(kRowBlock), 0, s, m, in, out, nwx, nw, rows,
                           ctl);
    } else {
        int rows = pick_rows(m / 2 + 1, kColsPerWave, m / 2 - 1);
        rows_grid(m / 2 + 1, kColsPerWave, m / 2 - 1, rows, nwx, nw, nb);
        hipLaunchKernelGGL((k2_d2a_rows<T, kChunkD2A>), dim3(nb), dim3(kRowBlock), 0, s, m, in, out, nwx, nw, rows,
                           ctl);
    }
}

template <typename T>
void launch_jac2_rows(int diag, int m, T c, const T* r, const T* vc, T* v, const Ctl* ctl, hipStream_t s)
{
    int nwx, nw, nb;
    if (diag) {
        int rows = pick_rows(m / 2, kPairsPerWave, m / 2);
        rows_grid(m / 2, kPairsPerWave, m / 2, rows, nwx, nw, nb);
        hipLaunchKernelGGL((k2_jdiag_rows<T, kChunkJDiag>), dim3(nb), dim3(kRowBlock), 0, s, m, c, r, vc, v, nwx, nw,
                           rows, ctl);
    } else {
        int rows = pick_rows(m / 2 + 1, kPairsPerWave, m - 1);
        rows_grid(m / 2 + 1, kPairsPerWave, m - 1, rows, nwx, nw, nb);
        hipLaunchKernelGGL((k2_jaxis_rows<T, false, kChunkJAxis>), dim3(nb), dim3(kRowBlock), 0, s, m, c, r, vc, v,
                           (double*)nullptr, nwx, nw, rows, ctl);
    }
}

template <typename T>
void launch_jac2_finest_rows(int n, T c, const T* r0, const T* vD, double* u, const Ctl* ctl, hipStream_t s)
{
    int nwx, nw, nb;
    int rows = pick_rows(n / 2 + 1, kPairsPerWave, n - 1);
    rows_grid(n / 2 + 1, kPairsPerWave, n - 1, rows, nwx, nw, nb);
    hipLaunchKernelGGL((k2_jaxis_rows<T, true, kChunkJAxis>), dim3(nb), dim3(kRowBlock), 0, s, n, c, r0, vD,
                       (T*)nullptr, u, nwx, nw, rows, ctl);
}

#define DMG_INST2R(T)                                                                                          \
    template void launch_resid_a2d<T>(int, const double*, const double*, T*, T*, double*, const Ctl*,         \
                                      hipStream_t);                                                            \
    template void launch_rs2_rows<T>(int, int, const T*, T*, const Ctl*, hipStream_t);                        \
    template void launch_jac2_rows<T>(int, int, T, const T*, const T*, T*, const Ctl*, hipStream_t);           \
    template void launch_jac2_finest_rows<T>(int, T, const T*, const T*, double*, const Ctl*, hipStream_t);
DMG_INST2R(double)
DMG_INST2R(float)

}  // namespace dmg

// 2D kernels of libdmg (Roberts, Section 2), driven by work items so that a
// single launch per level serves a batch of independent problems.
//
// Large levels (side >= 512) use row-marching kernels: a wavefront owns a
// band of columns and marches down a strip of rows holding a register window
// of a few rows; on an axis grid each lane owns the column pair (2t, 2t+1)
// (one point of each colour per row), so both half-sweeps of the red-black
// Jacobi run in one launch, the value needed from the neighbouring pair
// comes across lanes by shuffle, and the lanes at the band's edges are halo
// lanes so no value crosses a wave.  Loads are double-buffered (rows_march)
// and pairs move as one 16-byte access.  The finest residual also restricts
// onto the next two levels, the finest Jacobi runs the diagonal level's
// below it on the fly, and in single-problem plans the levels >= 16 restrict
// and relax two at a time (kb_rs_pair, kb_jac_pair).  Levels of sides 64 ..
// 256 of a single problem run in two tiled launches (kb_mid_down,
// kb_mid_up); small levels otherwise use one thread per point, and levels of
// side <= 32 run in one workgroup per problem (kb_coarse).
//
// Per point the arithmetic is the paper's: Eqs. (Erest2r), (Erest2b),
// (Eajacr), (Eajacb) and the axis-grid Jacobi, terms in the printed order.
#include "dmg_b2d.hpp"
#include "dmg_host.hpp"
#include "dmg_net_dev.hpp"
#include "dmg_rows.hpp"

#include <hip/hip_ext.h>

#include <map>
#include <mutex>

namespace dmg {

#define ITEM_GATE(ctls, prob) \
    if ((ctls)[(prob)].done) return

// ====================================================================== finest

// r = f - Lap_h(u) on rows [y0, y1) (stored as T, squared norm accumulated
// in double), then Eq. (Erest2r) onto the first diagonal level at those rows.
// FZ: Eq. (Erest2b) onto the axis level below it, from the diagonal values
// of three consecutive rows kept in registers (the strip then computes one
// diagonal row past its end; strips start on odd rows), and the diagonal
// level itself is not stored: the finest Jacobi restricts it again from r.
// Lane t owns the column pair (2t, 2t+1); a diagonal value needs the lanes
// beside it, and an FZ value the lanes beside those: lanes 1 .. 61 write r
// and r1, lanes 2 .. 62 write r2.
// NT: non-temporal f, r0 and r1 accesses (r0 and r1 are next read by the
// finest kernel, after the whole cycle: kept out of the caches, they leave
// them to the level arrays in between).  At most 128 VGPRs (four waves per
// SIMD keep enough loads in flight); the FP64 FZ variant needs a few more
// and runs three waves rather than spill (measured faster than halving its
// row chunk to stay at four).
// M4: the fourth-order residual of Section 2.3, Eq. (Efos2): f holds the
// right-hand side combination (8f + 4 neighbours)/12, made once per solve by
// kb_rhs4, and inv_h2 is 1/(6h^2) for the 9-point operator; the extra
// diagonal neighbours come from the rows already held, by neighbour-lane
// reads (its FZ variants run three waves per SIMD in both precisions).
// WF: the partial sums of f^2 over the same interior points too (the first
// evaluation of a solve, so that ||f|| needs no pass of its own).
// MIR (FZ strips of odd index): the strip is marched from its last row to
// its first, as the same march over the grid mirrored in y (rows m - j; m is
// even, so parities are unchanged); the stencil operands are passed in the
// unmirrored order, so every value has the same bits.  Two neighbouring
// strips then reach the halo rows they share at the same time, while those
// rows are still in L2.  A mirrored strip starts on an even row, so it
// computes one diagonal row before its start instead of one past its end.
// st0 = false (out-of-place solves): r is formed, restricted and summed but
// not stored.
constexpr int kResidPairs = 61;

// Eq. (Evpois): the residual at columns 2t, 2t+1 of one row from f there and
// u at the lane's pair (c), the grid row south (s) and north (n) of it and the
// columns 2t-1 (W) and 2t+2 (E); one expression for every kernel that forms
// it, so that they all get the same bits
__device__ inline void resid_pair(double inv_h2, double fx, double fy, double uW, double us0, double us1, double uc0,
                                  double uc1, double un0, double un1, double uE, double& x0, double& x1)
{
    x0 = fx - (uW + us0 + uc1 + un0 - 4 * uc0) * inv_h2;
    x1 = fy - (uc0 + us1 + uE + un1 - 4 * uc1) * inv_h2;
}

template <typename T, int CH, bool NT, bool FZ, bool M4, bool WF, bool MIR>
__device__ inline void resid_body(int m, double inv_h2, const Fin2<T>& it, const double* __restrict__ u, bool st0,
                                  int wv, int nwx, int rows, double& acc, double& accf)
{
    const auto f = gmem(it.f);
    const auto r0 = gmem(it.r0);
    const auto rD = gmem(it.r1);
    const auto rA2 = gmem(it.r2);
    const auto ug = gmem(u);
    const int lane = threadIdx.x & 63;
    const int wx = wv % nwx, sy = wv / nwx;
    const int t = wx * kResidPairs - 1 + lane;
    const int ya = 1 + sy * rows, yb = min(ya + rows, m);   // the strip's grid rows [ya, yb)
    const int y0 = MIR ? m - yb + 1 : ya;                   // the same rows as marched
    const int y1 = MIR ? m - ya + 1 : yb;
    const int dlo = MIR ? y0 - 1 : y0;                      // first diagonal row computed
    const int ylast = FZ && !MIR ? y1 + 1 : y1;             // last row of the march
    const int mc = m / 2;
    auto R = [&](int j) { return MIR ? m - j : j; };        // marched row -> grid row
    const bool useful = lane >= 1 && lane <= kResidPairs && t >= 0 && t <= m / 2;
    const bool useful2 = lane >= 2 && lane <= kResidPairs + 1 && t >= 1 && t <= mc - 1;
    const size_t w = (size_t)(m + 1);
    const int W = m / 2 + 1;
    const bool c0 = t >= 1 && 2 * t <= m - 1, c1 = t >= 0 && 2 * t + 1 <= m - 1;  // columns 2t, 2t+1 interior
    const bool colok = t >= 0 && t <= m / 2;
    // u at columns 2t, 2t+1 of marched row j (column m+1 does not exist)
    auto ldu = [&](int j, double& x, double& y) {
        x = y = 0;
        if (!colok || j < 0 || j > m) return;
        const auto p = ug + (size_t)R(j) * w + 2 * t;
        if (t < m / 2) { P2<double> v = ld_pair(p); x = v.x; y = v.y; }
        else x = p[0];
    };
    auto ldf = [&](int j, double& x, double& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        const auto q = f + (size_t)R(j) * w + 2 * t;
        P2<double> v = NT ? ld_pair_nt(q) : ld_pair(q);
        x = v.x; y = v.y;
    };
    struct Ck { double ux[CH], uy[CH], fx[CH], fy[CH]; };
    auto load = [&](int jb, Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            int j = jb + i;
            c.ux[i] = c.uy[i] = c.fx[i] = c.fy[i] = 0;
            if (j <= ylast) { ldu(j + 2, c.ux[i], c.uy[i]); ldf(j, c.fx[i], c.fy[i]); }
        }
    };
    const int jstart = dlo - 1;   // r rows from dlo - 1 on make the diagonal rows from dlo on
    double um0, um1, uc0, uc1, up0, up1;  // u rows j-1, j, j+1 (marched) of the lane's pair
    ldu(jstart - 1, um0, um1);
    ldu(jstart, uc0, uc1);
    ldu(jstart + 1, up0, up1);
    T rm2_0 = 0, rm2_1 = 0, rm1_0 = 0, rm1_1 = 0;  // r rows j-2, j-1 (as stored)
    T d3 = 0, d2 = 0;                               // FZ: diagonal values of rows j-3, j-2
    // P0: parity of jb (-1: not known at compile time).  With the vector
    // stores of NT, a select on a run-time parity between the two values of a
    // stored pair became a dynamically indexed vector kept in scratch memory.
    auto proc_p = [&](int jb, const Ck& c, auto P0) {
        static_for<0, CH>([&](auto I) {
            constexpr int i = decltype(I)::value;
            // rows of the last chunk past ylast are computed too: every output
            // below is guarded by its row range, and without an early exit per
            // row the compiler keeps the row window in place instead of
            // copying it on every row
            const int j = jb + i;
            bool rowin = j >= 1 && j <= m - 1;
            double uW = lane_up(uc1);   // u(2t-1, j)
            double uE = lane_down(uc0); // u(2t+2, j)
            // grid south / north rows of the lane's pair (marched j-1 / j+1 unless mirrored)
            const double us0 = MIR ? up0 : um0, us1 = MIR ? up1 : um1;
            const double un0 = MIR ? um0 : up0, un1 = MIR ? um1 : up1;
            double x0, x1;
            if constexpr (M4) {
                // Eq. (Efos2): -20 centre, 4 x (S, N, W, E), then NE, NW, SW, SE
                const double mW = lane_up(um1), mE = lane_down(um0);   // marched row j-1, columns 2t-1, 2t+2
                const double pW = lane_up(up1), pE = lane_down(up0);   // marched row j+1
                const double sW = MIR ? pW : mW, sE = MIR ? pE : mE;            // grid south row
                const double nW = MIR ? mW : pW, nE = MIR ? mE : pE;            // grid north row
                x0 = c.fx[i] - (-20 * uc0 + 4 * (us0 + un0 + uW + uc1) + un1 + nW + sW + us1) * inv_h2;
                x1 = c.fy[i] - (-20 * uc1 + 4 * (us1 + un1 + uc0 + uE) + nE + un0 + us0 + sE) * inv_h2;
            } else {
                resid_pair(inv_h2, c.fx[i], c.fy[i], uW, us0, us1, uc0, uc1, un0, un1, uE, x0, x1);
            }
            T r0j = (rowin && c0) ? (T)x0 : T(0);
            T r1j = (rowin && c1) ? (T)x1 : T(0);
            if (j >= y0 && j < y1 && useful) {
                const auto p = r0 + (size_t)R(j) * w + 2 * t;
                if (c0 && c1) {
                    if (st0) {
                        if (NT) st_pair_nt(p, r0j, r1j);
                        else st_pair(p, r0j, r1j);
                    }
                    acc += x0 * x0 + x1 * x1;
                    if constexpr (WF) accf += c.fx[i] * c.fx[i] + c.fy[i] * c.fy[i];
                }
                else if (c1) {
                    if (st0) p[1] = r1j;
                    acc += x1 * x1;
                    if constexpr (WF) accf += c.fy[i] * c.fy[i];
                }
                else if (c0) {
                    if (st0) p[0] = r0j;
                    acc += x0 * x0;
                    if constexpr (WF) accf += c.fx[i] * c.fx[i];
                }
            }
            if (j - 1 >= dlo) {
                // Eq. Erest2r at the diagonal point of row j-1 (a + j-1 even)
                constexpr int p0 = decltype(P0)::value;
                const int q = p0 >= 0 ? (p0 + i + 1) & 1 : (j - 1) & 1;
                T sh = q ? lane_down(rm1_0) : lane_up(rm1_1);
                T rc = q ? rm1_1 : rm1_0;
                T rw = q ? rm1_0 : sh;
                T re = q ? sh : rm1_1;
                T rlo = q ? rm2_1 : rm2_0;   // marched row j-2
                T rhi = q ? r1j : r0j;       // marched row j
                int a = 2 * t + q;
                const T d1 = MIR ? rs2_core(rc, rw, rhi, re, rlo) : rs2_core(rc, rw, rlo, re, rhi);
                if (!FZ && useful && a >= 1 && a <= m - 1 && j - 1 < y1) {
                    if (NT) __builtin_nontemporal_store(d1, rD + (size_t)R(j - 1) * W + t);
                    else rD[(size_t)R(j - 1) * W + t] = d1;
                }
                if constexpr (FZ) {
                    // Eq. (Erest2b) at axis point (t, B) of the level below,
                    // B = (j-2)/2: diagonal rows 2B-1 (d3), 2B (d2), 2B+1 (d1)
                    // as marched (mirrored: 2B+1, 2B, 2B-1 of the grid)
                    if (!(j & 1) && j - 2 >= y0 && j - 2 < y1) {
                        const int B = (j - 2) >> 1;
                        const T d3w = lane_up(d3), d1w = lane_up(d1);
                        if (useful2 && B >= 1 && B <= mc - 1)
                            rA2[(size_t)(MIR ? mc - B : B) * (mc + 1) + t] =
                                MIR ? rs2_core(d2, d1w, d1, d3, d3w) : rs2_core(d2, d3w, d3, d1, d1w);
                    }
                    d3 = d2;
                    d2 = d1;
                }
            }
            rm2_0 = rm1_0; rm2_1 = rm1_1; rm1_0 = r0j; rm1_1 = r1j;
            um0 = uc0; um1 = uc1; uc0 = up0; uc1 = up1; up0 = c.ux[i]; up1 = c.uy[i];
        });
    };
    auto proc = [&](int jb, const Ck& c) {
        if constexpr (NT) {
            if (jb & 1) proc_p(jb, c, Int<1>{});
            else proc_p(jb, c, Int<0>{});
        } else {
            proc_p(jb, c, Int<-1>{});   // run-time parity (no vector stores here)
        }
    };
    rows_march<CH, Ck>(jstart, ylast, load, proc);
}

template <typename T, int CH, bool NT, bool FZ, bool M4, bool WF>
__global__ void __launch_bounds__(kRowBlock) __attribute__((amdgpu_waves_per_eu((FZ && (sizeof(T) == 8 || M4)) || WF ? 3 : 4))) kb_resid(int m, double inv_h2, const Fin2<T>* __restrict__ items,
                                                      int nwx, int nwaves, int rows, const Ctl* __restrict__ ctls,
                                                      int oop)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const int wv = rows_wave_id(nwaves);
    // out of place: evaluation k reads the iterate of cycle k (u for even k, ub for odd k)
    const bool pp = oop && it.ub;
    const double* uk = pp && (ctls[it.prob].k & 1) ? it.ub : it.u;
    double acc = 0, accf = 0;
    if (wv < nwaves) {
        if (FZ && ((wv / nwx) & 1)) resid_body<T, CH, NT, FZ, M4, WF, true>(m, inv_h2, it, uk, !pp, wv, nwx, rows, acc, accf);
        else resid_body<T, CH, NT, FZ, M4, WF, false>(m, inv_h2, it, uk, !pp, wv, nwx, rows, acc, accf);
    }
    double sum = rows_block_sum(acc);
    if (threadIdx.x == 0) it.part[blockIdx.x] = sum;
    if constexpr (WF) {
        __syncthreads();   // the block sum's shared slots are reused
        double sf = rows_block_sum(accf);
        if (threadIdx.x == 0) it.partf[blockIdx.x] = sf;
    }
}

// One-thread-per-point residual for tiny grids (side < 4: no diagonal level);
// m4: the fourth-order residual as in kb_resid.
template <typename T>
__global__ void kb_resid_small(int n, double inv_h2, const Fin2<T>* __restrict__ items, const Ctl* __restrict__ ctls,
                               int m4)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    double acc = 0;
    size_t s = (size_t)n + 1;
    for (int q = threadIdx.x; q < (n - 1) * (n - 1); q += blockDim.x) {
        int a = q % (n - 1) + 1, b = q / (n - 1) + 1;
        size_t c = (size_t)b * s + a;
        const double* u = it.u;
        double lap = m4 ? (-20 * u[c] + 4 * (u[c - s] + u[c + s] + u[c - 1] + u[c + 1]) + u[c + 1 + s] +
                           u[c - 1 + s] + u[c - 1 - s] + u[c + 1 - s]) * inv_h2
                        : (u[c - 1] + u[c - s] + u[c + 1] + u[c + s] - 4 * u[c]) * inv_h2;
        double r = it.f[c] - lap;
        it.r0[c] = (T)r;
        acc += r * r;
    }
    double sum = rows_block_sum(acc);
    if (threadIdx.x == 0) it.part[0] = sum;
}

// The right-hand side combination of the fourth-order residual (Section 2.3,
// Eq. Efos2): g = (8 f + f(E) + f(N) + f(W) + f(S)) / 12 at interior nodes,
// made once per solve; reads f on boundary nodes too.  One thread per point,
// x fastest.
__global__ void kb_rhs4(int n, const double* __restrict__ f, double* __restrict__ g)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int b = blockIdx.y + 1;
    if (a > n - 1) return;
    const size_t s = (size_t)n + 1, c = (size_t)b * s + a;
    g[c] = (8 * f[c] + f[c + 1] + f[c + s] + f[c - 1] + f[c - s]) / 12;
}

// sum of f^2 over interior nodes, per problem (same partial count as kb_resid)
template <typename T>
__global__ void __launch_bounds__(kRowBlock) kb_sumsq(int n, const Fin2<T>* __restrict__ items,
                                                      const Ctl* __restrict__ ctls)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const size_t s = (size_t)n + 1;
    double acc = 0;
    // interior rows b = blockIdx.x + 1, + gridDim.x, ...; a row's columns
    // across the block's threads (coalesced, no division per element)
    for (int b = blockIdx.x + 1; b < n; b += gridDim.x) {
        const double* __restrict__ row = it.f + (size_t)b * s;
        for (int a = threadIdx.x + 1; a < n; a += blockDim.x) {
            const double x = row[a];
            acc += x * x;
        }
    }
    double sum = rows_block_sum(acc);
    if (threadIdx.x == 0) it.part[blockIdx.x] = sum;
}

// finest axis-grid Jacobi fused with u <- u + v (Section 1), row-marching
template <typename T, bool FINEST, int CH, bool NT>
__device__ inline void jaxis_body(int m, T cc, const T* __restrict__ rA, const T* __restrict__ vD,
                                  T* __restrict__ vA, double* __restrict__ u, int nwx, int nwaves, int rows)
{
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
    auto ldD = [&](int j) -> T { return (colok && j >= 0 && j <= m) ? vD[(size_t)j * W + t] : T(0); };
    // pair of an interior row: column m+1 is the next row's column 0 and never used
    auto ldR = [&](int j, T& x, T& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        P2<T> v = (FINEST && NT) ? ld_pair_nt(rA + (size_t)j * w + 2 * t) : *reinterpret_cast<const P2<T>*>(rA + (size_t)j * w + 2 * t);
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
    // window entering row j: vD rows j-1, j; F rows j-2, j-1; r at the C point of row j-1; u of row j-1
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
            T rF = q ? c.rx[i] : c.ry[i];  // F at column 2t+1-q
            T rC = q ? c.ry[i] : c.rx[i];  // C at column 2t+q
            // F at row j: vd[a-1,b] + vd[a,b-1] + vd[a+1,b] + vd[a,b+1]
            T nb = q ? __shfl_up(d0, 1) : __shfl_down(d0, 1);
            T vw = q ? nb : d0;
            T ve = q ? d0 : nb;
            int aF = 2 * t + 1 - q;
            T Fj = (aF >= 1 && aF <= m - 1 && j >= 1 && j <= m - 1) ? jac2_sum(cc, rF, vw, dm, ve, dp) : T(0);
            if (j - 1 >= y0) {
                int qq = (j - 1) & 1;
                T sb = qq ? __shfl_down(Fm1, 1) : __shfl_up(Fm1, 1);
                T cw = qq ? Fm1 : sb;
                T ce = qq ? sb : Fm1;
                T C = jac2_sum(cc, rCm1, cw, Fm2, ce, Fj);
                T vx = qq ? Fm1 : C;  // column 2t
                T vy = qq ? C : Fm1;  // column 2t+1
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

template <typename T, int CH, bool NT>
__global__ void __launch_bounds__(kRowBlock) kb_finest(int m, T cc, const Fin2<T>* __restrict__ items, int nwx,
                                                       int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    jaxis_body<T, true, CH, NT>(m, cc, it.r0, it.v1, nullptr, it.u, nwx, nwaves, rows);
}

// Axis Jacobi fused with the Jacobi of the diagonal level below it (Eqs.
// (Eajacr), (Eajacb)); on the finest level (D, below it D-1) also with
// u <- u + v (Section 1).  The
// diagonal level's new values are computed in the row march instead of being
// stored by one kernel and read by the next: a lane's diagonal point of row
// k is (2t + (k&1), k); F points (odd rows) come from two rows of the
// coarser axis level v2 (columns t, t+1), C points (even rows) from the F
// values of the rows above and below (lanes t-1, t), so the F row k+1 is
// computed one row ahead.  The diagonal level's residual is not read
// either: it is restricted (Eq. Erest2r) from the axis residual rows the
// march holds anyway (a window of three row pairs, loaded two rows ahead),
// so the residual kernel and kb_rs_pair do not store it.  These extra
// neighbour dependencies leave lanes 2 .. 61 to write u (lanes 0, 1, 62, 63
// are halo; a restricted value at lane 0 of an even row or lane 63 of an
// odd row lacks its outer neighbour and reaches no written point).  Same
// arithmetic cores as the per-level kernels: the results are bit-identical
// to restricting, running the diagonal Jacobi and then kb_finest.
constexpr int kFusePairs = 60;

// FINEST: add the axis values to u (else store them in vA).
// MIR (odd strips): the strip is marched from its last row to its first, as
// the same march over the grid mirrored in y (rows m - j; m is even, so row
// parities and the F/C structure are unchanged); the stencil operands are
// passed in the unmirrored order, so the values are the same bits.  Two
// neighbouring strips then reach the rows they share at the same time (both
// at their start or both at their end), while those rows are still in L2.
// PP (FINEST; out-of-place solves, levels of type T, the residual formed in
// double): the axis residual rows are not read but formed from the previous
// iterate uc and f (Eq. Evpois, the residual kernel's expression: the same
// bits, rounded to T as it rounds them), and the new iterate uc + v goes to u,
// another buffer, so no workgroup ever reads a value another one has
// updated.  The lane's u pairs of the rows it has loaded stay in registers
// (five rows) for the update; lanes 0 and 63 also load the one column beyond
// the band that their residual needs.
// RES (with PP): the kernel also forms the new iterate's residual, its norm
// partials and its two restrictions (Eqs. Erest2r, Erest2b) onto the axis
// level below the first diagonal one (rA2), as the residual kernel does for
// the next evaluation, from the new iterate's rows while they are still in
// registers.  The residual rows trail the Jacobi rows by two, the march
// starts three or four rows before the strip's first row and ends three or
// four rows past its last (the new iterate is formed, not written, there),
// and a wave owns 57 column pairs, lanes 4 .. 60: the new iterate is right in
// lanes 2 .. 61, its residual in 3 .. 60, the diagonal restriction in 3 .. 60
// and the axis one, which takes the diagonal values of the lane to the west,
// in 4 .. 60.
// Strips must start on odd rows (an even strip length), as in the residual
// kernel.  Returns the lane's part of the squared norm.
constexpr int kResPairs = 57;
// s_waitcnt operand of a wait for every vector-memory access (vmcnt 0, the
// export and LDS counts at their maxima; the GFX9 field layout)
constexpr int kWaitVmem0 = 0xF70;
// INNER: every lane's column pair t lies in 1 .. m/2 - 1 (a band away from
// both boundary columns), so every column check holds and folds away.
template <typename T, bool FINEST, bool NT, bool MIR, bool PP = false, bool RES = false, bool INNER = false>
__device__ inline double fused_body(int m, T cc, T cd, const T* __restrict__ rA, const T* __restrict__ v2,
                                    T* __restrict__ vA, double* __restrict__ u, int wv, int nwx, int rows,
                                    const double* __restrict__ uc = nullptr, const double* __restrict__ fr = nullptr,
                                    T* __restrict__ rA2 = nullptr)
{
    static_assert(!RES || (PP && FINEST), "the residual of the new iterate needs the out-of-place finest step");
    constexpr int kStride = RES ? kResPairs : kFusePairs, kLane0 = RES ? 4 : 2;
    const int lane = threadIdx.x & 63;
    const int wx = wv % nwx, sy = wv / nwx;
    const int t = wx * kStride - kLane0 + lane;
    const int ya = 1 + sy * rows, yb = min(ya + rows, m);   // the strip's rows [ya, yb)
    const int y0 = MIR ? m - yb + 1 : ya;                   // the same rows as marched
    const int y1 = MIR ? m - ya + 1 : yb;
    const int h = m / 2, W = h + 1;   // row length of v2 (side m/2)
    auto R = [&](int k) { return MIR ? m - k : k; };       // marched row -> grid row
    auto RB = [&](int B) { return MIR ? h - B : B; };      // the same on the level of side m/2
    const bool useful = lane >= kLane0 && lane < kStride + kLane0 && (INNER || (t >= 0 && t <= h));
    // RES: the residual rows [jstart, ylast] and the first diagonal row dlo, as
    // the residual kernel takes them (strips start on odd grid rows); the march
    // rows [jbeg, jend]
    const int dlo = MIR ? y0 - 1 : y0, jstart = dlo - 1, ylast = MIR ? y1 : y1 + 1;
    const int jbeg = RES ? jstart - 2 : y0 - 1, jend = RES ? ylast + 2 : y1;
    const bool colok = INNER || (t >= 0 && t <= h);
    const bool c0 = INNER || (t >= 1 && 2 * t <= m - 1), c1 = INNER || (t >= 0 && 2 * t + 1 <= m - 1);
    const size_t w = (size_t)(m + 1);
    const auto rAg = gmem(rA), v2g = gmem(v2);
    const auto ucg = gmem(uc), frg = gmem(fr);
    const auto vAg = gmem(vA), rA2g = gmem(rA2);
    const auto ug = gmem(u);
    auto ld2 = [&](int B) -> T { return (colok && B >= 0 && B <= h) ? v2g[(size_t)RB(B) * W + t] : T(0); };
    // pair of an interior row: column m+1 is the next row's column 0 and never used
    auto ldR = [&](int j, T& x, T& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        const auto p = rAg + (size_t)R(j) * w + 2 * t;
        P2<T> v = (FINEST && NT) ? ld_pair_nt(p) : ld_pair(p);
        x = c0 ? v.x : T(0);
        y = c1 ? v.y : T(0);
    };
    // Eq. (Erest2r) at the lane's diagonal point (2t + q, k) of marched row k
    // (Q: Int<q>, q = k & 1; grid row R(k) has the parity of k, m being even)
    // from the axis residual pairs of marched rows k-1 (m), k (c), k+1 (p),
    // the operands in grid order (south = the lower grid row); the same bits
    // as the stored restriction of the residual kernels
    auto rs1 = [&](auto Q, T mx, T my, T cx, T cy, T px, T py) -> T {
        if constexpr (decltype(Q)::value) {
            const T e = lane_down(cx);
            return MIR ? rs2_core(cy, cx, py, e, my) : rs2_core(cy, cx, my, e, py);
        } else {
            const T w_ = lane_up(cy);
            return MIR ? rs2_core(cx, w_, px, cy, mx) : rs2_core(cx, w_, mx, cy, px);
        }
    };
    // F point (2t+1, k), k odd, from v2 rows (k-1)/2 (vlo) and (k+1)/2 (vhi), as jac2_diagF
    auto f21 = [&](int k, T rF, T vlo, T vhi) -> T {
        const T vlo_e = lane_down(vlo), vhi_e = lane_down(vhi);
        if (!((INNER || (t >= 0 && t <= h - 1)) && k >= 1 && k <= m - 1)) return T(0);
        return MIR ? jac2_chain(cd, rF, vhi, vhi_e, vlo_e, vlo) : jac2_chain(cd, rF, vlo, vlo_e, vhi_e, vhi);
    };
    // C point (2t, k), k even, from the F rows k-1 (Fm) and k+1 (Fp), as jac2_diagC
    auto c21 = [&](int k, T rC, T Fm, T Fp) -> T {
        const T Fm_w = lane_up(Fm), Fp_w = lane_up(Fp);
        if (!((INNER || (t >= 1 && t <= h - 1)) && k >= 2 && k <= m - 2)) return T(0);
        return MIR ? jac2_sum(cd, rC, Fp_w, Fp, Fm, Fm_w) : jac2_sum(cd, rC, Fm_w, Fm, Fp, Fp_w);
    };
    auto fsr = [&](int k, T r1k) -> T { return f21(k, r1k, ld2((k - 1) >> 1), ld2((k + 1) >> 1)); };
    // PP: the previous iterate's pair at marched row k, and in e the column
    // beyond the band (lane 0: 2t-1, lane 63: 2t+2); column m+1 does not exist
    const double inv_h2 = (double)m * (double)m;
    auto ldU = [&](int k, double& x, double& y, double& e) {
        x = y = e = 0;
        if (!colok || k < 0 || k > m) return;
        const auto p = ucg + (size_t)R(k) * w + 2 * t;
        if (INNER || t < h) {
            P2<double> v = NT ? ld_pair_nt(p) : ld_pair(p);
            x = v.x;
            y = v.y;
        } else {
            x = p[0];
        }
        if (lane == 0 && (INNER || t >= 1)) e = p[-1];
        if (lane == 63 && (INNER || 2 * t + 2 <= m)) e = p[2];
    };
    auto ldF = [&](int k, double& x, double& y) {
        x = y = 0;
        if (!colok || k < 1 || k > m - 1) return;
        const auto q = frg + (size_t)R(k) * w + 2 * t;
        P2<double> v = NT ? ld_pair_nt(q) : ld_pair(q);
        x = v.x;
        y = v.y;
    };
    // PP: the axis residual pair of marched row k from the u pairs of marched
    // rows k-1 (a), k (b), k+1 (c), the outer column e of row k and f of row k,
    // zero where ldR reads zero
    auto r0row = [&](int k, double ax, double ay, double bx, double by, double cx, double cy, double e, double fx,
                     double fy, T& x, T& y) {
        double uW = lane_up(by), uE = lane_down(bx);
        if (lane == 0) uW = e;
        if (lane == 63) uE = e;
        x = y = 0;
        if (!colok || k < 1 || k > m - 1) return;
        double x0, x1;
        if (MIR) resid_pair(inv_h2, fx, fy, uW, cx, cy, bx, by, ax, ay, uE, x0, x1);
        else resid_pair(inv_h2, fx, fy, uW, ax, ay, bx, by, cx, cy, uE, x0, x1);
        x = c0 ? (T)x0 : T(0);
        y = c1 ? (T)x1 : T(0);
    };
    // The march starts on the even row j at or before jbeg, so that every
    // row's parity is known at compile time.  Window entering row j:
    // diagonal values of rows j-1 (dm), j (d0), Fn = F row j+1.  The axis
    // residual pairs of rows j-3 .. j+2 give the diagonal residuals of rows
    // j-2 .. j+1.
    const int j = jbeg & ~1;
    T a0x, a0y, a1x, a1y, a2x, a2y, sx, sy_, nx, ny, xx, xy;
    // PP: u pairs of rows jj-1 .. jj+2 (w0 .. w3) entering an odd row jj, of
    // rows jj-1 .. jj+3 (w0 .. w4) entering an even one; eS: the outer column
    // of the next odd row jj' plus 2
    double w0x = 0, w0y = 0, w1x = 0, w1y = 0, w2x = 0, w2y = 0, w3x = 0, w3y = 0, w4x = 0, w4y = 0, eS = 0;
    // RES: f pairs of rows jj-2 .. jj+2 (F0 .. F4) entering an even row jj,
    // of rows jj-2 .. jj+1 (F0 .. F3) entering an odd one: the residual of the
    // new iterate at row jj-2 takes f from F0, the pair the Jacobi's residual
    // loaded four or five rows earlier (no second load of f)
    double F0x = 0, F0y = 0, F1x = 0, F1y = 0, F2x = 0, F2y = 0, F3x = 0, F3y = 0, F4x = 0, F4y = 0;
    if constexpr (PP) {
        double ux_[8], uy_[8], ue_[8];
#pragma unroll
        for (int i = 0; i < 8; i++) ldU(j - 4 + i, ux_[i], uy_[i], ue_[i]);   // rows j-4 .. j+3
        T rx_[6], ry_[6];
#pragma unroll
        for (int i = 0; i < 6; i++) {   // residual rows j-3 .. j+2
            double fx, fy;
            ldF(j - 3 + i, fx, fy);
            r0row(j - 3 + i, ux_[i], uy_[i], ux_[i + 1], uy_[i + 1], ux_[i + 2], uy_[i + 2], ue_[i + 1], fx, fy, rx_[i],
                  ry_[i]);
            if (i == 1) { F0x = fx; F0y = fy; }
            if (i == 2) { F1x = fx; F1y = fy; }
            if (i == 3) { F2x = fx; F2y = fy; }
            if (i == 4) { F3x = fx; F3y = fy; }
            if (i == 5) { F4x = fx; F4y = fy; }
        }
        a0x = rx_[0]; a0y = ry_[0];
        a1x = rx_[1]; a1y = ry_[1];
        a2x = rx_[2]; a2y = ry_[2];
        sx = rx_[3]; sy_ = ry_[3];
        nx = rx_[4]; ny = ry_[4];
        xx = rx_[5]; xy = ry_[5];
        w0x = ux_[3]; w0y = uy_[3];
        w1x = ux_[4]; w1y = uy_[4];
        w2x = ux_[5]; w2y = uy_[5];
        w3x = ux_[6]; w3y = uy_[6];
        w4x = ux_[7]; w4y = uy_[7];
        eS = ue_[7];
    } else {
        ldR(j - 3, a0x, a0y);
        ldR(j - 2, a1x, a1y);
        ldR(j - 1, a2x, a2y);
        ldR(j, sx, sy_);
        ldR(j + 1, nx, ny);
        ldR(j + 2, xx, xy);
    }
    T dm, d0, vlo, Fn;
    {
        const T Fm = fsr(j - 1, rs1(Int<1>{}, a1x, a1y, a2x, a2y, sx, sy_));
        const T Fp = fsr(j + 1, rs1(Int<1>{}, sx, sy_, nx, ny, xx, xy));
        dm = Fm;
        d0 = c21(j, rs1(Int<0>{}, a2x, a2y, sx, sy_, nx, ny), Fm, Fp);
        Fn = Fp;
        vlo = ld2((j + 2) >> 1);
    }
    // raw inputs loaded a row ahead of their use: at odd jj the axis
    // residual pairs of rows jj+2 (a) and jj+3 (b) and v2 row (jj+3)/2; u of
    // row jj.  Entering row jj, (sx, sy_) holds the pair of row jj, (nx, ny)
    // that of row jj+1 and, at even jj, (xx, xy) that of row jj+2.
    // PP, at odd jj: u of rows jj+3 (u3) and jj+4 (u4) with their outer
    // columns, f of rows jj+2 and jj+3, instead of the residual pairs
    struct Ck {
        T ax, ay, bx, by, vhi;
        double ux, uy;
        double u3x, u3y, u4x, u4y, e3, e4, f2x, f2y, f3x, f3y;
    };
    // Pc: Int<jj & 1>; an even row's buffer holds at most the u pair (FINEST
    // without PP) and is otherwise constant zero
    auto load = [&](auto Pc, int jj, Ck& c) {
        constexpr int P = decltype(Pc)::value;
        if constexpr (PP) {
            c.ax = c.ay = c.bx = c.by = c.vhi = 0;
            c.ux = c.uy = 0;
            c.u3x = c.u3y = c.u4x = c.u4y = c.e3 = c.e4 = c.f2x = c.f2y = c.f3x = c.f3y = 0;
            if (jj > jend || !P) return;
            ldU(jj + 3, c.u3x, c.u3y, c.e3);
            ldU(jj + 4, c.u4x, c.u4y, c.e4);
            ldF(jj + 2, c.f2x, c.f2y);
            ldF(jj + 3, c.f3x, c.f3y);
            c.vhi = ld2((jj + 3) >> 1);
            return;
        }
        c.ax = c.ay = c.bx = c.by = c.vhi = 0;
        c.ux = c.uy = 0;
        c.u3x = c.u3y = c.u4x = c.u4y = c.e3 = c.e4 = c.f2x = c.f2y = c.f3x = c.f3y = 0;
        if (jj > y1) return;
        if (FINEST && useful && jj >= y0 && jj < y1 && (c0 || c1)) {
            P2<double> v = ld_pair(ug + (size_t)R(jj) * w + 2 * t);
            c.ux = v.x;
            c.uy = v.y;
        }
        if constexpr (P) {
            ldR(jj + 2, c.ax, c.ay);
            ldR(jj + 3, c.bx, c.by);
            c.vhi = ld2((jj + 3) >> 1);
        }
    };
    T Fm2 = 0, Fm1 = 0, rCm1 = 0;
    double uxm1 = 0, uym1 = 0;
    // RES: the new iterate's pairs of rows k-1 (q_m) and k (q_c) entering the
    // residual of row k = jj-2; the residual pairs of rows k-1, k-2 and the
    // diagonal values of rows k-3, k-2, as in the residual kernel; the norm
    double qmx = 0, qmy = 0, qcx = 0, qcy = 0;
    T rm1_0 = 0, rm1_1 = 0, rm2_0 = 0, rm2_1 = 0, d3 = 0, d2 = 0;
    double acc = 0;
    const bool useful2 = useful && (INNER || (t >= 1 && t <= h - 1));
    // A row step's stores wait in registers and are issued at the start of
    // the next odd row step, right after its loads have arrived.  The odd
    // step's loads go out before the even step; a store issued after them
    // would have to complete before the odd step can use them (a wait on the
    // vector-memory count covers every access issued before the one it
    // needs), so the even step's arithmetic would no longer hide their
    // latency; and stores issued early in the odd step are done before the
    // loop's next wait.  No wave reads what these stores write while the
    // kernel runs.
    bool pw = false, pr = false, qw = false;   // pending: even row, restriction, odd row
    size_t po = 0, pro = 0, qo = 0;
    double pux = 0, puy = 0, qux = 0, quy = 0;
    T pvx = 0, pvy = 0, prv = 0, qvx = 0, qvy = 0;
    auto store_row = [&](bool ok, size_t o, double ux, double uy, T vx, T vy) {
        if (!ok) return;
        if constexpr (FINEST) {
            if (c0 && c1) st_pair(ug + o, ux, uy);
            else if (c1) ug[o + 1] = uy;
            else if (c0) ug[o] = ux;
        } else {
            if (c0 && c1) st_pair(vAg + o, vx, vy);
            else if (c1) vAg[o + 1] = vy;
            else if (c0) vAg[o] = vx;
        }
    };
    auto flush = [&]() {
        store_row(qw, qo, qux, quy, qvx, qvy);
        store_row(pw, po, pux, puy, pvx, pvy);
        if constexpr (RES) {
            if (pr) rA2g[pro] = prv;
        }
        qw = pw = pr = false;
    };
    auto proc = [&](auto Pc, int jj, const Ck& c) {
        constexpr int P = decltype(Pc)::value;   // jj & 1 (the march calls it for jj <= jend only)
        T cax = c.ax, cay = c.ay, cbx = c.bx, cby = c.by;   // residual pairs of rows jj+2, jj+3 (odd jj)
        if constexpr (PP) {
            if constexpr (P) {
                // every load of this row step is needed right here; waiting for
                // all of them at once, ahead of the step's stores, spares the
                // loop a wait that would also cover those stores
                __builtin_amdgcn_s_waitcnt(kWaitVmem0);
                flush();
                r0row(jj + 2, w2x, w2y, w3x, w3y, c.u3x, c.u3y, eS, c.f2x, c.f2y, cax, cay);
                r0row(jj + 3, w3x, w3y, c.u3x, c.u3y, c.u4x, c.u4y, c.e3, c.f3x, c.f3y, cbx, cby);
            }
        }
        T dp;
        if constexpr (P) {   // row jj+1 even: its C points from F rows jj (= d0) and jj+2
            const T r1c = rs1(Int<0>{}, sx, sy_, nx, ny, cax, cay);
            const T r1f = rs1(Int<1>{}, nx, ny, cax, cay, cbx, cby);
            const T F2 = f21(jj + 2, r1f, vlo, c.vhi);
            dp = c21(jj + 1, r1c, d0, F2);
            Fn = F2;
            vlo = c.vhi;
        } else {        // row jj+1 odd: its F points, computed one row ago
            dp = Fn;
        }
        constexpr int q = P;
        const T rF = q ? sx : sy_;   // F at column 2t+1-q
        const T rC = q ? sy_ : sx;   // C at column 2t+q
        T nb;
        if constexpr (q) nb = lane_up(d0);
        else nb = lane_down(d0);
        const T vw = q ? nb : d0;
        const T ve = q ? d0 : nb;
        const int aF = 2 * t + 1 - q;
        const T Fj = ((INNER || (aF >= 1 && aF <= m - 1)) && jj >= 1 && jj <= m - 1)
                         ? (MIR ? jac2_sum(cc, rF, vw, dp, ve, dm) : jac2_sum(cc, rF, vw, dm, ve, dp))
                         : T(0);
        {   // the C points of row jj-1 and the update there (written from row y0 on)
            constexpr int qq = 1 - P;
            T sb;
            if constexpr (qq) sb = lane_down(Fm1);
            else sb = lane_up(Fm1);
            const T cw = qq ? Fm1 : sb;
            const T ce = qq ? sb : Fm1;
            const T C = MIR ? jac2_sum(cc, rCm1, cw, Fj, ce, Fm2) : jac2_sum(cc, rCm1, cw, Fm2, ce, Fj);
            const T vx = qq ? Fm1 : C;   // column 2t
            const T vy = qq ? C : Fm1;   // column 2t+1
            const size_t o = (size_t)R(jj - 1) * w + 2 * t;
            const double ox = PP ? w0x : uxm1, oy = PP ? w0y : uym1;   // the iterate at row jj-1
            if constexpr (RES) {
                // the new iterate's pair of row jj-1 (the old values off the interior)
                const bool rin = jj - 1 >= 1 && jj - 1 <= m - 1;
                const double npx = (rin && c0) ? ox + (double)vx : ox, npy = (rin && c1) ? oy + (double)vy : oy;
                // its residual row k = jj-2 from u' rows k-1 (q_m), k (q_c), k+1 (np).
                // The pipeline runs from the march's first row on: the rows before
                // jstart (and after ylast) only pass through its registers and reach
                // no output (the norm and the stores are guarded), so its state needs
                // no branch per row.
                const int k = jj - 2;
                const double fx = F0x, fy = F0y;
                const double uW = lane_up(qcy), uE = lane_down(qcx);
                const bool rowin = k >= 1 && k <= m - 1;
                double x0, x1;
                if (MIR) resid_pair(inv_h2, fx, fy, uW, npx, npy, qcx, qcy, qmx, qmy, uE, x0, x1);
                else resid_pair(inv_h2, fx, fy, uW, qmx, qmy, qcx, qcy, npx, npy, uE, x0, x1);
                const T r0j = (rowin && c0) ? (T)x0 : T(0), r1j = (rowin && c1) ? (T)x1 : T(0);
                // the residual kernel's sums: x0^2 + x1^2, or the one interior column's
                const double s2 = (c0 ? x0 * x0 : 0.0) + (c1 ? x1 * x1 : 0.0);
                if (k >= y0 && k < y1 && useful) acc += s2;
                {   // Eq. (Erest2r) at the diagonal point of row k-1, then Eq.
                    // (Erest2b) onto the axis level below it at even k
                    constexpr int q = 1 - P;   // (k - 1) & 1, k = jj - 2
                    T sh;
                    if constexpr (q) sh = lane_down(rm1_0);
                    else sh = lane_up(rm1_1);
                    const T rc = q ? rm1_1 : rm1_0;
                    const T rw = q ? rm1_0 : sh;
                    const T re = q ? sh : rm1_1;
                    const T rlo = q ? rm2_1 : rm2_0;
                    const T rhi = q ? r1j : r0j;
                    const T d1 = MIR ? rs2_core(rc, rw, rhi, re, rlo) : rs2_core(rc, rw, rlo, re, rhi);
                    if constexpr (!P) {   // a restriction store, pending (see above)
                        const int B = (k - 2) >> 1;
                        const T d3w = lane_up(d3), d1w = lane_up(d1);
                        pr = k - 2 >= y0 && k - 2 < y1 && useful2 && B >= 1 && B <= h - 1;
                        pro = (size_t)(MIR ? h - B : B) * (h + 1) + t;
                        prv = MIR ? rs2_core(d2, d1w, d1, d3, d3w) : rs2_core(d2, d3w, d3, d1, d1w);
                    }
                    d3 = d2;
                    d2 = d1;
                }
                rm2_0 = rm1_0;
                rm2_1 = rm1_1;
                rm1_0 = r0j;
                rm1_1 = r1j;
                qmx = qcx;
                qmy = qcy;
                qcx = npx;
                qcy = npy;
            }
            const bool wr = useful && (!RES || jj - 1 < y1) && jj - 1 >= y0;
            if constexpr (!P) {   // pending until the next row step
                pw = wr;
                po = o;
                pux = ox + (double)vx;
                puy = oy + (double)vy;
                pvx = vx;
                pvy = vy;
            } else {
                if constexpr (!PP) flush();
                qw = wr;
                qo = o;
                qux = ox + (double)vx;
                quy = oy + (double)vy;
                qvx = vx;
                qvy = vy;
            }
        }
        Fm2 = Fm1;
        Fm1 = Fj;
        rCm1 = rC;
        dm = d0;
        d0 = dp;
        uxm1 = c.ux;
        uym1 = c.uy;
        // slide the residual pairs one row
        sx = nx;
        sy_ = ny;
        if constexpr (P) {
            nx = cax;
            ny = cay;
            xx = cbx;
            xy = cby;
        } else {
            nx = xx;
            ny = xy;
        }
        if constexpr (PP) {   // and the iterate's rows
            w0x = w1x; w0y = w1y;
            w1x = w2x; w1y = w2y;
            w2x = w3x; w2y = w3y;
            if constexpr (P) {
                w3x = c.u3x; w3y = c.u3y;
                w4x = c.u4x; w4y = c.u4y;
                eS = c.e4;
            } else {
                w3x = w4x; w3y = w4y;
            }
        }
        if constexpr (RES) {   // and f
            F0x = F1x; F0y = F1y;
            F1x = F2x; F1y = F2y;
            F2x = F3x; F2y = F3y;
            if constexpr (P) {
                F3x = c.f2x; F3y = c.f2y;
                F4x = c.f3x; F4y = c.f3y;
            } else {
                F3x = F4x; F3y = F4y;
            }
        }
    };
    rows_march_parity<Ck>(j, jend, load, proc);
    flush();   // the last row steps' stores
    return acc;
}

template <typename T, bool NT>
__global__ void __launch_bounds__(kRowBlock) kb_finest_fused(int m, T cc, T cd, const Fin2<T>* __restrict__ items,
                                                             int nwx, int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int t0 = (wv % nwx) * kFusePairs - 2;   // the column pair of lane 0
    const bool inner = t0 >= 1 && t0 + 63 <= m / 2 - 1;
    auto run = [&](auto Mc, auto Ic) {
        fused_body<T, true, NT, decltype(Mc)::value != 0, false, false, decltype(Ic)::value != 0>(
            m, cc, cd, it.r0, it.v2, nullptr, it.u, wv, nwx, rows);
    };
    if ((wv / nwx) & 1) {
        if (inner) run(Int<1>{}, Int<1>{});
        else run(Int<1>{}, Int<0>{});
    } else {
        if (inner) run(Int<0>{}, Int<1>{});
        else run(Int<0>{}, Int<0>{});
    }
}

// Out-of-place solve step (one FP64 problem): cycle k (the control block's
// count when the cycle runs) reads the iterate of cycle k-1 and writes that of
// cycle k; even k live in u, odd k in ub.
// (T: the type of the levels and the correction; FP32-refined solves use
// float, the residual and the iterate staying double)
template <typename T>
__global__ void __launch_bounds__(kRowBlock) __attribute__((amdgpu_waves_per_eu(4))) kb_finest_oop(int m, T cc, T cd,
                                                           const Fin2<T>* __restrict__ items, int nwx,
                                                           int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const bool odd = ctls[it.prob].k & 1;
    const double* uc = odd ? it.u : it.ub;
    double* un = odd ? it.ub : it.u;
    if ((wv / nwx) & 1)
        fused_body<T, true, false, true, true>(m, cc, cd, nullptr, it.v2, nullptr, un, wv, nwx, rows, uc, it.f);
    else
        fused_body<T, true, false, false, true>(m, cc, cd, nullptr, it.v2, nullptr, un, wv, nwx, rows, uc, it.f);
}

// The same step, which also evaluates the new iterate (the residual kernel's
// work for the next evaluation, see RES above): each block's norm partial
// goes to part[blockIdx.x], and block 0 clears part[gridDim.x .. nparts), so
// the finalize kernel sums as many partials as after the residual kernel.
template <typename T>
__global__ void __launch_bounds__(kRowBlock) __attribute__((amdgpu_waves_per_eu(3))) kb_finest_res(int m, T cc, T cd,
                                                           const Fin2<T>* __restrict__ items, int nwx,
                                                           int nwaves, int rows, const Ctl* __restrict__ ctls,
                                                           int nparts)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const int wv = rows_wave_id(nwaves);
    const bool odd = ctls[it.prob].k & 1;
    const double* uc = odd ? it.u : it.ub;
    double* un = odd ? it.ub : it.u;
    double acc = 0;
    if (wv < nwaves) {   // no early return: the block sum below synchronises the block
        const int t0 = (wv % nwx) * kResPairs - 4;   // the column pair of lane 0
        const bool inner = t0 >= 1 && t0 + 63 <= m / 2 - 1;
        auto run = [&](auto Mc, auto Ic) {
            return fused_body<T, true, false, decltype(Mc)::value != 0, true, true, decltype(Ic)::value != 0>(
                m, cc, cd, nullptr, it.v2, nullptr, un, wv, nwx, rows, uc, it.f, it.r2);
        };
        if ((wv / nwx) & 1) acc = inner ? run(Int<1>{}, Int<1>{}) : run(Int<1>{}, Int<0>{});
        else acc = inner ? run(Int<0>{}, Int<1>{}) : run(Int<0>{}, Int<0>{});
    }
    const double sum = rows_block_sum(acc);
    if (threadIdx.x == 0) it.part[blockIdx.x] = sum;
    if (blockIdx.x == 0)
        for (int i = (int)gridDim.x + (int)threadIdx.x; i < nparts; i += blockDim.x) it.part[i] = 0.0;
}

// The Jacobi of an axis level L (side m, coefficient cc) with that of the
// diagonal level L-1 below it (coefficient cd) computed in the same march
template <typename T>
__global__ void __launch_bounds__(kRowBlock) kb_jac_pair(int m, T cc, T cd, const JPair2<T>* __restrict__ items,
                                                         int nwx, int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const JPair2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int t0 = (wv % nwx) * kFusePairs - 2;   // the column pair of lane 0
    const bool inner = t0 >= 1 && t0 + 63 <= m / 2 - 1;
    auto run = [&](auto Mc, auto Ic) {
        fused_body<T, false, false, decltype(Mc)::value != 0, false, false, decltype(Ic)::value != 0>(
            m, cc, cd, it.rA, it.v2, it.vA, nullptr, wv, nwx, rows);
    };
    if ((wv / nwx) & 1) {
        if (inner) run(Int<1>{}, Int<1>{});
        else run(Int<1>{}, Int<0>{});
    } else {
        if (inner) run(Int<0>{}, Int<1>{});
        else run(Int<0>{}, Int<0>{});
    }
}

// tiny finest grids: one thread per point (both half-sweeps recomputed)
template <typename T>
__global__ void kb_finest_small(int n, T cc, const Fin2<T>* __restrict__ items, const Ctl* __restrict__ ctls)
{
    const Fin2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    for (int q = threadIdx.x; q < (n / 2 + 1) * (n - 1); q += blockDim.x) {
        int tt = q % (n / 2 + 1), b = q / (n / 2 + 1) + 1;
        int aC = 2 * tt + (b & 1), aF = 2 * tt + 1 - (b & 1);
        if (aF >= 1 && aF < n) { size_t o = idxA(n, aF, b); it.u[o] = it.u[o] + (double)jac2_axisF(it.r0, it.v1, n, cc, aF, b); }
        if (aC >= 1 && aC < n) { size_t o = idxA(n, aC, b); it.u[o] = it.u[o] + (double)jac2_axisC(it.r0, it.v1, n, cc, aC, b); }
    }
}

// ============================================================= level kernels

// Eq. (Erest2r): axis grid (side m) -> diagonal grid (side m), row-marching
template <typename T, int CH>
__global__ void __launch_bounds__(kRowBlock) kb_a2d_rows(int m, const Item2<T>* __restrict__ items, int nwx,
                                                         int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const T* __restrict__ rA = it.in;
    T* __restrict__ rD = it.r;
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
            if (useful && a >= 1 && a <= m - 1) rD[(size_t)j * W + t] = rs2_core(rc, rw, rs, re, rn);
            rm0 = rc0; rm1 = rc1; rc0 = c.x[i]; rc1 = c.y[i];
        }
    };
    rows_march<CH, Ck>(y0, y1 - 1, load, proc);
}

// Eqs. (Erest2r) then (Erest2b) in one march: the residual of an axis level
// L (side m) onto the diagonal level L-1 and from there onto the axis level
// L-2 (side m/2), the diagonal values of three consecutive rows kept in
// registers, as the residual kernel does below the finest level.  Level
// L-1's residual is not stored (kb_jac_pair restricts it again); lanes
// 2 .. 62 write r2; strips start on odd rows (rows is even) and compute one
// diagonal row past their end.
template <typename T, int CH>
__global__ void __launch_bounds__(kRowBlock) kb_rs_pair(int m, const RsPair2<T>* __restrict__ items, int nwx,
                                                        int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const RsPair2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const auto rA = gmem(it.rA);
    const auto rA2 = gmem(it.r2);
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int wx = wv % nwx, sy = wv / nwx;
    const int t = wx * kResidPairs - 1 + lane;
    const int y0 = 1 + sy * rows;
    const int y1 = min(y0 + rows, m);
    const int mc = m / 2;
    const bool useful2 = lane >= 2 && lane <= kResidPairs + 1 && t >= 1 && t <= mc - 1;
    const bool colok = t >= 0 && t <= m / 2;
    const bool c0 = t >= 1 && 2 * t <= m - 1, c1 = t >= 0 && 2 * t + 1 <= m - 1;
    const size_t w = (size_t)(m + 1);
    auto ldr = [&](int j, T& x, T& y) {
        x = y = 0;
        if (!colok || j < 1 || j > m - 1) return;
        P2<T> v = ld_pair(rA + (size_t)j * w + 2 * t);
        x = c0 ? v.x : T(0);
        y = c1 ? v.y : T(0);
    };
    struct Ck { T x[CH], y[CH]; };
    auto load = [&](int jb, Ck& c) {
#pragma unroll
        for (int i = 0; i < CH; i++) {
            c.x[i] = c.y[i] = 0;
            if (jb + i <= y1) ldr(jb + i + 1, c.x[i], c.y[i]);
        }
    };
    T rm0, rm1, rc0, rc1;
    ldr(y0 - 1, rm0, rm1);
    ldr(y0, rc0, rc1);
    T d3 = 0, d2 = 0;   // diagonal values of rows j-2, j-1
    // the march starts on the strip's first row, which is odd (rows is a
    // power of two), and CH is even: row jb + i has the parity of i + 1
    static_assert(CH % 2 == 0, "row parities are fixed by the chunk position");
    auto proc = [&](int jb, const Ck& c) {
        static_for<0, CH>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const int j = jb + i;   // past y1 too (the store below is guarded)
            constexpr int q = (i + 1) & 1;
            T sh;
            if constexpr (q) sh = lane_down(rc0);
            else sh = lane_up(rc1);
            const T rc = q ? rc1 : rc0;
            const T rw = q ? rc0 : sh;
            const T re = q ? sh : rc1;
            const T rs = q ? rm1 : rm0;
            const T rn = q ? c.y[i] : c.x[i];
            const T d1 = rs2_core(rc, rw, rs, re, rn);
            // axis point (t, B) of level L-2, B = (j-1)/2: diagonal rows 2B-1, 2B, 2B+1
            if (q && j - 1 >= y0 && j - 1 < y1) {
                const int B = (j - 1) >> 1;
                const T d3w = lane_up(d3), d1w = lane_up(d1);
                if (useful2 && B >= 1 && B <= mc - 1) rA2[(size_t)B * (mc + 1) + t] = rs2_core(d2, d3w, d3, d1, d1w);
            }
            d3 = d2;
            d2 = d1;
            rm0 = rc0; rm1 = rc1; rc0 = c.x[i]; rc1 = c.y[i];
        });
    };
    rows_march<CH, Ck>(y0, y1, load, proc);
}

// Eq. (Erest2b): diagonal grid (side m) -> axis grid (side m/2), row-marching.
// Lane owns coarse column A (lane 0 is a halo lane) and marches over coarse rows B.
template <typename T, int CH>
__global__ void __launch_bounds__(kRowBlock) kb_d2a_rows(int m, const Item2<T>* __restrict__ items, int nwx,
                                                         int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const T* __restrict__ rD = it.in;
    T* __restrict__ rA2 = it.r;
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
            if (useful) rA2[(size_t)B * (mc + 1) + A] = rs2_core(q.c[i], lo_w, lo, hi, hi_w);
            lo = hi;
        }
    };
    rows_march<CH, Ck>(B0, B1 - 1, load, proc);
}

// Eqs. (Eajacr), (Eajacb): Jacobi on a diagonal grid (side m) from the axis
// grid of side m/2.  Lane owns column A of the compacted rows: F = (2A+1, 2B+1)
// and C = (2A, 2B).
template <typename T, int CH>
__global__ void __launch_bounds__(kRowBlock) kb_jdiag_rows(int m, T cc, const Item2<T>* __restrict__ items, int nwx,
                                                           int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    const T* __restrict__ rD = it.r;
    const T* __restrict__ vA2 = it.in;
    T* __restrict__ vD = it.v;
    const int lane = threadIdx.x & 63;
    const int wv = rows_wave_id(nwaves);
    if (wv >= nwaves) return;
    const int h = m / 2;
    const int wx = wv % nwx, sy = wv / nwx;
    const int A = wx * kPairsPerWave - 1 + lane;
    const int B0 = sy * rows;  // coarse rows B: F row 2B+1 (B in [0,h-1]), C row 2B (B in [1,h-1])
    const int B1 = min(B0 + rows, h);
    const bool useful = lane >= 1 && lane <= kPairsPerWave && A >= 0 && A <= h - 1;
    const bool colok = A >= 0 && A <= h;
    const int W = m / 2 + 1;
    const size_t wc = (size_t)(h + 1);
    auto ldv = [&](int B, bool ok) -> T { return (ok && colok && B >= 0 && B <= h) ? vA2[(size_t)B * wc + A] : T(0); };
    auto ldr = [&](int row, bool ok) -> T {
        return (ok && colok && A <= h - 1 + ((row & 1) ? 0 : 1) && row >= 0 && row <= m) ? rD[(size_t)row * W + A] : T(0);
    };
    T vb = ldv(B0 >= 1 ? B0 - 1 : 0, true);
    T Fprev = 0;  // F of the odd row 2B-1
    if (B0 >= 1) {
        T vn = ldv(B0, true);
        T rf = ldr(2 * B0 - 1, true);
        T vb_e = __shfl_down(vb, 1), vn_e = __shfl_down(vn, 1);
        Fprev = jac2_chain(cc, rf, vb, vb_e, vn_e, vn);
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
            T F = jac2_chain(cc, q.rf[i], vb, vb_e, vn_e, vn);
            T Fw = __shfl_up(F, 1), Fpw = __shfl_up(Fprev, 1);
            if (useful) {
                vD[(size_t)(2 * B + 1) * W + A] = F;
                if (B >= 1 && A >= 1) vD[(size_t)(2 * B) * W + A] = jac2_sum(cc, q.rc[i], Fpw, Fprev, F, Fw);
            }
            Fprev = F;
            vb = vn;
        }
    };
    rows_march<CH, Ck>(B0, B1 - 1, load, proc);
}

// axis-grid Jacobi of a coarser level (stores v)
template <typename T, int CH>
__global__ void __launch_bounds__(kRowBlock) kb_jaxis_rows(int m, T cc, const Item2<T>* __restrict__ items, int nwx,
                                                           int nwaves, int rows, const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.y];
    ITEM_GATE(ctls, it.prob);
    jaxis_body<T, false, CH, false>(m, cc, it.r, it.in, it.v, nullptr, nwx, nwaves, rows);
}

// ------------------------------------------------------ one thread per point
template <typename T>
__global__ void __launch_bounds__(256) kb_rs_a2d(int m, const Item2<T>* __restrict__ items, const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.z];
    ITEM_GATE(ctls, it.prob);
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1;
    if (col > m / 2 || b >= m) return;
    int a = 2 * col + (b & 1);
    if (a < 1 || a >= m) return;
    it.r[idxD(m, a, b)] = rs2_a2d(it.in, m, a, b);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_rs_d2a(int m, const Item2<T>* __restrict__ items, const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.z];
    ITEM_GATE(ctls, it.prob);
    int mc = m / 2;
    int A = blockIdx.x * blockDim.x + threadIdx.x + 1;
    int B = blockIdx.y + 1;
    if (A >= mc || B >= mc) return;
    it.r[idxA(mc, A, B)] = rs2_d2a(it.in, m, A, B);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_jac_diag(int m, T cc, const Item2<T>* __restrict__ items,
                                                   const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.z];
    ITEM_GATE(ctls, it.prob);
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    int B = blockIdx.y;
    int h = m / 2;
    if (A >= h || B >= h) return;
    int a = 2 * A + 1, b = 2 * B + 1;
    it.v[idxD(m, a, b)] = jac2_diagF(it.r, it.in, m, cc, a, b);
    if (A >= 1 && B >= 1) it.v[idxD(m, 2 * A, 2 * B)] = jac2_diagC(it.r, it.in, m, cc, 2 * A, 2 * B);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_jac_axis(int m, T cc, const Item2<T>* __restrict__ items,
                                                   const Ctl* __restrict__ ctls)
{
    const Item2<T> it = items[blockIdx.z];
    ITEM_GATE(ctls, it.prob);
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y + 1;
    if (t > m / 2 || b >= m) return;
    int aC = 2 * t + (b & 1), aF = 2 * t + 1 - (b & 1);
    if (aF >= 1 && aF < m) it.v[idxA(m, aF, b)] = jac2_axisF(it.r, it.in, m, cc, aF, b);
    if (aC >= 1 && aC < m) it.v[idxA(m, aC, b)] = jac2_axisC(it.r, it.in, m, cc, aC, b);
}

// ------------------------------------------------------ mid levels, fused
// A single problem with n >= 512 would run its levels of side 256 .. 64
// (aligned levels 14 .. 9) one thread per point or inside the one-workgroup
// coarse kernel: latency-bound steps.  These two kernels do that work in one
// launch each.  A workgroup owns a tile of the output and recomputes in LDS
// the part of every intermediate level its tile depends on (halo included);
// it writes only the points it owns.  Every value goes through the same
// point arithmetic as the per-level kernels, so the results are
// bit-identical to theirs.  Regions are square [lo, lo + W) in a level's own
// coordinates (diagonal levels use the points with an even index sum);
// entries off the interior are 0, the boundary value.
constexpr int kMidTiles = 8;        // tiles per side: 64 workgroups
constexpr int kMidThreads = 1024;   // 16 waves: the level steps are latency-bound

template <typename T>
struct MReg {   // a level's region in LDS
    T* p;
    int a0, b0, w;
    __device__ T& at(int a, int b) const { return p[(b - b0) * w + (a - a0)]; }
};

// restriction steps region -> region (each point as rs2_a2d / rs2_d2a);
// `own` points are also stored to the level's global array
template <typename T, typename Own>
__device__ inline void mid_a2d(const MReg<T>& in, const MReg<T>& out, int m, T* g, Own own)
{
    for (int q = threadIdx.x; q < out.w * out.w; q += blockDim.x) {
        const int a = out.a0 + q % out.w, b = out.b0 + q / out.w;
        T x = T(0);
        if (a >= 1 && a < m && b >= 1 && b < m && !((a + b) & 1)) {
            x = rs2_core(in.at(a, b), in.at(a - 1, b), in.at(a, b - 1), in.at(a + 1, b), in.at(a, b + 1));
            if (own(a, b)) g[idxD(m, a, b)] = x;
        }
        out.p[q] = x;
    }
}
template <typename T, typename Own>
__device__ inline void mid_d2a(const MReg<T>& in, const MReg<T>& out, int mc, T* g, Own own)
{
    for (int q = threadIdx.x; q < out.w * out.w; q += blockDim.x) {
        const int A = out.a0 + q % out.w, B = out.b0 + q / out.w;
        T x = T(0);
        if (A >= 1 && A < mc && B >= 1 && B < mc) {
            const int a = 2 * A, b = 2 * B;
            x = rs2_core(in.at(a, b), in.at(a - 1, b - 1), in.at(a + 1, b - 1), in.at(a + 1, b + 1), in.at(a - 1, b + 1));
            if (own(A, B)) g[idxA(mc, A, B)] = x;
        }
        out.p[q] = x;
    }
}

template <typename T>
__global__ void __launch_bounds__(kMidThreads) kb_mid_down(const T* __restrict__ r14, T* __restrict__ r13,
                                                           T* __restrict__ r12, T* __restrict__ r11, T* __restrict__ r10,
                                                           T* __restrict__ r9, T* __restrict__ r8,
                                                           const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    constexpr int W13 = 51, W12 = 25, W11 = 23, W10 = 11, W9 = 9;
    __shared__ T S13[W13 * W13], S12[W12 * W12], S11[W11 * W11], S10[W10 * W10], S9[W9 * W9];
    const int tx = blockIdx.x % kMidTiles, ty = blockIdx.x / kMidTiles;
    // tile (tx, ty) owns level-8 points [4t+1, 4t+4], levels 10 and 9 [8t+1, 8t+8],
    // 12 and 11 [16t+1, 16t+16], 13 [32t+1, 32t+32]
    auto own = [tx, ty](int s) {
        return [tx, ty, s](int a, int b) { return a > s * tx && a <= s * tx + s && b > s * ty && b <= s * ty + s; };
    };
    const MReg<T> R13{S13, 32 * tx - 5, 32 * ty - 5, W13}, R12{S12, 16 * tx - 2, 16 * ty - 2, W12};
    const MReg<T> R11{S11, 16 * tx - 1, 16 * ty - 1, W11}, R10{S10, 8 * tx, 8 * ty, W10};
    const MReg<T> R9{S9, 8 * tx + 1, 8 * ty + 1, W9};
    // level 13 from level 14 (global), Eq. (Erest2r) as rs2_a2d
    auto own13 = own(32);
    for (int q = threadIdx.x; q < W13 * W13; q += blockDim.x) {
        const int a = R13.a0 + q % W13, b = R13.b0 + q / W13;
        T x = T(0);
        if (a >= 1 && a <= 255 && b >= 1 && b <= 255 && !((a + b) & 1)) {
            x = rs2_a2d(r14, 256, a, b);
            if (own13(a, b)) r13[idxD(256, a, b)] = x;
        }
        S13[q] = x;
    }
    __syncthreads();
    mid_d2a(R13, R12, 128, r12, own(16));
    __syncthreads();
    mid_a2d(R12, R11, 128, r11, own(16));
    __syncthreads();
    mid_d2a(R11, R10, 64, r10, own(8));
    __syncthreads();
    mid_a2d(R10, R9, 64, r9, own(8));
    __syncthreads();
    // level 8, the tile itself, Eq. (Erest2b)
    if (threadIdx.x < 16) {
        const int A = 4 * tx + 1 + threadIdx.x % 4, B = 4 * ty + 1 + threadIdx.x / 4;
        if (A <= 31 && B <= 31) {
            const int a = 2 * A, b = 2 * B;
            r8[idxA(32, A, B)] = rs2_core(R9.at(a, b), R9.at(a - 1, b - 1), R9.at(a + 1, b - 1), R9.at(a + 1, b + 1),
                                          R9.at(a - 1, b + 1));
        }
    }
}

// Jacobi steps on a region: F points over the whole region, then (after a
// barrier) C points over the region less its border, from the stored F
// values.  Diagonal levels: F from the coarser axis level `vc` (region, or
// global when vcg is set), as jac2_diagF; axis levels: F from the diagonal
// level of the same side, as jac2_axisF.  r: the level's global residual.
template <typename T>
__device__ inline void mid_jdiag(const MReg<T>& L, const MReg<T>* vc, const T* vcg, const T* r, int m, T cc)
{
    const int w = m / 2 + 1;
    for (int q = threadIdx.x; q < L.w * L.w; q += blockDim.x) {
        const int a = L.a0 + q % L.w, b = L.b0 + q / L.w;
        if (a >= 1 && a < m && b >= 1 && b < m && (a & b & 1)) {
            if (vcg) {
                L.p[q] = jac2_diagF(r, vcg, m, cc, a, b);
            } else {
                const int A0 = (a - 1) >> 1, B0 = (b - 1) >> 1;
                L.p[q] = jac2_chain(cc, r[b * w + (a >> 1)], vc->at(A0, B0), vc->at(A0 + 1, B0), vc->at(A0 + 1, B0 + 1),
                                    vc->at(A0, B0 + 1));
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < L.w * L.w; q += blockDim.x) {
        const int la = q % L.w, lb = q / L.w, a = L.a0 + la, b = L.b0 + lb;
        if (la >= 1 && la < L.w - 1 && lb >= 1 && lb < L.w - 1 && a >= 1 && a < m && b >= 1 && b < m && !((a | b) & 1))
            L.p[q] = jac2_sum(cc, r[b * w + (a >> 1)], L.p[q - L.w - 1], L.p[q - L.w + 1], L.p[q + L.w + 1],
                              L.p[q + L.w - 1]);
    }
    __syncthreads();
}
template <typename T>
__device__ inline void mid_jaxis(const MReg<T>& L, const MReg<T>& vd, const T* r, int m, T cc)
{
    const int w = m + 1;
    for (int q = threadIdx.x; q < L.w * L.w; q += blockDim.x) {
        const int a = L.a0 + q % L.w, b = L.b0 + q / L.w;
        if (a >= 1 && a < m && b >= 1 && b < m && ((a + b) & 1))
            L.p[q] = jac2_sum(cc, r[b * w + a], vd.at(a - 1, b), vd.at(a, b - 1), vd.at(a + 1, b), vd.at(a, b + 1));
    }
    __syncthreads();
    for (int q = threadIdx.x; q < L.w * L.w; q += blockDim.x) {
        const int la = q % L.w, lb = q / L.w, a = L.a0 + la, b = L.b0 + lb;
        if (la >= 1 && la < L.w - 1 && lb >= 1 && lb < L.w - 1 && a >= 1 && a < m && b >= 1 && b < m && !((a + b) & 1))
            L.p[q] = jac2_sum(cc, r[b * w + a], L.p[q - 1], L.p[q - L.w], L.p[q + 1], L.p[q + L.w]);
    }
    __syncthreads();
}

// Jacobi up from v8 (axis 32) through v9 (diagonal 64), v10 (axis 64), v11
// (diagonal 128), v12 (axis 128), v13 (diagonal 256) to v14 (axis 256).
// Tile (tx, ty) owns level-14 and 13 points [32t+1, 32t+32], levels 12 and
// 11 [16t+1, 16t+16], levels 10 and 9 [8t+1, 8t+8].  r[k], v[k], c[k]:
// level 9 + k.
template <typename T>
struct MidUp {
    const T* r[6];
    T* v[6];
    T c[6];
};
template <typename T>
__global__ void __launch_bounds__(kMidThreads) kb_mid_up(const T* __restrict__ v8, MidUp<T> L, const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    constexpr int W9 = 20, W10 = 16, W11 = 26, W12 = 22, W13 = 38, W14 = 34;
    __shared__ T S9[W9 * W9], S10[W10 * W10], S11[W11 * W11], S12[W12 * W12], S13[W13 * W13], S14[W14 * W14];
    const int tx = blockIdx.x % kMidTiles, ty = blockIdx.x / kMidTiles;
    const MReg<T> L9{S9, 8 * tx - 5, 8 * ty - 5, W9}, L10{S10, 8 * tx - 3, 8 * ty - 3, W10};
    const MReg<T> L11{S11, 16 * tx - 4, 16 * ty - 4, W11}, L12{S12, 16 * tx - 2, 16 * ty - 2, W12};
    const MReg<T> L13{S13, 32 * tx - 2, 32 * ty - 2, W13}, L14{S14, 32 * tx, 32 * ty, W14};
    for (int q = threadIdx.x; q < W13 * W13; q += blockDim.x) {
        S13[q] = T(0);
        if (q < W9 * W9) S9[q] = T(0);
        if (q < W10 * W10) S10[q] = T(0);
        if (q < W11 * W11) S11[q] = T(0);
        if (q < W12 * W12) S12[q] = T(0);
        if (q < W14 * W14) S14[q] = T(0);
    }
    __syncthreads();
    mid_jdiag(L9, (const MReg<T>*)nullptr, v8, L.r[0], 64, L.c[0]);
    mid_jaxis(L10, L9, L.r[1], 64, L.c[1]);
    mid_jdiag(L11, &L10, (const T*)nullptr, L.r[2], 128, L.c[2]);
    mid_jaxis(L12, L11, L.r[3], 128, L.c[3]);
    // owned points of levels 9 .. 12
    for (int q = threadIdx.x; q < 16 * 16; q += blockDim.x) {
        const int a = 16 * tx + 1 + q % 16, b = 16 * ty + 1 + q / 16;
        if (a <= 127 && b <= 127) {
            if (!((a + b) & 1)) L.v[2][idxD(128, a, b)] = L11.at(a, b);
            L.v[3][idxA(128, a, b)] = L12.at(a, b);
        }
        if (q < 64) {
            const int a8 = 8 * tx + 1 + q % 8, b8 = 8 * ty + 1 + q / 8;
            if (a8 <= 63 && b8 <= 63) {
                if (!((a8 + b8) & 1)) L.v[0][idxD(64, a8, b8)] = L9.at(a8, b8);
                L.v[1][idxA(64, a8, b8)] = L10.at(a8, b8);
            }
        }
    }
    mid_jdiag(L13, &L12, (const T*)nullptr, L.r[4], 256, L.c[4]);
    // level 14: F on [32t, 32t+33] from level 13; owned points of level 13
    const T* r14 = L.r[5];
    for (int q = threadIdx.x; q < W14 * W14; q += blockDim.x) {
        const int a = L14.a0 + q % W14, b = L14.b0 + q / W14;
        if (a >= 1 && a <= 255 && b >= 1 && b <= 255 && ((a + b) & 1))
            S14[q] = jac2_sum(L.c[5], r14[idxA(256, a, b)], L13.at(a - 1, b), L13.at(a, b - 1), L13.at(a + 1, b),
                              L13.at(a, b + 1));
    }
    for (int q = threadIdx.x; q < 32 * 32; q += blockDim.x) {
        const int a = 32 * tx + 1 + q % 32, b = 32 * ty + 1 + q / 32;
        if (a <= 255 && b <= 255 && !((a + b) & 1)) L.v[4][idxD(256, a, b)] = L13.at(a, b);
    }
    __syncthreads();
    // level 14, the tile: F from LDS, C from its four F neighbours
    for (int q = threadIdx.x; q < 32 * 32; q += blockDim.x) {
        const int a = 32 * tx + 1 + q % 32, b = 32 * ty + 1 + q / 32;
        if (a > 255 || b > 255) continue;
        L.v[5][idxA(256, a, b)] =
            ((a + b) & 1) ? L14.at(a, b)
                          : jac2_sum(L.c[5], r14[idxA(256, a, b)], L14.at(a - 1, b), L14.at(a, b - 1), L14.at(a + 1, b),
                                     L14.at(a, b + 1));
    }
}

// ------------------------------------------------------------ coarse levels
// Aligned levels top .. 0 of one problem per workgroup: restriction down to
// the 3x3 grid, its Jacobi from a zero correction, Jacobi back up to top.
// The levels stay in global memory (L2-resident): their stencils issue
// about twenty reads per point, more than the fifteen LDS operations a wave
// can keep in flight, and staging them in LDS measured slower (33 us against
// 22 us per cycle on MI355X).
template <typename T>
struct CoarseLev {
    LevInfo<T> l[kCoarseLevels];
    int top_cap;   // highest level run here (levels above it run in the fused mid-level kernels)
};
constexpr int kCoarseThreadsB = 1024;

// the level arrays of one problem
template <typename T>
struct GLevs {
    const Coarse2B<T>& it;
    const T* z;
    __device__ T* r(int l) const { return it.r[l]; }
    __device__ T* v(int l) const { return it.v[l]; }
    __device__ const T* zero() const { return z; }
};

// restriction into lam for lam = hi-1 down to lo
template <typename T, typename LV>
__device__ void coarse_down(const CoarseLev<T>& L, const LV& it, int hi, int lo)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int lam = hi - 1; lam >= lo; lam--) {
        const LevInfo<T>& Fi = L.l[lam + 1];
        const T* rf = it.r(lam + 1);
        T* rc = it.r(lam);
        int m = Fi.m;
        if (!Fi.diag) {  // axis -> diagonal, same side
            int w = m / 2 + 1;
            for (int q = tid; q < w * (m - 1); q += nt) {
                int col = q % w, b = q / w + 1;
                int a = 2 * col + (b & 1);
                if (a >= 1 && a < m) rc[idxD(m, a, b)] = rs2_a2d(rf, m, a, b);
            }
        } else {         // diagonal -> axis of side m/2
            int mc = m / 2;
            for (int q = tid; q < (mc - 1) * (mc - 1); q += nt) {
                int A = q % (mc - 1) + 1, B = q / (mc - 1) + 1;
                rc[idxA(mc, A, B)] = rs2_d2a(rf, m, A, B);
            }
        }
        __syncthreads();
    }
}

// Jacobi at lam = lo .. hi (lam = 0 from a zero correction).  Levels of side
// >= kCoarseTwoPassSide store their F points first and take the C points'
// neighbours from there after a barrier, instead of recomputing four F
// values per C point (same operands, same order, same result).
constexpr int kCoarseTwoPassSide = 16;
template <typename T, typename LV>
__device__ void coarse_up(const CoarseLev<T>& L, const LV& it, int lo, int hi)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int lam = lo; lam <= hi; lam++) {
        const LevInfo<T>& Li = L.l[lam];
        const T* vc = lam == 0 ? it.zero() : it.v(lam - 1);
        const T* r = it.r(lam);
        T* v = it.v(lam);
        int m = Li.m;
        T cc = Li.c;
        const bool two = m >= kCoarseTwoPassSide;
        if (Li.diag) {
            int h = m / 2;
            for (int q = tid; q < h * h; q += nt) {
                int A = q % h, B = q / h;
                v[idxD(m, 2 * A + 1, 2 * B + 1)] = jac2_diagF(r, vc, m, cc, 2 * A + 1, 2 * B + 1);
                if (!two && A >= 1 && B >= 1) v[idxD(m, 2 * A, 2 * B)] = jac2_diagC(r, vc, m, cc, 2 * A, 2 * B);
            }
            if (two) {
                __syncthreads();
                for (int q = tid; q < (h - 1) * (h - 1); q += nt) {
                    int A = q % (h - 1) + 1, B = q / (h - 1) + 1;
                    v[idxD(m, 2 * A, 2 * B)] = jac2_diagC_stored(r, v, m, cc, 2 * A, 2 * B);
                }
            }
        } else {
            int w = m / 2 + 1;
            for (int q = tid; q < w * (m - 1); q += nt) {
                int t = q % w, b = q / w + 1;
                int aC = 2 * t + (b & 1), aF = 2 * t + 1 - (b & 1);
                if (aF >= 1 && aF < m) v[idxA(m, aF, b)] = jac2_axisF(r, vc, m, cc, aF, b);
                if (!two && aC >= 1 && aC < m) v[idxA(m, aC, b)] = jac2_axisC(r, vc, m, cc, aC, b);
            }
            if (two) {
                __syncthreads();
                for (int q = tid; q < w * (m - 1); q += nt) {
                    int t = q % w, b = q / w + 1;
                    int aC = 2 * t + (b & 1);
                    if (aC >= 1 && aC < m) v[idxA(m, aC, b)] = jac2_axisC_stored(r, v, m, cc, aC, b);
                }
            }
        }
        __syncthreads();
    }
}

// Levels 0 .. kCoarseLdsTop (side <= 32, 2277 points per array) run in LDS:
// each of their steps then waits on LDS instead of L2.  The larger levels
// stay in global memory, so batched launches still fit two workgroups per CU.
constexpr int kCoarseLdsTop = 8;
constexpr int kCoarseLdsPts = 2304;   // >= the points of levels 0 .. 8

template <typename T>
struct SLevs {
    T* lds;            // r of the staged levels, then v at + kCoarseLdsPts
    const int* off;    // offset of each staged level
    const T* z;        // zero correction below level 0 (in LDS)
    __device__ T* r(int l) const { return lds + off[l]; }
    __device__ T* v(int l) const { return lds + kCoarseLdsPts + off[l]; }
    __device__ const T* zero() const { return z; }
};

template <typename T>
__device__ inline int lev2_points(const LevInfo<T>& l)
{
    return l.diag ? (l.m + 1) * (l.m / 2 + 1) : (l.m + 1) * (l.m + 1);
}

template <typename T>
__global__ void __launch_bounds__(kCoarseThreadsB) kb_coarse(CoarseLev<T> L, const Coarse2B<T>* __restrict__ items,
                                                             const T* __restrict__ zero, const Ctl* __restrict__ ctls)
{
    __shared__ T lds[2 * kCoarseLdsPts + 64];
    __shared__ int off[kCoarseLdsTop + 1];
    const Coarse2B<T>& it = items[blockIdx.x];
    ITEM_GATE(ctls, it.prob);
    const int tid = threadIdx.x, nt = blockDim.x;
    const GLevs<T> G{it, zero};
    const int top = min(it.top, L.top_cap);
    const int st = min(top, kCoarseLdsTop);      // highest staged level
    if (tid == 0) {
        int o = 0;
        for (int l = 0; l <= st; l++) {
            off[l] = o;
            o += lev2_points(L.l[l]);
        }
    }
    __syncthreads();
    // global part of the restriction: into levels top-1 .. st
    coarse_down(L, G, top, st);
    // stage r of level st; zero the other staged arrays (boundary entries
    // stay 0) and the zero correction below level 0
    const int nst = off[st] + lev2_points(L.l[st]);
    for (int q = tid; q < nst; q += nt) {
        lds[q] = q >= off[st] ? it.r[st][q - off[st]] : T(0);
        lds[kCoarseLdsPts + q] = T(0);
    }
    if (tid < 64) lds[2 * kCoarseLdsPts + tid] = T(0);
    __syncthreads();
    const SLevs<T> S{lds, off, lds + 2 * kCoarseLdsPts};
    coarse_down(L, S, st, 0);
    coarse_up(L, S, 0, st);
    // every staged level back to global memory (r below st, v of all)
    for (int q = tid; q < nst; q += nt) {
        int l = 0;
        while (l < st && q >= off[l + 1]) l++;
        const int k = q - off[l];
        if (l < st) it.r[l][k] = lds[q];
        it.v[l][k] = lds[kCoarseLdsPts + q];
    }
    __syncthreads();
    coarse_up(L, G, st + 1, top);
}

// ------------------------------------------------- learned coarse correction
// The cut level c (axis grid, 17 x 17 points) of one problem per workgroup.

__device__ inline double block_sum_d(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[w];
    return s;
}

// ||r - A v||^2 over the interior of an axis level of side m, A the 5-point
// Laplacian with spacing 1/m (the equation Lap v = r of Section 1)
template <typename T>
__device__ double cut_resid2(const T* __restrict__ r, const T* __restrict__ v, int m, double* red)
{
    double s = 0, m2 = (double)m * m;
    for (int q = threadIdx.x; q < (m - 1) * (m - 1); q += blockDim.x) {
        int a = q % (m - 1) + 1, b = q / (m - 1) + 1;
        size_t o = idxA(m, a, b), w = (size_t)(m + 1);
        double av = ((double)v[o - 1] + (double)v[o + 1] + (double)v[o - w] + (double)v[o + w] - 4.0 * (double)v[o]) * m2;
        double d = (double)r[o] - av;
        s += d * d;
    }
    return block_sum_d(s, red);
}

// Network inference on r_c (natural 17 x 17, spacing H = 1/16): the C
// points (a+b even) of the estimate of A_c^{-1} r_c go to vD (the diagonal
// level below, D layout of side 16).  Returns ||r_c||^2.
template <typename T>
__device__ double net_cut_2d(const T* __restrict__ rc, T* __restrict__ vD, const bf16_t* __restrict__ wf, bf16_t* A,
                             bf16_t* B, float* out0, short* linq, double* red)
{
    using N = NetGeo<2>;
    net_zero(A, N::ACT);
    net_zero(B, N::ACT);
    net_fill_lin<2>(linq);
    double ss = 0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        double x = (double)rc[N::lin(q)];
        ss += x * x;
    }
    ss = block_sum_d(ss, red);
    double rms = sqrt(ss / N::NIN);
    double sc = rms > 0 ? 1.0 / rms : 0.0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        int p = N::lin(q);
        A[p * kNetCh] = f2bf((float)((double)rc[p] * sc));
    }
    __syncthreads();
    const int WLY = N::WLY;
    net_conv_fwd<2, true>(A, B, nullptr, wf, linq);
    __syncthreads();
    net_conv_fwd<2, true>(B, A, nullptr, wf + WLY, linq);
    __syncthreads();
    net_conv_fwd<2, true>(A, B, nullptr, wf + 2 * WLY, linq);
    __syncthreads();
    net_conv_fwd<2, false>(B, nullptr, out0, wf + 3 * WLY, linq);
    __syncthreads();
    const double back = rms / ((N::G - 1) * (N::G - 1));
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        int a = q % N::IN + 1, b = q / N::IN + 1;
        if (((a + b) & 1) == 0) vD[idxD(N::G - 1, a, b)] = (T)((double)out0[q] * back);
    }
    __syncthreads();
    return ss;
}

// The coarse kernel with the network at the cut level.  Net state per
// problem (Ctl::net): 1 on the first cycle, where both the network and the
// plain sub-cycle run, the plain one's cut-level residual reduction becomes
// the bar theta and the better of the two is kept; 2 afterwards, where a
// cycle whose network correction misses the bar falls back to the plain
// sub-cycle and switches the network off (state 0) for the rest of the solve.
template <typename T>
__global__ void __launch_bounds__(kCoarseThreadsB) kb_coarse_net(CoarseLev<T> L, const Coarse2B<T>* __restrict__ items,
                                                                 const T* __restrict__ zero, Ctl* __restrict__ ctls,
                                                                 const bf16_t* __restrict__ wf)
{
    using N = NetGeo<2>;
    const Coarse2B<T>& it = items[blockIdx.x];
    ITEM_GATE(ctls, it.prob);
    Ctl* c = &ctls[it.prob];
    const int top = min(it.top, L.top_cap), cut = kNetCut;
    const int state = top >= cut ? c->net : 0;
    const GLevs<T> S{it, zero};
    if (state == 0) {
        coarse_down(L, S, top, 0);
        coarse_up(L, S, 0, top);
        return;
    }
    __shared__ __align__(16) bf16_t A[N::ACT];
    __shared__ __align__(16) bf16_t B[N::ACT];
    __shared__ float out0[N::TILES * 16];
    __shared__ short linq[N::LQ];
    __shared__ double red[kCoarseThreadsB / 64];
    __shared__ T vsave[(N::G) * (N::G / 2 + 1)];
    const int m = L.l[cut].m;
    const int nD = (int)sizeD(m);
    coarse_down(L, S, top, cut);
    double rn2 = net_cut_2d<T>(S.r(cut), S.v(cut - 1), wf, A, B, out0, linq, red);
    coarse_up(L, S, cut, cut);
    double qn = cut_resid2<T>(S.r(cut), S.v(cut), m, red);
    int next = state, used = 0;
    double theta = c->theta, qfirst = c->q_net;
    if (state == 1 || !(qn <= theta * theta * rn2)) {
        if (state == 1)
            for (int q = threadIdx.x; q < nD; q += blockDim.x) vsave[q] = S.v(cut - 1)[q];
        __syncthreads();
        coarse_down(L, S, cut, 0);
        coarse_up(L, S, 0, cut);
        double qp = cut_resid2<T>(S.r(cut), S.v(cut), m, red);
        if (state == 1) {
            theta = rn2 > 0 ? sqrt(qp / rn2) : 0.0;
            qfirst = rn2 > 0 ? sqrt(qn / rn2) : 0.0;
            if (qn <= qp) {   // the network wins the first cycle
                for (int q = threadIdx.x; q < nD; q += blockDim.x) S.v(cut - 1)[q] = vsave[q];
                __syncthreads();
                coarse_up(L, S, cut, cut);
                next = 2;
                used = 1;
            } else {
                next = 0;
            }
        } else {
            next = 0;
        }
    } else {
        used = 1;
    }
    coarse_up(L, S, cut + 1, top);
    if (threadIdx.x == 0) {
        c->net = next;
        c->theta = theta;
        c->q_net = qfirst;
        c->net_used += used;
        if (next == 0) c->net_off = 1;
    }
}

// ================================================================ decisions
// Per-problem norm and stopping decision (Section 1): one workgroup per
// problem sums its partials in a fixed order.  kind 0: ||f|| into fnorm;
// kind 1: relative residual of evaluation ctl.k, then stop when it is <= rtol,
// not finite, grew three times in a row above the start, or after
// max_cycles cycles.  A problem that stops decrements *nactive.  host (a
// single problem's solve): a pinned host copy of the control block that
// receives the decision, the relative residual and its history entry.
template <typename T>
__global__ void __launch_bounds__(256) kb_finalize(int kind, const Fin2<T>* __restrict__ items, int nparts,
                                                   Ctl* __restrict__ ctls, int* __restrict__ nactive,
                                                   Ctl* __restrict__ host)
{
    const Fin2<T> it = items[blockIdx.x];
    Ctl* c = &ctls[it.prob];
    if (c->done) return;
    __shared__ double red[256];
    auto reduce = [&](const double* a) {
        double s = 0;
        for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += a[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        const double t = red[0];
        __syncthreads();
        return t;
    };
    // kind 2: ||f|| from the residual kernel's f^2 partials, then as kind 1
    if (kind == 2) {
        const double tf = reduce(it.partf);
        if (threadIdx.x == 0) c->fnorm = sqrt(tf);
        kind = 1;
    }
    const double tot = reduce(it.part);
    if (threadIdx.x != 0) return;
    if (kind == 0) {
        c->fnorm = sqrt(tot);
        return;
    }
    int k = c->k;  // evaluation index = cycles run so far
    double rn = sqrt(tot);
    double rr = c->fnorm > 0 ? rn / c->fnorm : rn;
    c->last = rr;
    if (k <= kMaxCycles) c->hist[k] = rr;
    c->k = k + 1;
    if (c->mode == 0) return;
    int finite = isfinite(rr);
    if (k == 0) {
        c->rr0 = rr;
        c->prev = rr;
        c->grow = 0;
        if (rr <= c->rtol) { c->status = 0; c->done = 1; }
        else if (c->max_cycles == 0) { c->status = -8; c->done = 1; }
        else if (!finite) { c->status = -6; c->done = 1; }
    } else {
        if (!finite) { c->status = -6; c->done = 1; }
        else {
            c->grow = (rr > c->prev) ? c->grow + 1 : 0;
            c->prev = rr;
            if (c->grow >= 3 && rr > c->rr0) { c->status = -7; c->done = 1; }
            else if (rr <= c->rtol) { c->status = 0; c->done = 1; }
            else if (k >= c->max_cycles) { c->status = -8; c->done = 1; }
        }
    }
    if (c->done) {
        c->cycles = k;
        atomicSub(nactive, 1);
    }
    // a single problem's state straight into host memory (read by the host
    // after an event or a synchronisation that follows this kernel)
    if (host) {
        if (k <= kMaxCycles) host->hist[k] = rr;
        host->last = rr;
        host->status = c->status;
        host->cycles = c->cycles;
        host->done = c->done;
        host->k = k + 1;   // evaluations done: what the host loop polls
    }
}

__global__ void kb_ctl_reset(Ctl* ctls, int nprob, int mode, int max_cycles, double rtol, int* nactive, int net)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) *nactive = nprob;
    if (p >= nprob) return;
    Ctl* c = &ctls[p];
    c->done = 0;
    c->status = 0;
    c->cycles = 0;
    c->grow = 0;
    c->mode = mode;
    c->max_cycles = max_cycles;
    c->k = 0;
    c->rtol = rtol;
    c->fnorm = 0;
    c->rr0 = c->prev = c->last = 0;
    c->net = net;
    c->theta = 0;
    c->q_net = 0;
    c->net_used = 0;
    c->net_off = 0;
}

template <typename T>
void launch_b_finalize(int kind, const Fin2<T>* items, int nitems, int nparts, Ctl* ctls, int* nactive, hipStream_t s,
                       Ctl* host)
{
    hipLaunchKernelGGL(kb_finalize<T>, dim3(nitems), dim3(256), 0, s, kind, items, nparts, ctls, nactive,
                       nitems == 1 ? host : nullptr);
}

void launch_b_ctl_reset(Ctl* ctls, int nprob, int mode, int max_cycles, double rtol, int* nactive, int net,
                        hipStream_t s)
{
    hipLaunchKernelGGL(kb_ctl_reset, dim3((nprob + 255) / 256), dim3(256), 0, s, ctls, nprob, mode, max_cycles, rtol,
                       nactive, net);
}

// level -> natural double array (parity tests)
template <typename T>
__global__ void kb_level_get(int diag, int m, const T* __restrict__ src, double* __restrict__ dst)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y;
    if (a > m || b > m) return;
    double x = 0;
    if (!diag) x = (double)src[idxA(m, a, b)];
    else if (((a + b) & 1) == 0) x = (double)src[idxD(m, a, b)];
    dst[idxA(m, a, b)] = x;
}

// restricted residual of aligned level lam of every coarse item's problem,
// natural layout (points off a diagonal level read 0), problem-major
template <typename T>
__global__ void kb_coarse_export(int lam, int diag, int m, const Coarse2B<T>* __restrict__ items,
                                 double* __restrict__ dst)
{
    const Coarse2B<T>& it = items[blockIdx.x];
    double* d = dst + (size_t)it.prob * sizeA(m);
    const T* src = lam <= it.top ? it.r[lam] : nullptr;
    for (int q = threadIdx.x; q < (int)sizeA(m); q += blockDim.x) {
        int a = q % (m + 1), b = q / (m + 1);
        double x = 0;
        if (src) {
            if (!diag) x = (double)src[idxA(m, a, b)];
            else if (((a + b) & 1) == 0) x = (double)src[idxD(m, a, b)];
        }
        d[q] = x;
    }
}

template <typename T>
void launch_b_coarse_export(int lam, int diag, int m, const Coarse2B<T>* items, int nitems, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(kb_coarse_export<T>, dim3(nitems), dim3(256), 0, s, lam, diag, m, items, dst);
}

template <typename T>
void launch_b_level_get(int diag, int m, const T* src, double* dst, hipStream_t s)
{
    dim3 g((m + 1 + 255) / 256, m + 1);
    hipLaunchKernelGGL(kb_level_get<T>, g, dim3(256), 0, s, diag, m, src, dst);
}

// ================================================================= launchers
constexpr int kChunkRsPair = 2;
constexpr int kChunkResid = 4, kChunkA2D = 1, kChunkD2A = 4, kChunkJDiag = 2, kChunkJAxis = 1;
constexpr int kTargetWavesResid = 8192;  // ~120 VGPRs: 16 waves per CU
constexpr int kRowsMinSide = 512;        // smaller levels: one thread per point
// Non-temporal f and r0 accesses (a compile-time choice: a branch inside the
// kernels measured slower) only where one array alone is larger than the
// 256 MB MALL could keep; measured on MI355X: -5% solve time at 4097^2,
// +3.5% on the batch of grids up to 1025^2 if used there.
static inline bool nt_hint(int n) { return n >= 4096; }

// Strip length: the longest (fewest halo rows) that still gives the grid
// about `target` waves, so every wave is resident in one round.
static inline int pick_rows(int ncols_units, int per_wave, int nrows, int target = kTargetWaves)
{
    int nwx = (ncols_units + per_wave - 1) / per_wave;
    int r = kMaxRows;
    while (r > 4 && (long)nwx * ((nrows + r - 1) / r) < target) r >>= 1;
    return r;
}

// Waves of `kern` (kRowBlock threads per block) the device holds at once,
// from the compiled kernel's occupancy; cached per kernel and device.
static int resident_waves(const void* kern)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto key = std::make_pair(kern, dev);
    std::lock_guard<std::mutex> lock(mu);
    auto f = cache.find(key);
    if (f != cache.end()) return f->second;
    int blocks = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, kRowBlock, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        blocks = cus = 0;
    const int w = blocks * cus * kWavesPerBlock;
    cache[key] = w;
    return w;
}

// Strip length for a single problem: the shortest whose waves all fit on the
// device at once (more waves in flight, one round, no tail); pick_rows when
// no length up to 2 kMaxRows fits or the count is unknown.
static inline int fill_rows(const void* kern, int ncols_units, int per_wave, int nrows)
{
    const int cap = resident_waves(kern);
    const int nwx = (ncols_units + per_wave - 1) / per_wave;
    if (cap > 0)
        for (int r = 4; r <= 2 * kMaxRows; r++)
            if ((long)nwx * ((nrows + r - 1) / r) <= cap) return r;
    return pick_rows(ncols_units, per_wave, nrows);
}

static inline void rows_grid(int ncols_units, int per_wave, int nrows, int rows, int& nwx, int& nwaves, int& nblocks)
{
    nwx = (ncols_units + per_wave - 1) / per_wave;
    int nsy = (nrows + rows - 1) / rows;
    nwaves = nwx * nsy;
    nblocks = (nwaves + kWavesPerBlock - 1) / kWavesPerBlock;
}

// kind: 0 a2d restriction, 1 d2a restriction, 2 diagonal Jacobi, 3 axis Jacobi
int b_default_rows(int kind, int m)
{
    if (m < kRowsMinSide) return 0;
    switch (kind) {
    case 0: return pick_rows(m / 2 + 1, kPairsPerWave, m - 1);
    case 1: return pick_rows(m / 2 + 1, kColsPerWave, m / 2 - 1);
    case 2: return pick_rows(m / 2, kPairsPerWave, m / 2);
    default: return pick_rows(m / 2 + 1, kPairsPerWave, m - 1);
    }
}

int b_resid_parts(int n)
{
    if (n < 4) return 1;
    int nwx, nw, nb;
    rows_grid(n / 2 + 1, kResidPairs, n - 1, pick_rows(n / 2 + 1, kResidPairs, n - 1, kTargetWavesResid), nwx, nw,
              nb);
    return nb;
}

// A launch that takes the events of an open timing bracket, if any
template <typename K, typename... Args>
static void launch_timed(K kern, dim3 g, dim3 b, hipStream_t s, Args... args)
{
    TimedSlot*& ts = timed_slot();
    if (ts) {
        hipExtLaunchKernelGGL(kern, g, b, 0, s, ts->beg, ts->end, 0, args...);
        ts = nullptr;
    } else {
        hipLaunchKernelGGL(kern, g, b, 0, s, args...);
    }
}

__global__ void kb_copy_ring(int n, const double* __restrict__ src, double* __restrict__ dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const size_t w = (size_t)n + 1;
    dst[i] = src ? src[i] : 0.0;                                     // row 0
    dst[(size_t)n * w + i] = src ? src[(size_t)n * w + i] : 0.0;     // row n
    dst[(size_t)i * w] = src ? src[(size_t)i * w] : 0.0;             // column 0
    dst[(size_t)i * w + n] = src ? src[(size_t)i * w + n] : 0.0;     // column n
}

void launch_b_copy_ring(int n, const double* src, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(kb_copy_ring, dim3((n + 1 + 255) / 256), dim3(256), 0, s, n, src, dst);
}

// End of an out-of-place solve: the interior of the last iterate into u when
// it is in ub (odd cycle count), and ub's boundary back to zero.
__global__ void kb_oop_finish(int n, const Ctl* __restrict__ ctl, double* __restrict__ ub, double* __restrict__ u)
{
    const size_t w = (size_t)n + 1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        ub[i] = 0.0;
        ub[(size_t)n * w + i] = 0.0;
        ub[(size_t)i * w] = 0.0;
        ub[(size_t)i * w + n] = 0.0;
    }
    if (!(ctl->cycles & 1)) return;
    for (int b = blockIdx.x + 1; b < n; b += gridDim.x)
        for (int a = threadIdx.x + 1; a < n; a += blockDim.x) u[(size_t)b * w + a] = ub[(size_t)b * w + a];
}

void launch_b_oop_finish(int n, const Ctl* ctl, double* ub, double* u, hipStream_t s)
{
    hipLaunchKernelGGL(kb_oop_finish, dim3(n - 1 < 2048 ? n - 1 : 2048), dim3(256), 0, s, n, ctl, ub, u);
}

void launch_b_rhs4(int n, const double* f, double* g, hipStream_t s)
{
    hipLaunchKernelGGL(kb_rhs4, dim3((n - 1 + 255) / 256, n - 1), dim3(256), 0, s, n, f, g);
}

template <typename T>
void launch_b_resid(int n, int fused, int order, const Fin2<T>* items, int nitems, const Ctl* ctls, hipStream_t s,
                    int withf, int oop)
{
    const bool m4 = order == 4;
    double inv_h2 = m4 ? (double)n * (double)n / 6 : (double)n * (double)n;
    if (n < 4) {
        launch_timed(kb_resid_small<T>, dim3(1, nitems), dim3(kRowBlock), s, n, inv_h2, items, ctls, m4 ? 1 : 0);
        return;
    }
    int nwx, nw, nb;
    // rows is a power of two >= 4: every strip starts on an odd row
    int rows = pick_rows(n / 2 + 1, kResidPairs, n - 1, kTargetWavesResid);
    rows_grid(n / 2 + 1, kResidPairs, n - 1, rows, nwx, nw, nb);
    const int pp = oop && fused && n >= 8 && !m4 ? 1 : 0;
    auto go = [&](auto kern) {
        launch_timed(kern, dim3(nb, nitems), dim3(kRowBlock), s, n, inv_h2, items, nwx, nw, rows, ctls, pp);
    };
    const bool nt = nt_hint(n);
    auto pick = [&](auto M, auto F) {
        constexpr bool M4 = decltype(M)::value != 0, WF = decltype(F)::value != 0;
        if (fused && n >= 8) {
            if (nt) go(kb_resid<T, kChunkResid, true, true, M4, WF>);
            else go(kb_resid<T, kChunkResid, false, true, M4, WF>);
        } else {
            if (nt) go(kb_resid<T, kChunkResid, true, false, M4, WF>);
            else go(kb_resid<T, kChunkResid, false, false, M4, WF>);
        }
    };
    if (m4) { if (withf) pick(Int<1>{}, Int<1>{}); else pick(Int<1>{}, Int<0>{}); }
    else { if (withf) pick(Int<0>{}, Int<1>{}); else pick(Int<0>{}, Int<0>{}); }
}

template <typename T>
void launch_b_sumsq(int n, const Fin2<T>* items, int nitems, const Ctl* ctls, hipStream_t s)
{
    hipLaunchKernelGGL(kb_sumsq<T>, dim3(b_resid_parts(n), nitems), dim3(kRowBlock), 0, s, n, items, ctls);
}

template <typename T>
void launch_b_finest(int n, T c, T c1, int fused, const Fin2<T>* items, int nitems, const Ctl* ctls, hipStream_t s,
                     int oop)
{
    if (n < 8) {
        launch_timed(kb_finest_small<T>, dim3(1, nitems), dim3(kRowBlock), s, n, c, items, ctls);
        return;
    }
    int nwx, nw, nb;
    if (fused && oop && nitems == 1) {
        auto go = [&](auto kern) {
            const int rows = fill_rows((const void*)kern, n / 2 + 1, kFusePairs, n - 1);
            rows_grid(n / 2 + 1, kFusePairs, n - 1, rows, nwx, nw, nb);
            launch_timed(kern, dim3(nb, 1), dim3(kRowBlock), s, n, c, c1, items, nwx, nw, rows, ctls);
        };
        // plain loads: the iterate and f rows a strip shares with its
        // neighbour are then still in L2 when the neighbour reads them
        // (non-temporal ones measured 485.7 against 467.4 MB per launch)
        go(kb_finest_oop<T>);
        return;
    }
    if (fused) {
        auto go = [&](auto kern) {
            const int rows = nitems == 1 ? fill_rows((const void*)kern, n / 2 + 1, kFusePairs, n - 1)
                                         : pick_rows(n / 2 + 1, kFusePairs, n - 1);
            rows_grid(n / 2 + 1, kFusePairs, n - 1, rows, nwx, nw, nb);
            launch_timed(kern, dim3(nb, nitems), dim3(kRowBlock), s, n, c, c1, items, nwx, nw, rows, ctls);
        };
        if (nt_hint(n)) go(kb_finest_fused<T, true>);
        else go(kb_finest_fused<T, false>);
        return;
    }
    int rows = pick_rows(n / 2 + 1, kPairsPerWave, n - 1);
    rows_grid(n / 2 + 1, kPairsPerWave, n - 1, rows, nwx, nw, nb);
    if (nt_hint(n))
        launch_timed((kb_finest<T, kChunkJAxis, true>), dim3(nb, nitems), dim3(kRowBlock), s, n, c, items, nwx,
                     nw, rows, ctls);
    else
        launch_timed((kb_finest<T, kChunkJAxis, false>), dim3(nb, nitems), dim3(kRowBlock), s, n, c, items, nwx,
                     nw, rows, ctls);
}

// the grid of kb_finest_res: one round of waves, strips of even length
template <typename T>
static void finest_res_grid(int n, int& rows, int& nwx, int& nw, int& nb)
{
    rows = fill_rows((const void*)kb_finest_res<T>, n / 2 + 1, kResPairs, n - 1);
    rows += rows & 1;
    rows_grid(n / 2 + 1, kResPairs, n - 1, rows, nwx, nw, nb);
}

template <typename T>
bool b_finest_res_fits(int n, int nparts)
{
    if (n < 8) return false;
    int rows, nwx, nw, nb;
    finest_res_grid<T>(n, rows, nwx, nw, nb);
    return nb <= nparts;
}

template <typename T>
void launch_b_finest_res(int n, T c, T c1, const Fin2<T>* items, const Ctl* ctls, int nparts, hipStream_t s)
{
    int rows, nwx, nw, nb;
    finest_res_grid<T>(n, rows, nwx, nw, nb);
    launch_timed(kb_finest_res<T>, dim3(nb, 1), dim3(kRowBlock), s, n, c, c1, items, nwx, nw, rows, ctls, nparts);
}

template <typename T>
void launch_b_rs_pair(int m, const RsPair2<T>* items, int nitems, const Ctl* ctls, hipStream_t s)
{
    int nwx, nw, nb;
    // rows is a power of two >= 4: every strip starts on an odd row
    int rows = pick_rows(m / 2 + 1, kResidPairs, m - 1);
    rows_grid(m / 2 + 1, kResidPairs, m - 1, rows, nwx, nw, nb);
    hipLaunchKernelGGL((kb_rs_pair<T, kChunkRsPair>), dim3(nb, nitems), dim3(kRowBlock), 0, s, m, items, nwx, nw, rows,
                       ctls);
}

template <typename T>
void launch_b_jac_pair(int m, T cc, T cd, const JPair2<T>* items, int nitems, const Ctl* ctls, hipStream_t s)
{
    int nwx, nw, nb;
    int rows = pick_rows(m / 2 + 1, kFusePairs, m - 1);
    rows_grid(m / 2 + 1, kFusePairs, m - 1, rows, nwx, nw, nb);
    hipLaunchKernelGGL(kb_jac_pair<T>, dim3(nb, nitems), dim3(kRowBlock), 0, s, m, cc, cd, items, nwx, nw, rows, ctls);
}

template <typename T>
void launch_b_restrict(int diag_in, int m, int rows, const Item2<T>* items, int nitems, const Ctl* ctls,
                       hipStream_t s)
{
    int nwx, nw, nb;
    if (!diag_in) {
        if (rows <= 0) {
            dim3 g((m / 2 + 1 + 255) / 256, m - 1, nitems);
            hipLaunchKernelGGL(kb_rs_a2d<T>, g, dim3(256), 0, s, m, items, ctls);
            return;
        }
        rows_grid(m / 2 + 1, kPairsPerWave, m - 1, rows, nwx, nw, nb);
        hipLaunchKernelGGL((kb_a2d_rows<T, kChunkA2D>), dim3(nb, nitems), dim3(kRowBlock), 0, s, m, items, nwx, nw,
                           rows, ctls);
    } else {
        int mc = m / 2;
        if (mc < 2) return;
        if (rows <= 0) {
            dim3 g((mc - 1 + 255) / 256, mc - 1, nitems);
            hipLaunchKernelGGL(kb_rs_d2a<T>, g, dim3(256), 0, s, m, items, ctls);
            return;
        }
        rows_grid(m / 2 + 1, kColsPerWave, m / 2 - 1, rows, nwx, nw, nb);
        hipLaunchKernelGGL((kb_d2a_rows<T, kChunkD2A>), dim3(nb, nitems), dim3(kRowBlock), 0, s, m, items, nwx, nw,
                           rows, ctls);
    }
}

template <typename T>
void launch_b_jacobi(int diag, int m, int rows, T c, const Item2<T>* items, int nitems, const Ctl* ctls,
                     hipStream_t s)
{
    int nwx, nw, nb;
    if (diag) {
        if (rows <= 0) {
            dim3 g((m / 2 + 255) / 256, m / 2, nitems);
            hipLaunchKernelGGL(kb_jac_diag<T>, g, dim3(256), 0, s, m, c, items, ctls);
            return;
        }
        rows_grid(m / 2, kPairsPerWave, m / 2, rows, nwx, nw, nb);
        hipLaunchKernelGGL((kb_jdiag_rows<T, kChunkJDiag>), dim3(nb, nitems), dim3(kRowBlock), 0, s, m, c, items, nwx,
                           nw, rows, ctls);
    } else {
        if (rows <= 0) {
            dim3 g((m / 2 + 1 + 255) / 256, m - 1, nitems);
            hipLaunchKernelGGL(kb_jac_axis<T>, g, dim3(256), 0, s, m, c, items, ctls);
            return;
        }
        rows_grid(m / 2 + 1, kPairsPerWave, m - 1, rows, nwx, nw, nb);
        hipLaunchKernelGGL((kb_jaxis_rows<T, kChunkJAxis>), dim3(nb, nitems), dim3(kRowBlock), 0, s, m, c, items, nwx,
                           nw, rows, ctls);
    }
}

template <typename T>
void launch_b_mid_down(const T* r14, T* const* r, const Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(kb_mid_down<T>, dim3(kMidTiles * kMidTiles), dim3(kMidThreads), 0, s, r14, r[5], r[4], r[3],
                       r[2], r[1], r[0], ctl);
}

template <typename T>
void launch_b_mid_up(const T* v8, const T* const* r, T* const* v, const T* c, const Ctl* ctl, hipStream_t s)
{
    MidUp<T> L;
    for (int k = 0; k < 6; k++) {
        L.r[k] = r[k];
        L.v[k] = v[k];
        L.c[k] = c[k];
    }
    hipLaunchKernelGGL(kb_mid_up<T>, dim3(kMidTiles * kMidTiles), dim3(kMidThreads), 0, s, v8, L, ctl);
}

template <typename T>
void launch_b_coarse(const LevInfo<T>* lev, const Coarse2B<T>* items, int nitems, const T* zero, const Ctl* ctls,
                     hipStream_t s, int top_cap)
{
    CoarseLev<T> L;
    for (int i = 0; i < kCoarseLevels; i++) L.l[i] = lev[i];
    L.top_cap = top_cap;
    hipLaunchKernelGGL(kb_coarse<T>, dim3(nitems), dim3(kCoarseThreadsB), 0, s, L, items, zero, ctls);
}

template <typename T>
void launch_b_coarse_net(const LevInfo<T>* lev, const Coarse2B<T>* items, int nitems, const T* zero, Ctl* ctls,
                         const bf16_t* wf, hipStream_t s, int top_cap)
{
    CoarseLev<T> L;
    for (int i = 0; i < kCoarseLevels; i++) L.l[i] = lev[i];
    L.top_cap = top_cap;
    hipLaunchKernelGGL(kb_coarse_net<T>, dim3(nitems), dim3(kCoarseThreadsB), 0, s, L, items, zero, ctls, wf);
}

#define DMG_INSTB(T)                                                                                            \
    template void launch_b_resid<T>(int, int, int, const Fin2<T>*, int, const Ctl*, hipStream_t, int, int);                   \
    template void launch_b_sumsq<T>(int, const Fin2<T>*, int, const Ctl*, hipStream_t);                        \
    template void launch_b_finest<T>(int, T, T, int, const Fin2<T>*, int, const Ctl*, hipStream_t, int);          \
    template bool b_finest_res_fits<T>(int, int);                                                              \
    template void launch_b_finest_res<T>(int, T, T, const Fin2<T>*, const Ctl*, int, hipStream_t);            \
    template void launch_b_restrict<T>(int, int, int, const Item2<T>*, int, const Ctl*, hipStream_t);          \
    template void launch_b_jac_pair<T>(int, T, T, const JPair2<T>*, int, const Ctl*, hipStream_t);              \
    template void launch_b_rs_pair<T>(int, const RsPair2<T>*, int, const Ctl*, hipStream_t);                    \
    template void launch_b_jacobi<T>(int, int, int, T, const Item2<T>*, int, const Ctl*, hipStream_t);         \
    template void launch_b_coarse<T>(const LevInfo<T>*, const Coarse2B<T>*, int, const T*, const Ctl*, hipStream_t, \
                                     int);                                                                    \
    template void launch_b_finalize<T>(int, const Fin2<T>*, int, int, Ctl*, int*, hipStream_t, Ctl*);          \
    template void launch_b_level_get<T>(int, int, const T*, double*, hipStream_t);                           \
    template void launch_b_coarse_net<T>(const LevInfo<T>*, const Coarse2B<T>*, int, const T*, Ctl*, const bf16_t*, \
                                         hipStream_t, int);                                                     \
    template void launch_b_coarse_export<T>(int, int, int, const Coarse2B<T>*, int, double*, hipStream_t);       \
    template void launch_b_mid_down<T>(const T*, T* const*, const Ctl*, hipStream_t);                         \
    template void launch_b_mid_up<T>(const T*, const T* const*, T* const*, const T*, const Ctl*, hipStream_t);
DMG_INSTB(double)
DMG_INSTB(float)

}  // namespace dmg

// 3D kernels of libdmg: restrictions Eqs. (Erred), (Ermagc), (Ermagm),
// (Erblu) and the Jacobi steps Eqs. (Emprolm)-(Egprolr) of Roberts,
// Section 3.  As in 2D, each Jacobi thread owns the points of one cell and
// recomputes the first-half-sweep values its second-half-sweep point needs,
// so both half-sweeps run in one launch.
#include "dmg_launch.hpp"
#include "dmg_launch3.hpp"
#include "dmg_net_dev.hpp"
#include "dmg_rows.hpp"

namespace dmg {

#define DMG_GATE(ctl) \
    if ((ctl) != nullptr && (ctl)->done) return

// ------------------------------------------------------------ restriction

// The one-thread-per-point kernels below take blockDim.y rows of a plane per
// workgroup (x: the row's points, blockDim.x of them at a time), so that a
// short row does not leave most of a 256-thread workgroup idle.

// green (side m) -> red (side m): one thread per R-layout slot
template <typename T>
__global__ void __launch_bounds__(256) k3_rs_g2r(int m, const T* __restrict__ rG, T* __restrict__ rR, const Ctl* ctl)
{
    DMG_GATE(ctl);
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    int b = blockIdx.y * blockDim.y + threadIdx.y + 1, c = blockIdx.z + 1;
    if (col > m / 2 || b >= m) return;
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
    int B = blockIdx.y * blockDim.y + threadIdx.y, C = blockIdx.z;
    if (A >= h || B >= h) return;
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
    int B = blockIdx.y * blockDim.y + threadIdx.y + 1, C = blockIdx.z + 1;
    if (A >= mc || B >= mc) return;
    rB[idxG(mc, A, B, C)] = rs3_m2b(rE, rO, m, A, B, C);
}

// red (side m) -> magenta, plane-marching (sides >= 128).  A workgroup owns
// 32 x 8 magenta half-index columns (A, B) and marches a chunk of fine
// planes c: plane c holds corners (c even) or cube centres (c odd), and both
// stencils read red planes c-1, c, c+1 only.  Each red plane is staged in
// LDS once per chunk (the tile's slots plus a one-slot halo, rows 2B0-1 ..
// 2B0+16), a ring of three planes; the next plane is loaded into registers
// while the current one is computed.  Same terms in the same order as
// rs3_r2mE / rs3_r2mO.
constexpr int kRmTA = 32, kRmTB = 8, kRmThreads = kRmTA * kRmTB;
constexpr int kRmS = kRmTA + 2, kRmH = 2 * kRmTB + 2, kRmN = kRmS * kRmH;
constexpr int kRmP = (kRmN + kRmThreads - 1) / kRmThreads;   // staged red slots per thread

template <typename T>
__global__ void __launch_bounds__(kRmThreads) k3_r2m_planes(int m, const T* __restrict__ rR, T* __restrict__ rE,
                                                             T* __restrict__ rO, int nta, int ntb, int zc,
                                                             const Ctl* ctl)
{
    DMG_GATE(ctl);
    __shared__ T Rp[3][kRmN];
    const int h = m / 2;
    const int bid = xcd_block();   // tiles of one die are neighbours
    const int ta = bid % nta, tb = (bid / nta) % ntb, tz = bid / (nta * ntb);
    const int A0 = ta * kRmTA, B0 = tb * kRmTB;
    const int z0 = 1 + tz * zc, z1 = min(z0 + zc, m);   // output planes [z0, z1)
    const int tid = threadIdx.x;
    const int yb = 2 * B0 - 1, sb = A0 - 1;   // fine row and slot of staged element 0
    // staged red value e of plane c (0 off the grid)
    auto rload = [&](int c, int e) -> T {
        if (e >= kRmN) return T(0);
        const int b = yb + e / kRmS, sl = sb + e % kRmS;
        const int a = 2 * sl + ((b + c) & 1);
        if (sl < 0 || a > m || b < 0 || b > m || c < 0 || c > m) return T(0);
        return rR[idxR(m, a, b, c)];
    };
    T nx[kRmP];
#pragma unroll
    for (int k = 0; k < kRmP; k++) {
        const int e = tid + k * kRmThreads;
        const T v0 = rload(z0 - 1, e), v1 = rload(z0, e);
        if (e < kRmN) {
            Rp[(z0 + 2) % 3][e] = v0;
            Rp[z0 % 3][e] = v1;
        }
        nx[k] = rload(z0 + 1, e);
    }
    const int A = A0 + tid % kRmTA, B = B0 + tid / kRmTA;
    for (int c = z0; c < z1; c++) {
#pragma unroll
        for (int k = 0; k < kRmP; k++) {   // red plane c+1
            const int e = tid + k * kRmThreads;
            if (e < kRmN) Rp[(c + 1) % 3][e] = nx[k];
        }
        if (c + 1 < z1) {
#pragma unroll
            for (int k = 0; k < kRmP; k++) nx[k] = rload(c + 2, tid + k * kRmThreads);
        }
        __syncthreads();
        const T* Rm = Rp[(c + 2) % 3];   // plane c-1
        const T* R0 = Rp[c % 3];
        const T* Rq = Rp[(c + 1) % 3];   // plane c+1
        // staged position of red point (a, b) of any plane
        auto at = [&](int a, int b) { return (b - yb) * kRmS + ((a >> 1) - sb); };
        if (c & 1) {   // cube centre (2A+1, 2B+1, c), Eq. (Ermagm)
            const int a = 2 * A + 1, b = 2 * B + 1;
            if (A < h && B < h)
                rO[idxMO(m, a, b, c)] = (R0[at(a + 1, b)] + R0[at(a - 1, b)] + R0[at(a, b + 1)] + R0[at(a, b - 1)] +
                                         Rq[at(a, b)] + Rm[at(a, b)]) * (T(1) / T(6));
        } else {       // corner (2A, 2B, c), Eq. (Ermagc)
            const int a = 2 * A, b = 2 * B;
            if (A >= 1 && A < h && B >= 1 && B < h && c >= 2 && c <= m - 2)
                rE[idxME(m, a, b, c)] =
                    (12 * R0[at(a, b)] + R0[at(a + 1, b + 1)] + R0[at(a + 1, b - 1)] + R0[at(a - 1, b - 1)] +
                     R0[at(a - 1, b + 1)] + Rq[at(a + 1, b)] + Rm[at(a + 1, b)] + Rm[at(a - 1, b)] + Rq[at(a - 1, b)] +
                     Rq[at(a, b + 1)] + Rm[at(a, b + 1)] + Rm[at(a, b - 1)] + Rq[at(a, b - 1)]) * (T(1) / T(24));
        }
        __syncthreads();
    }
}

// smaller red levels (too few tiles at 128), and single-precision levels
// (half the bytes: the point kernel measured as fast), use one thread per point
constexpr int kRmPlMinSide = 256;

// a 256-thread block shape for rows of len points: x the row (a multiple of
// 64, at most 256), y the rows per block; and the grid over rows x planes
inline void row_blocks(int len, int rows, int planes, dim3& blk, dim3& grd)
{
    const int bx = len >= 256 ? 256 : (len + 63) / 64 * 64;
    blk = dim3(bx, 256 / bx);
    grd = dim3((len + bx - 1) / bx, (rows + blk.y - 1) / blk.y, planes);
}

template <typename T>
void launch_rs3(const Lev3<T>& F, const Lev3<T>& Cc, const Ctl* ctl, hipStream_t s)
{
    int m = F.m;
    dim3 blk, g;
    if (Cc.kind == 1) {
        // slot m/2 holds no interior point (a >= m): rows of m/2 slots
        row_blocks(m / 2, m - 1, m - 1, blk, g);
        hipLaunchKernelGGL(k3_rs_g2r<T>, g, blk, 0, s, m, F.r, Cc.r, ctl);
    } else if (Cc.kind == 2) {
        if (m >= kRmPlMinSide && sizeof(T) == 8) {
            const int h = m / 2, nta = (h + kRmTA - 1) / kRmTA, ntb = (h + kRmTB - 1) / kRmTB, zc = 8;
            const int ntz = (m - 1 + zc - 1) / zc;
            hipLaunchKernelGGL(k3_r2m_planes<T>, dim3(nta * ntb * ntz), dim3(kRmThreads), 0, s, m, F.r, Cc.r, Cc.r2,
                               nta, ntb, zc, ctl);
            return;
        }
        row_blocks(m / 2, m / 2, m / 2, blk, g);
        hipLaunchKernelGGL(k3_rs_r2m<T>, g, blk, 0, s, m, F.r, Cc.r, Cc.r2, ctl);
    } else {
        int mc = m / 2;
        if (mc < 2) return;
        row_blocks(mc - 1, mc - 1, mc - 1, blk, g);
        hipLaunchKernelGGL(k3_rs_m2b<T>, g, blk, 0, s, m, F.r, F.r2, Cc.r, ctl);
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

// ------------------------------------------------------- plane-marching Jacobi
// Large levels: a workgroup owns an (x, y) tile and marches a chunk of z
// planes.  For each plane it computes the first-half-sweep values of the
// tile plus a one-point halo once, into a ring of three LDS planes; the
// second-half-sweep points of the plane behind then read the values they
// need from LDS, summed in the same order as the per-point functions, so the
// results equal those of the one-thread-per-point kernels bit for bit.

constexpr int kPlTX = 64, kPlTY = 8, kPlThreads = 256;
constexpr int kPlW = kPlTX + 2;   // tile width plus a one-point halo
constexpr int kRdTX = 32, kRdW = kRdTX + 2;        // red tiles: 32 slots (64 x positions) wide
constexpr int kRdTY = 16, kRdH = kRdTY + 2;        // red tiles: rows (with 512 threads; 8 rows and
constexpr int kRdThreads = 512;                     // 256 threads, or 32 rows and 1024, measured slower)

// ---- green: F points (a+b+c odd), Eq. (Egprolg).  The red grid is staged
// plane by plane in LDS over the tile plus a two-point halo: row (b, c) of
// the red grid holds a = 2s + ((b+c)&1) at slot s, so the 35 slots from
// s = (x0-3)/2 cover a in [x0-2, x0+65] for either parity and load as one
// contiguous run; each red value is then loaded once instead of once per
// F neighbour.
// Green tiles: 64 x 16 points, 512 threads (the red halo rows of a plane are
// 1.25 times the tile's instead of 1.5 for 64 x 8).
constexpr int kGrTY = 16, kGrThreads = 512, kGrH = kGrTY + 2;
constexpr int kGrRS = 35, kGrRH = kGrTY + 4;                    // red LDS plane: rows y0-2 .. y0+17
constexpr int kGrRN = kGrRS * kGrRH;
constexpr int kGrRP = (kGrRN + kGrThreads - 1) / kGrThreads;   // red slots per thread

// Green grid of side m, Eqs. (Egprolg), (Egprolr): F points from the red
// grid vR, then C points (a+b+c even) from the six new F values.  FINEST
// adds the correction to u instead of storing it.  Thread (oly, opr) owns
// the x pair (oa, oa+1) = (x0 + 2 opr, x0 + 2 opr + 1) of row y0 + oly: one
// point of the pair is an F point of a plane and the other a C point, so the
// thread reads the pair's residuals of a plane as one 16-byte access and
// computes the F value of its own pair itself; 82 threads also compute one F
// point of the one-point halo ring of the tile (rows y0-1 and y0+16, and the
// one column of x0-1, x0+64 that holds an F point of the row).  Per plane c
// a thread stages red slots of plane c+2 into registers, writes those of
// plane c+1 into the red ring, computes F values of plane c into a second
// ring, and then the pair of plane c-1 from them; the inputs of the next
// plane are loaded meanwhile.
template <typename T, bool FINEST>
__global__ void __launch_bounds__(kGrThreads) k3_green_planes(int m, T cc, const T* __restrict__ rG,
                                                               const T* __restrict__ vR, T* __restrict__ vG,
                                                               double* __restrict__ u, int ntx, int nty, int zc,
                                                               const Ctl* ctl)
{
    DMG_GATE(ctl);
    constexpr int W = kPlW;
    constexpr int NH = 2 * (kPlW / 2) + kGrTY;   // F points of the halo ring per plane
    __shared__ T F[3][kGrH * kPlW];
    __shared__ T R[3][kGrRN];
    const int bid = xcd_block();   // tiles of one die are neighbours
    const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = bid / (ntx * nty);
    const int x0 = 1 + tx * kPlTX, y0 = 1 + ty * kGrTY, z0 = 1 + tz * zc;
    const int z1 = min(z0 + zc, m);   // output planes [z0, z1)
    const int tid = threadIdx.x;
    const int h = m / 2;
    const size_t NN = (size_t)(m + 1) * (m + 1), PR = (size_t)(m + 1) * (h + 1);   // plane strides: G, R layouts
    // What does not depend on the plane is worked out once per thread.
    // Staged red slot e: row b = y0-2 + e / 35, slot s = (x0-3)/2 + e % 35,
    // point a = 2 s + ((b+c) & 1) (inside iff 0 <= s < h, or s = h with a even).
    int roff[kGrRP];
    bool rok[kGrRP], rsh[kGrRP], rodd[kGrRP];
#pragma unroll
    for (int i = 0; i < kGrRP; i++) {
        const int e = tid + i * kGrThreads;
        const int b = y0 - 2 + e / kGrRS, sl = (x0 - 3) / 2 + e % kGrRS;
        rok[i] = e < kGrRN && b >= 0 && b <= m && sl >= 0 && sl <= h;
        rsh[i] = sl == h;
        rodd[i] = b & 1;
        roff[i] = b * (h + 1) + sl;
    }
    auto rload = [&](int c, int i) -> T {
        const bool ok = rok[i] && c >= 0 && c <= m && !(rsh[i] && ((rodd[i] ^ c) & 1));
        return ok ? vR[(size_t)c * PR + roff[i]] : T(0);
    };
    // the thread's pair (oa, oa+1) of row ob; ext position (oly+1, 2 opr+1)
    const int oly = tid / (kPlTX / 2), opr = tid % (kPlTX / 2);
    const int ob = y0 + oly, oa = x0 + 2 * opr;
    const bool orow = ob < m;
    const bool pok = orow && oa < m;                 // the pair holds an interior point
    const int ooff = ob * (m + 1) + oa;              // in-plane G offset of the pair
    const int obpar = (oa + ob) & 1;
    // halo F point (tid < NH): ext row hy, column hx(c); a = x0-1 + hx, b = y0-1 + hy
    int hy = 0, hj = 0;
    bool hside = false;
    if (tid < NH) {
        if (tid < 2 * (kPlW / 2)) {
            hy = tid < kPlW / 2 ? 0 : kGrH - 1;
            hj = tid % (kPlW / 2);
        } else {
            hy = 1 + tid - 2 * (kPlW / 2);
            hside = true;
        }
    }
    const int hb = y0 - 1 + hy;
    // ext column of the halo point in plane c (an F point: a + b + c odd)
    auto hcol = [&](int c) {
        const int q = (hb + c) & 1;
        return hside ? (q ? 0 : W - 1) : 2 * hj + 1 - q;
    };
    auto hin = [&](int c, int hx) {
        const int a = x0 - 1 + hx;
        return tid < NH && a > 0 && a < m && hb > 0 && hb < m && c > 0 && c < m;
    };
    auto hload = [&](int c) -> T {
        const int hx = hcol(c);
        return hin(c, hx) ? rG[(size_t)c * NN + hb * (m + 1) + x0 - 1 + hx] : T(0);
    };
    auto pload = [&](const T* p, int c) -> P2<T> {   // the thread's pair of plane c
        if (!pok || c < 1 || c >= m) return P2<T>{T(0), T(0)};
        return *reinterpret_cast<const P2<T>*>(p + (size_t)c * NN + ooff);
    };
    // F value at ext position (ly, lx) of plane c from the staged red planes
    // Rm, R0, Rq (c-1, c, c+1), same arithmetic and order as jac3_greenF
    auto fval = [&](const T* Rm, const T* R0, const T* Rq, int ly, int lx, T r) -> T {
        const int par = lx & 1;
        const int l = (ly + 1) * kGrRS + (lx >> 1) + 1;
        const T n0 = R0[l + par];       // (a+1, b, c)
        const T n1 = R0[l - 1 + par];   // (a-1, b, c)
        const T sm = n0 + n1 + R0[l + kGrRS] + R0[l - kGrRS] + Rq[l] + Rm[l];
        return (-cc * r + sm) * (T(1) / T(6));
    };
    // rings rotated at the start of every plane step c: Rm, R0, Rq hold red
    // planes c-1, c, c+1 (Rq written in the step); after the step's F values
    // are written, Fa, Fb, Fc hold those of planes c-2, c-1, c
    T *Rm = R[2], *R0 = R[0], *Rq = R[1];
    T *Fa = F[0], *Fb = F[1], *Fc = F[2];
    // prologue: red planes z0-2 (R0) and z0-1 (Rq) into LDS; red plane z0,
    // the residual pair and the halo residual of plane z0-1 into registers
    T rr[kGrRP];
#pragma unroll
    for (int i = 0; i < kGrRP; i++) {
        const int e = tid + i * kGrThreads;
        const T a0 = rload(z0 - 2, i), a1 = rload(z0 - 1, i);
        if (e < kGrRN) {
            R0[e] = a0;
            Rq[e] = a1;
        }
        rr[i] = rload(z0, i);
    }
    P2<T> rpn = pload(rG, z0 - 1);           // residual pair of the next plane to take F values of
    P2<T> rpc = P2<T>{T(0), T(0)};          // ... of plane c, then (next step) of the output plane
    T rh = hload(z0 - 1);
    P2<double> un = P2<double>{0.0, 0.0};
    for (int c = z0 - 1; c <= z1; c++) {
        {
            T* t = Rm; Rm = R0; R0 = Rq; Rq = t;
            T* f = Fa; Fa = Fb; Fb = Fc; Fc = f;
        }
#pragma unroll
        for (int i = 0; i < kGrRP; i++) {   // red plane c+1
            const int e = tid + i * kGrThreads;
            if (e < kGrRN) Rq[e] = rr[i];
        }
        const P2<T> rpo = rpc;   // the output plane's pair (c-1)
        rpc = rpn;
        const T rhc = rh;
        const P2<double> uo = un;
        if (c + 1 <= z1) {   // next plane's inputs
#pragma unroll
            for (int i = 0; i < kGrRP; i++) rr[i] = rload(c + 2, i);
            rpn = pload(rG, c + 1);
            rh = hload(c + 1);
        }
        if (FINEST && c >= z0 && c < z1 && pok) un = *reinterpret_cast<const P2<double>*>(u + (size_t)c * NN + ooff);
        __syncthreads();
        {   // the pair's F point of plane c (pF: 0 if oa, 1 if oa+1)
            const int pF = ((obpar + c) & 1) ^ 1;
            const int a = oa + pF;
            const bool in = orow && a < m && c > 0 && c < m;
            Fc[(oly + 1) * W + 2 * opr + 1 + pF] = in ? fval(Rm, R0, Rq, oly + 1, 2 * opr + 1 + pF, pF ? rpc.y : rpc.x)
                                                      : T(0);
        }
        if (tid < NH) {
            const int hx = hcol(c);
            Fc[hy * W + hx] = hin(c, hx) ? fval(Rm, R0, Rq, hy, hx, rhc) : T(0);
        }
        __syncthreads();
        const int co = c - 1;
        if (co >= z0 && orow) {
            const T* Fm = Fa;   // plane co - 1
            const T* F0 = Fb;
            const T* Fq = Fc;   // plane co + 1
            const int pco = (obpar + co) & 1;   // 1: the pair's first point is an F point
            T v[2];
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int l = (oly + 1) * W + (2 * opr + 1 + k);
                if ((pco + k) & 1) {
                    v[k] = F0[l];
                } else {
                    const T sm = F0[l + 1] + F0[l - 1] + F0[l + W] + F0[l - W] + Fq[l] + Fm[l];
                    v[k] = (-cc * (k ? rpo.y : rpo.x) + sm) * (T(1) / T(6));
                }
            }
            const size_t q = (size_t)co * NN + ooff;
            if (oa + 1 < m) {
                if (FINEST) *reinterpret_cast<P2<double>*>(u + q) = P2<double>{uo.x + (double)v[0], uo.y + (double)v[1]};
                else *reinterpret_cast<P2<T>*>(vG + q) = P2<T>{v[0], v[1]};
            } else if (oa < m) {
                if (FINEST) u[q] = uo.x + (double)v[0];
                else vG[q] = v[0];
            }
        }
        // no barrier here: the next step writes only Rq (the slot of plane
        // c-1, last read before this step's second barrier) before its first
        // barrier, and the F slot this step's outputs read only after it
    }
}

// ---- red: face centres (two odd indices), Eq. (Erprolr) and its cyclic
// permutations; corners (all even), Eq. (Erprolm).  Tiles are in R-layout
// slots: slot s of row (b, c) is the point a = 2s + ((b+c)&1).  The magenta
// grid is staged plane by plane in LDS: plane c holds the corners (c even)
// or the cube centres (c odd) at half indices (a>>1, b>>1), over the tile
// plus a one-point halo (36 x 7 values), so each magenta value is loaded
// once; face centres read their six magenta neighbours from there.
constexpr int kMsW = kRdTX + 4, kMsH = kRdTY / 2 + 3, kMsN = kMsW * kMsH;
constexpr int kMsP = (kMsN + kRdThreads - 1) / kRdThreads;   // staged magenta values per thread

template <typename T>
__global__ void __launch_bounds__(kRdThreads) k3_red_planes(int m, T c1, T c2, const T* __restrict__ rR,
                                                             const T* __restrict__ vE, const T* __restrict__ vO,
                                                             T* __restrict__ vR, int ntx, int nty, int zc,
                                                             const Ctl* ctl)
{
    DMG_GATE(ctl);
    constexpr int W = kRdW, NP = (kRdH * kRdW + kRdThreads - 1) / kRdThreads;   // F slots per thread
    constexpr int NO = kRdTY * kRdTX / kRdThreads;                              // outputs per thread
    __shared__ T F[3][kRdH * kRdW];
    __shared__ T M[3][kMsN];
    const int bid = xcd_block();   // tiles of one die are neighbours
    const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = bid / (ntx * nty);
    const int s0 = tx * kRdTX, y0 = 1 + ty * kRdTY, z0 = 1 + tz * zc;
    const int z1 = min(z0 + zc, m);
    const int tid = threadIdx.x;
    const int h = m / 2;
    const int iL = s0 - 2, jL = (y0 - 1) / 2 - 1;   // half indices of staged value 0
    const size_t PR = (size_t)(m + 1) * (h + 1);      // plane strides: R layout,
    const size_t PE = (size_t)(h + 1) * (h + 1), PO = (size_t)h * h;   // magenta corners, centres
    // What does not depend on the plane is worked out once per thread: the
    // in-plane offsets of its staged magenta values (corner planes, centre
    // planes), of its F slots (and their row parity, slot, staging base) and
    // of its output points.
    int meo[kMsP], moo[kMsP];
#pragma unroll
    for (int k = 0; k < kMsP; k++) {
        const int e = tid + k * kRdThreads;
        const int i = iL + e % kMsW, j = jL + e / kMsW;
        meo[k] = (e < kMsN && i >= 0 && i <= h && j >= 0 && j <= h) ? j * (h + 1) + i : -1;
        moo[k] = (e < kMsN && i >= 0 && i < h && j >= 0 && j < h) ? j * h + i : -1;
    }
    auto mload = [&](int c, int k) -> T {
        if (c & 1) return (moo[k] >= 0 && c >= 1 && c < m) ? vO[(size_t)(c >> 1) * PO + moo[k]] : T(0);
        return (meo[k] >= 0 && c >= 0 && c <= m) ? vE[(size_t)(c >> 1) * PE + meo[k]] : T(0);
    };
    // F slot p: row b = y0-1 + p / W, slot sl = s0-1 + p % W, point a = 2 sl + ((b+c) & 1)
    int foff[NP], fbase[NP];
    bool fodd[NP], frow[NP], fsl0[NP], fslok[NP];
#pragma unroll
    for (int k = 0; k < NP; k++) {
        const int p = tid + k * kRdThreads;
        const int b = y0 - 1 + p / W, sl = s0 - 1 + p % W;
        frow[k] = p < kRdH * kRdW && b >= 1 && b < m;
        fodd[k] = b & 1;
        fsl0[k] = sl == 0;
        fslok[k] = sl >= 0 && sl <= h - 1;
        foff[k] = b * (h + 1) + sl;
        fbase[k] = ((b >> 1) - jL) * kMsW + (sl - iL);
    }
    // is F slot k a face centre of plane c, and an interior one (a in [1, m-1])
    auto fface = [&](int c, int k) { return fodd[k] || (c & 1); };
    auto finside = [&](int c, int k) {
        const bool par = (fodd[k] ^ c) & 1;   // parity of a
        return frow[k] && c >= 1 && c < m && fslok[k] && (!fsl0[k] || par);
    };
    auto fload = [&](int c, T (&rf)[NP]) {   // F residuals of plane c (0 for corners and points off the interior)
#pragma unroll
        for (int k = 0; k < NP; k++)
            rf[k] = (fface(c, k) && finside(c, k)) ? rR[(size_t)c * PR + foff[k]] : T(0);
    };
    // output point k: row b = y0 + e / 32, slot sl = s0 + e % 32
    int ooff[NO], ol[NO];
    bool orow[NO], oodd[NO], osl0[NO], oslok[NO];
#pragma unroll
    for (int k = 0; k < NO; k++) {
        const int e = tid + k * kRdThreads;
        const int ly = e / kRdTX, ls = e % kRdTX;
        const int b = y0 + ly, sl = s0 + ls;
        orow[k] = b < m;
        oodd[k] = b & 1;
        osl0[k] = sl == 0;
        oslok[k] = sl <= h - 1;
        ooff[k] = b * (h + 1) + sl;
        ol[k] = (ly + 1) * W + (ls + 1);
    }
    // rings of LDS planes, rotated at the start of every plane step c: Mm, M0,
    // Mq hold magenta planes c-1, c, c+1 (Mq written in the step); after the
    // step's F values are written, Fa, Fb, Fc hold those of planes c-2, c-1, c
    T *Mm = M[2], *M0 = M[0], *Mq = M[1];
    T *Fa = F[0], *Fb = F[1], *Fc = F[2];
    // prologue: magenta planes z0-2 (M0) and z0-1 (Mq) into LDS, plane z0 and
    // the F residuals of plane z0-1 into registers
#pragma unroll
    for (int k = 0; k < kMsP; k++) {
        const int e = tid + k * kRdThreads;
        const T a0 = mload(z0 - 2, k), a1 = mload(z0 - 1, k);
        if (e < kMsN) {
            M0[e] = a0;
            Mq[e] = a1;
        }
    }
    T mn[kMsP];
#pragma unroll
    for (int k = 0; k < kMsP; k++) mn[k] = mload(z0, k);
    T rf[NP];
    fload(z0 - 1, rf);
    T rn[NO];
#pragma unroll
    for (int k = 0; k < NO; k++) rn[k] = T(0);
    for (int c = z0 - 1; c <= z1; c++) {
        {
            T* t = Mm; Mm = M0; M0 = Mq; Mq = t;
            T* f = Fa; Fa = Fb; Fb = Fc; Fc = f;
        }
#pragma unroll
        for (int k = 0; k < kMsP; k++) {   // magenta plane c+1
            const int e = tid + k * kRdThreads;
            if (e < kMsN) Mq[e] = mn[k];
        }
        T rfc[NP], rc[NO];
#pragma unroll
        for (int k = 0; k < NP; k++) rfc[k] = rf[k];
#pragma unroll
        for (int k = 0; k < NO; k++) rc[k] = rn[k];
        if (c + 1 <= z1) {
#pragma unroll
            for (int k = 0; k < kMsP; k++) mn[k] = mload(c + 2, k);
            fload(c + 1, rf);
        }
        if (c >= z0 && c < z1 && !(c & 1)) {   // corners of this plane need rR next iteration
#pragma unroll
            for (int k = 0; k < NO; k++)
                if (orow[k] && !oodd[k] && !osl0[k] && oslok[k]) rn[k] = rR[(size_t)c * PR + ooff[k]];
        }
        __syncthreads();
        // face centres of plane c, same arithmetic and order as jac3_redF
        // (base: the staged position of the slot's own half indices)
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const int p = tid + k * kRdThreads;
            if (p >= kRdH * kRdW || !fface(c, k)) continue;
            T v = T(0);
            if (finside(c, k)) {
                const int q = fbase[k];
                T sm;
                if (!(c & 1))        // a, b odd: centres above and below, corners around
                    sm = 2 * (Mq[q] + Mm[q]) + M0[q + kMsW + 1] + M0[q + 1] + M0[q] + M0[q + kMsW];
                else if (fodd[k])    // b odd, a even: centres at a +- 1, corners at b +- 1 above and below
                    sm = 2 * (M0[q] + M0[q - 1]) + Mq[q + kMsW] + Mm[q + kMsW] + Mm[q] + Mq[q];
                else                 // b even, a odd: centres at b +- 1, corners at a +- 1 above and below
                    sm = 2 * (M0[q] + M0[q - kMsW]) + Mq[q + 1] + Mq[q] + Mm[q] + Mm[q + 1];
                v = (-c1 * rfc[k] + sm) * T(0.125);
            }
            Fc[p] = v;
        }
        __syncthreads();
        const int co = c - 1;
        if (co >= z0) {
            const T* Fm = Fa;   // plane co-1
            const T* F0 = Fb;   // plane co
            const T* Fq = Fc;   // plane co+1
#pragma unroll
            for (int k = 0; k < NO; k++) {
                const bool par = (oodd[k] ^ co) & 1;   // parity of a
                if (!orow[k] || !oslok[k] || (osl0[k] && !par)) continue;
                const int l = ol[k];
                const bool corner = !oodd[k] && !(co & 1);   // then a is even too
                T v;
                if (!corner) {
                    v = F0[l];
                } else {
                    // corner: slots a/2 (= l) and a/2 - 1 (= l - 1); rows b +- 1 are l +- W; the
                    // twelve faces in the order of Eq. (Erprolm) as jac3_redC sums them
                    T sm = F0[l + W] + F0[l - W] + F0[l - W - 1] + F0[l + W - 1]
                         + Fq[l] + Fm[l] + Fm[l - 1] + Fq[l - 1]
                         + Fq[l + W] + Fm[l + W] + Fm[l - W] + Fq[l - W];
                    v = (-c2 * rc[k] + sm) * (T(1) / T(12));
                }
                vR[(size_t)co * PR + ooff[k]] = v;
            }
        }
        // no barrier here: before its first barrier the next step writes only
        // Mq (the slot of plane c-1, last read before this step's second
        // barrier); the F slot it then writes is the one read here
    }
}

// ------------------------------------------ residual fused with green -> red
// r = f - Lap_h(u) (Eq. Evpois, 7-point, in double, stored as T) on the
// finest green grid, its squared norm, and Eq. (Erred) onto the red grid of
// the same side, in one pass.  A workgroup marches an (x, y) tile through a
// chunk of z planes: planes of u (tile plus a two-point halo) go through a
// ring of three LDS planes, the residual of each plane (tile plus a
// one-point halo) through a second ring, and the red points of the plane
// behind read their seven residuals from LDS.  The next plane's u and f are
// loaded while the current one is processed.
// Tiles of 64 x 16 points and 512 threads: the u halo of a plane is then
// 1.25 times the tile (1.5 for 64 x 8) at the same four waves per SIMD.
constexpr int kRsTY = 16, kRsThreads = 512;
constexpr int kRsUW = kPlTX + 4, kRsUH = kRsTY + 4;   // u region
constexpr int kRsRW = kPlTX + 2, kRsRH = kRsTY + 2;   // residual region
constexpr int kRsUS = (kRsUW * kRsUH + kRsThreads - 1) / kRsThreads;
constexpr int kRsFS = (kRsRW * kRsRH + kRsThreads - 1) / kRsThreads;

template <typename T, bool M4>
__global__ void __launch_bounds__(kRsThreads) k3_resid_planes(int n, double inv_h2, const double* __restrict__ u,
                                                               const double* __restrict__ f, T* __restrict__ r0,
                                                               T* __restrict__ rR, double* __restrict__ partial,
                                                               int ntx, int nty, int zc, const Ctl* ctl)
{
    DMG_GATE(ctl);
    __shared__ double U[3][kRsUW * kRsUH];
    __shared__ T Rr[3][kRsRW * kRsRH];
    __shared__ double red[kRsThreads / 64];
    const int bid = xcd_block();   // tiles of one die are neighbours
    const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = bid / (ntx * nty);
    const int x0 = 1 + tx * kPlTX, y0 = 1 + ty * kRsTY, z0 = 1 + tz * zc;
    const int z1 = min(z0 + zc, n);
    const int tid = threadIdx.x;
    const size_t NN = (size_t)(n + 1) * (n + 1);   // plane stride of the G layout
    // Everything about a thread's points that does not depend on the plane is
    // worked out once: the (x, y) offset within a plane of each staged u and
    // f point (-1 off the grid or past the region) and, per residual point,
    // its LDS position and whether it is owned.
    int uoff[kRsUS], foff[kRsFS], rl[kRsFS];
    bool rown[kRsFS];
#pragma unroll
    for (int i = 0; i < kRsUS; i++) {
        const int p = tid + i * kRsThreads;
        const int a = x0 - 2 + p % kRsUW, b = y0 - 2 + p / kRsUW;
        uoff[i] = (p < kRsUW * kRsUH && a >= 0 && a <= n && b >= 0 && b <= n) ? b * (n + 1) + a : -1;
    }
#pragma unroll
    for (int i = 0; i < kRsFS; i++) {
        const int p = tid + i * kRsThreads;
        const int lx = p % kRsRW, ly = p / kRsRW;
        const int a = x0 - 1 + lx, b = y0 - 1 + ly;
        foff[i] = (p < kRsRW * kRsRH && a >= 1 && a < n && b >= 1 && b < n) ? b * (n + 1) + a : -1;
        rl[i] = (ly + 1) * kRsUW + (lx + 1);
        rown[i] = lx >= 1 && lx <= kPlTX && ly >= 1 && ly <= kRsTY;
    }
    auto uload = [&](int c, int i) -> double {
        return (uoff[i] >= 0 && c >= 0 && c <= n) ? u[(size_t)c * NN + uoff[i]] : 0.0;
    };
    auto fload = [&](int c, int i) -> double {
        return (foff[i] >= 0 && c >= 1 && c < n) ? __builtin_nontemporal_load(f + (size_t)c * NN + foff[i]) : 0.0;
    };
    // the thread's red output point: row ly of the tile, pair k; its column
    // alternates with the plane's parity
    const int oly = tid / (kPlTX / 2), ok = tid % (kPlTX / 2);
    const int ob = y0 + oly;
    // rings of LDS planes, rotated at the start of every step: in step c, Um,
    // U0, Uq hold u of planes c-1, c, c+1 (Uq written in the step), and after
    // its residual is written Rq, Rm, R0 hold the residual of planes c-2, c-1, c
    double *Um = U[0], *U0 = U[1], *Uq = U[2];
    T *Rm = Rr[0], *R0 = Rr[1], *Rq = Rr[2];
    // u planes z0-2 and z0-1 into LDS; registers: u of plane z0, f of plane z0-1
    {
        double a0[kRsUS], a1[kRsUS];
#pragma unroll
        for (int i = 0; i < kRsUS; i++) { a0[i] = uload(z0 - 2, i); a1[i] = uload(z0 - 1, i); }
#pragma unroll
        for (int i = 0; i < kRsUS; i++) {
            const int p = tid + i * kRsThreads;
            if (p < kRsUW * kRsUH) { Um[p] = a0[i]; U0[p] = a1[i]; }
        }
    }
    {   // as after a step z0-2: U0 holds plane z0-2, Uq plane z0-1
        double* t = Uq; Uq = U0; U0 = Um; Um = t;
    }
    // two register sets in turn, each holding the u plane and the f plane of
    // one step, so every load is issued two planes ahead of its use
    double uA[kRsUS], fA[kRsFS], uB[kRsUS], fB[kRsFS];
#pragma unroll
    for (int i = 0; i < kRsUS; i++) { uA[i] = uload(z0, i); uB[i] = uload(z0 + 1, i); }
#pragma unroll
    for (int i = 0; i < kRsFS; i++) { fA[i] = fload(z0 - 1, i); fB[i] = fload(z0, i); }
    double acc = 0;
    // plane c: u plane c+1 from the set into LDS, the residual of plane c, then
    // the red points of plane c-1; the set is refilled with planes c+3 and c+2
    auto step = [&](int c, double (&un)[kRsUS], double (&fn)[kRsFS]) {
        {   // rotate: plane c-1 <- c <- c+1, the oldest buffer takes plane c+1
            double* t = Um; Um = U0; U0 = Uq; Uq = t;
            T* r = Rm; Rm = R0; R0 = Rq; Rq = r;
        }
#pragma unroll
        for (int i = 0; i < kRsUS; i++) {
            const int p = tid + i * kRsThreads;
            if (p < kRsUW * kRsUH) Uq[p] = un[i];
        }
        double fc[kRsFS];
#pragma unroll
        for (int i = 0; i < kRsFS; i++) fc[i] = fn[i];
        if (c + 2 <= z1) {
#pragma unroll
            for (int i = 0; i < kRsUS; i++) un[i] = uload(c + 3, i);
#pragma unroll
            for (int i = 0; i < kRsFS; i++) fn[i] = fload(c + 2, i);
        }
        __syncthreads();
        const bool cin = c >= 1 && c < n, cown = c >= z0 && c < z1;
#pragma unroll
        for (int i = 0; i < kRsFS; i++) {
            const int p = tid + i * kRsThreads;
            if (p >= kRsRW * kRsRH) continue;
            T rt = T(0);
            if (cin && foff[i] >= 0) {
                const int l = rl[i];
                double lap;
                if constexpr (M4) {
                    // Eq. (Efos4): -24 centre, 2 x (6 faces), then the 12 edges
                    // (xy, yz, xz planes); inv_h2 is 1/(6h^2), fc the
                    // right-hand side combination
                    const int W = kRsUW;
                    lap = (-24 * U0[l] + 2 * (U0[l - W] + U0[l + W] + U0[l - 1] + U0[l + 1] + Uq[l] + Um[l]) +
                           U0[l + 1 + W] + U0[l - 1 + W] + U0[l - 1 - W] + U0[l + 1 - W] + Uq[l + W] + Um[l + W] +
                           Um[l - W] + Uq[l - W] + Uq[l + 1] + Uq[l - 1] + Um[l - 1] + Um[l + 1]) * inv_h2;
                } else {
                    lap = (U0[l + 1] + U0[l - 1] + U0[l + kRsUW] + U0[l - kRsUW] + Uq[l] + Um[l] - 6 * U0[l]) * inv_h2;
                }
                double r = fc[i] - lap;
                rt = (T)r;
                if (rown[i] && cown) {
                    __builtin_nontemporal_store(rt, r0 + (size_t)c * NN + foff[i]);
                    acc += r * r;
                }
            }
            R0[p] = rt;
        }
        __syncthreads();
        const int co = c - 1;
        if (co >= z0) {
            const T* Pm = Rq;   // residual plane co-1
            const T* P0 = Rm;   // plane co
            const T* Pq = R0;   // plane co+1 = c
            const int a = x0 + ((x0 + ob + co) & 1) + 2 * ok;   // the red point (a+b+co even) of pair k
            if (ob < n && a < n) {
                const int l = (oly + 1) * kRsRW + (a - x0 + 1);
                T sum = 6 * P0[l] + P0[l + 1] + P0[l - 1] + P0[l + kRsRW] + P0[l - kRsRW] + Pq[l] + Pm[l];
                rR[idxR(n, a, ob, co)] = sum * (T(1) / T(12));
            }
        }
    };
    for (int c = z0 - 1; c <= z1; c += 2) {
        step(c, uA, fA);
        if (c + 1 <= z1) step(c + 1, uB, fB);
    }
    // block sum of the squared residual, one partial per workgroup
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0;
        for (int w = 0; w < kRsThreads / 64; w++) t += red[w];
        partial[blockIdx.x] = t;
    }
}

inline void resid3_grid(int n, int& ntx, int& nty, int& zc, int& nb)
{
    ntx = (n - 1 + kPlTX - 1) / kPlTX;
    nty = (n - 1 + kRsTY - 1) / kRsTY;
    // the longest z chunk (the fewest halo planes read twice) that still
    // gives 512 workgroups, two per CU (measured at 257^3: 32 planes, 99 us,
    // against 102 for 16 and 108 for 8)
    zc = 32;
    while (zc > 4 && (long)ntx * nty * ((n - 1 + zc - 1) / zc) < 512) zc >>= 1;
    nb = ntx * nty * ((n - 1 + zc - 1) / zc);
}

// number of norm partials the fused kernel writes (0: not used at this size)
int resid3_fused_parts(int n)
{
    if (n < 128) return 0;
    int ntx, nty, zc, nb;
    resid3_grid(n, ntx, nty, zc, nb);
    return nb;
}

template <typename T>
void launch_resid3_fused(int n, const double* u, const double* f, T* r0, T* rR, double* partial, const Ctl* ctl,
                         hipStream_t s, int order)
{
    int ntx, nty, zc, nb;
    resid3_grid(n, ntx, nty, zc, nb);
    if (order == 4)
        hipLaunchKernelGGL((k3_resid_planes<T, true>), dim3(nb), dim3(kRsThreads), 0, s, n, (double)n * n / 6, u, f, r0,
                           rR, partial, ntx, nty, zc, ctl);
    else
        hipLaunchKernelGGL((k3_resid_planes<T, false>), dim3(nb), dim3(kRsThreads), 0, s, n, (double)n * n, u, f, r0,
                           rR, partial, ntx, nty, zc, ctl);
}

// The right-hand side combination of the fourth-order residual (Section
// 3.3, Eq. Efos4): g = (6 f + the six face neighbours of f) / 12 at interior
// nodes, made once per solve; reads f on boundary nodes too.
__global__ void k3_rhs4(int n, const double* __restrict__ f, double* __restrict__ g)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int b = blockIdx.y + 1, c = blockIdx.z + 1;
    if (a > n - 1) return;
    const size_t s = (size_t)n + 1, s2 = s * s, q = (size_t)c * s2 + (size_t)b * s + a;
    g[q] = (6 * f[q] + f[q + 1] + f[q + s] + f[q - 1] + f[q - s] + f[q + s2] + f[q - s2]) / 12;
}

void launch_rhs4_3d(int n, const double* f, double* g, hipStream_t s)
{
    hipLaunchKernelGGL(k3_rhs4, dim3((n - 1 + 255) / 256, n - 1, n - 1), dim3(256), 0, s, n, f, g);
}

// ---- magenta of side m, Eqs. (Emprolm), (Emprolb), in half indices (A,B,C):
// cube centres (2A+1, 2B+1, 2C+1), 0 <= A,B,C < m/2, from the blue grid (the
// green grid of side m/2), then interior corners (2A, 2B, 2C) from the eight
// new centres around them.  A workgroup marches a tile of centres (plus one
// centre of halo below in A and B) through a chunk of C planes.  Each blue
// plane is staged in LDS once (the tile's region plus one, a ring of two
// planes: centre plane C reads blue planes C and C+1); the corner plane C
// reads centre planes C-1 and C from a ring of two LDS planes.
constexpr int kMgTX = 32, kMgW = kMgTX + 1, kMgH = kPlTY + 1;
constexpr int kMgBW = kMgW + 1, kMgBH = kMgH + 1, kMgBN = kMgBW * kMgBH;   // staged blue region

template <typename T>
__global__ void __launch_bounds__(kPlThreads) k3_mag_planes(int m, T cc, const T* __restrict__ rE,
                                                             const T* __restrict__ rO, const T* __restrict__ vB,
                                                             T* __restrict__ vE, T* __restrict__ vO, int ntx, int nty,
                                                             int zc, const Ctl* ctl)
{
    DMG_GATE(ctl);
    constexpr int W = kMgW, NP = (kMgW * kMgH + kPlThreads - 1) / kPlThreads, NO = kMgTX * kPlTY / kPlThreads;
    constexpr int NB = (kMgBN + kPlThreads - 1) / kPlThreads;
    __shared__ T F[2][kMgW * kMgH];
    __shared__ T Bs[2][kMgBN];
    const int h = m / 2;
    const int bid = xcd_block();   // tiles of one die are neighbours
    const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = bid / (ntx * nty);
    const int A0 = tx * kMgTX, B0 = ty * kPlTY, C0 = tz * zc;
    const int C1 = min(C0 + zc, h);   // centre planes [C0, C1) and corner planes [C0, C1) are output
    const int tid = threadIdx.x;
    const size_t PB = (size_t)(h + 1) * (h + 1), PO = (size_t)h * h, PE = (size_t)(h + 1) * (h + 1);
    // plane-invariant per-thread data: staged blue offsets, centre slots, corner outputs
    int boff[NB];
#pragma unroll
    for (int k = 0; k < NB; k++) {
        const int e = tid + k * kPlThreads;
        const int A = A0 - 1 + e % kMgBW, B = B0 - 1 + e / kMgBW;
        boff[k] = (e < kMgBN && A >= 0 && A <= h && B >= 0 && B <= h) ? B * (h + 1) + A : -1;
    }
    auto bload = [&](int C, int k) -> T {
        return (boff[k] >= 0 && C >= 0 && C <= h) ? vB[(size_t)C * PB + boff[k]] : T(0);
    };
    int poff[NP], pq[NP];
    bool pok[NP], pown[NP];
#pragma unroll
    for (int j = 0; j < NP; j++) {
        const int p = tid + j * kPlThreads;
        const int A = A0 - 1 + p % W, B = B0 - 1 + p / W;
        pok[j] = p < kMgW * kMgH && A >= 0 && A < h && B >= 0 && B < h;
        pown[j] = pok[j] && A >= A0 && B >= B0;
        poff[j] = B * h + A;
        pq[j] = (p / W) * kMgBW + p % W;   // staged blue position of (A, B)
    }
    auto rload = [&](int C, int j) -> T { return (pok[j] && C >= 0 && C < h) ? rO[(size_t)C * PO + poff[j]] : T(0); };
    int ooff[NO], ol[NO];
    bool oin[NO];
#pragma unroll
    for (int k = 0; k < NO; k++) {
        const int e = tid + k * kPlThreads;
        const int A = A0 + e % kMgTX, B = B0 + e / kMgTX;
        oin[k] = A >= 1 && A < h && B >= 1 && B < h;
        ooff[k] = B * (h + 1) + A;
        ol[k] = (B - B0 + 1) * W + (A - A0 + 1);   // centre (A, B); (A-1) is l-1, (B-1) is l-W
    }
    // prologue: blue plane C0-1 into LDS; registers: blue plane C0, the centre
    // residuals of plane C0-1
    T *Bm = Bs[0], *Bq = Bs[1];   // in step C: blue planes C (Bm) and C+1 (Bq)
#pragma unroll
    for (int k = 0; k < NB; k++) {
        const int e = tid + k * kPlThreads;
        const T v = bload(C0 - 1, k);
        if (e < kMgBN) Bq[e] = v;
    }
    T bn[NB], rnx[NP];
#pragma unroll
    for (int k = 0; k < NB; k++) bn[k] = bload(C0, k);
#pragma unroll
    for (int j = 0; j < NP; j++) rnx[j] = rload(C0 - 1, j);
    T rn[NO];
#pragma unroll
    for (int k = 0; k < NO; k++) rn[k] = T(0);
    T *Fm = F[0], *F0 = F[1];   // in step C: centre planes C-1 (Fm) and C (F0)
    for (int C = C0 - 1; C < C1; C++) {
        {
            T* t = Bm; Bm = Bq; Bq = t;
            T* f = Fm; Fm = F0; F0 = f;
        }
#pragma unroll
        for (int k = 0; k < NB; k++) {   // blue plane C+1
            const int e = tid + k * kPlThreads;
            if (e < kMgBN) Bq[e] = bn[k];
        }
        T rr[NP], rc[NO];
#pragma unroll
        for (int j = 0; j < NP; j++) rr[j] = rnx[j];
#pragma unroll
        for (int k = 0; k < NO; k++) rc[k] = rn[k];
        if (C + 1 < C1) {
#pragma unroll
            for (int k = 0; k < NB; k++) bn[k] = bload(C + 2, k);
#pragma unroll
            for (int j = 0; j < NP; j++) rnx[j] = rload(C + 1, j);
        }
        if (C + 1 >= C0 && C + 1 < C1 && C + 1 >= 1) {   // corners of plane C+1 need rE next iteration
#pragma unroll
            for (int k = 0; k < NO; k++)
                if (oin[k]) rn[k] = rE[(size_t)(C + 1) * PE + ooff[k]];
        }
        __syncthreads();
        // centres of plane C, same arithmetic and order as jac3_magF
#pragma unroll
        for (int j = 0; j < NP; j++) {
            const int p = tid + j * kPlThreads;
            if (p >= kMgW * kMgH) continue;
            T v = T(0);
            if (pok[j] && C >= 0 && C < h) {
                const int q = pq[j], w = kMgBW;
                v = (-cc * rr[j] + Bq[q + 1 + w] + Bm[q + 1 + w] + Bq[q + 1] + Bm[q + 1] + Bq[q + w] + Bm[q + w] +
                     Bq[q] + Bm[q]) * T(0.125);
                if (pown[j] && C >= C0) vO[(size_t)C * PO + poff[j]] = v;
            }
            F0[p] = v;
        }
        __syncthreads();
        if (C >= C0 && C >= 1) {   // corner plane C from centre planes C-1 and C
#pragma unroll
            for (int k = 0; k < NO; k++) {
                if (!oin[k]) continue;
                const int l = ol[k];
                // the eight centres in the order of Eq. (Emprolb) as jac3_magC sums them
                T sm = F0[l] + Fm[l] + F0[l - W] + Fm[l - W] + F0[l - 1] + Fm[l - 1] + F0[l - W - 1] + Fm[l - W - 1];
                vE[(size_t)C * PE + ooff[k]] = (-cc * rc[k] + sm) * T(0.125);
            }
        }
        // no barrier here: before its first barrier the next step writes only
        // Bq (the slot of blue plane C, last read before this step's second
        // barrier); the centre slot it then writes is the one read here
    }
}

constexpr int kPlMinSide = 128;   // smaller levels: one thread per point
constexpr int kRdPlMinSide = 128, kGrPlMinSide = 128;   // the red and green steps

// z planes per workgroup (measured on MI355X at 257^3: 8 at side 256,
// longer chunks leave too few workgroups in flight; 4 at side 128, where 8
// leaves two waves per SIMD)
inline int pl_zchunk(int m) { return m >= 256 ? 8 : 4; }
// green steps (64 x 16 tiles): the longest chunk that still gives 512
// workgroups (measured at 257^3: 32 planes 109 us, 16 planes 110, 8 planes
// with 64 x 8 tiles 118)
inline int gr_zchunk(int m)
{
    const long tiles = (long)((m - 1 + kPlTX - 1) / kPlTX) * ((m - 1 + kGrTY - 1) / kGrTY);
    int zc = 32;
    while (zc > 4 && tiles * ((m - 1 + zc - 1) / zc) < 512) zc >>= 1;
    return zc;
}

template <typename T>
void launch_jac3(const Lev3<T>& L, const Lev3<T>& Cr, T* zero, const Ctl* ctl, hipStream_t s)
{
    int m = L.m;
    const T* vc = Cr.v ? Cr.v : zero;
    if (L.kind == 2) {
        if (m >= kPlMinSide) {
            int h = m / 2, ntx = (h + kMgTX - 1) / kMgTX, nty = (h + kPlTY - 1) / kPlTY, zc = pl_zchunk(m);
            int ntz = (h + zc - 1) / zc;
            hipLaunchKernelGGL(k3_mag_planes<T>, dim3(ntx * nty * ntz), dim3(kPlThreads), 0, s, m, L.c, L.r, L.r2, vc,
                               L.v, L.v2, ntx, nty, zc, ctl);
        } else {
            dim3 g((m / 2 + 255) / 256, m / 2, m / 2);
            hipLaunchKernelGGL(k3_jac_mag<T>, g, dim3(256), 0, s, m, L.c, L.r, L.r2, vc, L.v, L.v2, ctl);
        }
    } else if (L.kind == 1) {
        if (m >= kRdPlMinSide) {
            int ntx = (m / 2 + kRdTX - 1) / kRdTX, nty = (m - 1 + kRdTY - 1) / kRdTY, zc = pl_zchunk(m);
            int ntz = (m - 1 + zc - 1) / zc;
            hipLaunchKernelGGL(k3_red_planes<T>, dim3(ntx * nty * ntz), dim3(kRdThreads), 0, s, m, L.c, L.c2, L.r,
                               Cr.v, Cr.v2, L.v, ntx, nty, zc, ctl);
        } else {
            dim3 g((m / 2 + 255) / 256, m / 2, m / 2);
            hipLaunchKernelGGL(k3_jac_red<T>, g, dim3(256), 0, s, m, L.c, L.c2, L.r, Cr.v, Cr.v2, L.v, ctl);
        }
    } else {
        if (m >= kGrPlMinSide) {
            int ntx = (m - 1 + kPlTX - 1) / kPlTX, nty = (m - 1 + kGrTY - 1) / kGrTY, zc = gr_zchunk(m);
            int ntz = (m - 1 + zc - 1) / zc;
            hipLaunchKernelGGL((k3_green_planes<T, false>), dim3(ntx * nty * ntz), dim3(kGrThreads), 0, s, m, L.c, L.r,
                               vc, L.v, nullptr, ntx, nty, zc, ctl);
        } else {
            dim3 g((m / 2 + 1 + 255) / 256, m - 1, m - 1);
            hipLaunchKernelGGL(k3_jac_green<T>, g, dim3(256), 0, s, m, L.c, L.r, vc, L.v, ctl);
        }
    }
}

template <typename T>
void launch_jac3_finest(int n, T c, const T* r0, const T* vR, double* u, const Ctl* ctl, hipStream_t s)
{
    if (n >= kPlMinSide) {
        int ntx = (n - 1 + kPlTX - 1) / kPlTX, nty = (n - 1 + kGrTY - 1) / kGrTY, zc = gr_zchunk(n);
        int ntz = (n - 1 + zc - 1) / zc;
        hipLaunchKernelGGL((k3_green_planes<T, true>), dim3(ntx * nty * ntz), dim3(kGrThreads), 0, s, n, c, r0, vR,
                           nullptr, u, ntx, nty, zc, ctl);
        return;
    }
    dim3 g((n / 2 + 1 + 255) / 256, n - 1, n - 1);
    hipLaunchKernelGGL(k3_jac_finest<T>, g, dim3(256), 0, s, n, c, r0, vR, u, ctl);
}

// ------------------------------------------------------ level-group kernels
// One level group of side m (green m -> red m -> magenta m -> blue = green
// m/2) in one launch each way, for the sides where the per-level launches
// are too small to fill the chip (16 .. 64).  A workgroup owns the fine
// points with every index in [8t, 8t+8) of its tile t = (tx, ty, tz) and
// computes each intermediate level over the tile plus the halo the next
// step needs, in LDS; every point is computed with the arithmetic and term
// order of the per-point functions (rs3_*, jac3_*), so the values equal
// theirs bit for bit.  Owned points of every level are stored.  All global
// loads of a workgroup are issued at its start (into registers, a fixed
// number per thread), so the level steps that follow wait on LDS only.
constexpr int kGrpT = 8, kGrpThreads = 1024;
// (at side 128 the per-level kernels are faster: 4096 tiles re-read their
// halos from L2 more than the launches cost; measured on MI355X)
constexpr int kGrpMinSide = 16, kGrpMaxDown = 64, kGrpMaxUp = 64;

__device__ inline bool grp_in(int a, int m) { return a >= 1 && a <= m - 1; }
constexpr int grp_per(int n) { return (n + kGrpThreads - 1) / kGrpThreads; }

// restriction: green r (G, side m) -> red r, magenta r (E, O), blue r (G, side m/2)
template <typename T>
__global__ void __launch_bounds__(kGrpThreads) k3_down_group(int m, const T* __restrict__ rG, T* __restrict__ rR,
                                                             T* __restrict__ rE, T* __restrict__ rO,
                                                             T* __restrict__ rB, int nt, const Ctl* ctl)
{
    DMG_GATE(ctl);
    // boxes (fine indices, per dimension): green [8t-3, 8t+9], red [8t-2, 8t+8],
    // magenta [8t-1, 8t+7]; blue points 4t .. 4t+3
    constexpr int GW = kGrpT + 5, RW = kGrpT + 3, MW = kGrpT + 1, NT = kGrpThreads;
    constexpr int NG = GW * GW * GW, NR = RW * RW * RW, NM = MW * MW * MW, H = kGrpT / 2;
    __shared__ T G[NG];
    __shared__ T R[NR];
    __shared__ T M[NM];
    const int bid = xcd_block();
    const int tx = bid % nt, ty = (bid / nt) % nt, tz = bid / (nt * nt);
    const int ox = kGrpT * tx, oy = kGrpT * ty, oz = kGrpT * tz;   // first owned fine index
    const int tid = threadIdx.x;
    auto own = [&](int a, int b, int c) {
        return a >= ox && a < ox + kGrpT && b >= oy && b < oy + kGrpT && c >= oz && c < oz + kGrpT;
    };
    {
        T g[grp_per(NG)];
#pragma unroll
        for (int k = 0; k < grp_per(NG); k++) {
            const int p = tid + k * NT;
            const int a = ox - 3 + p % GW, b = oy - 3 + (p / GW) % GW, c = oz - 3 + p / (GW * GW);
            g[k] = (p < NG && a >= 0 && a <= m && b >= 0 && b <= m && c >= 0 && c <= m) ? rG[idxG(m, a, b, c)] : T(0);
        }
#pragma unroll
        for (int k = 0; k < grp_per(NG); k++)
            if (tid + k * NT < NG) G[tid + k * NT] = g[k];
    }
    __syncthreads();
    // Eq. (Erred), as rs3_g2r
#pragma unroll
    for (int kk = 0; kk < grp_per(NR); kk++) {
        const int p = tid + kk * NT;
        if (p >= NR) break;
        const int i = p % RW, j = (p / RW) % RW, k = p / (RW * RW);
        const int a = ox - 2 + i, b = oy - 2 + j, c = oz - 2 + k;
        T v = T(0);
        if (!((a + b + c) & 1) && grp_in(a, m) && grp_in(b, m) && grp_in(c, m)) {
            const int q = ((k + 1) * GW + (j + 1)) * GW + (i + 1), w = GW, w2 = GW * GW;
            v = (6 * G[q] + G[q + 1] + G[q - 1] + G[q + w] + G[q - w] + G[q + w2] + G[q - w2]) * (T(1) / T(12));
            if (own(a, b, c)) rR[idxR(m, a, b, c)] = v;
        }
        R[p] = v;
    }
    __syncthreads();
    // Eqs. (Ermagc), (Ermagm), as rs3_r2mE / rs3_r2mO
#pragma unroll
    for (int kk = 0; kk < grp_per(NM); kk++) {
        const int p = tid + kk * NT;
        if (p >= NM) break;
        const int i = p % MW, j = (p / MW) % MW, k = p / (MW * MW);
        const int a = ox - 1 + i, b = oy - 1 + j, c = oz - 1 + k;
        auto r = [&](int da, int db, int dc) { return R[((k + 1 + dc) * RW + (j + 1 + db)) * RW + (i + 1 + da)]; };
        T v = T(0);
        if (!((a | b | c) & 1) && grp_in(a, m) && grp_in(b, m) && grp_in(c, m)) {
            v = (12 * r(0, 0, 0)
                 + r(1, 1, 0) + r(1, -1, 0)
                 + r(-1, -1, 0) + r(-1, 1, 0)
                 + r(1, 0, 1) + r(1, 0, -1)
                 + r(-1, 0, -1) + r(-1, 0, 1)
                 + r(0, 1, 1) + r(0, 1, -1)
                 + r(0, -1, -1) + r(0, -1, 1)) * (T(1) / T(24));
            if (own(a, b, c)) rE[idxME(m, a, b, c)] = v;
        } else if ((a & b & c & 1) && grp_in(a, m) && grp_in(b, m) && grp_in(c, m)) {
            v = (r(1, 0, 0) + r(-1, 0, 0) + r(0, 1, 0) + r(0, -1, 0) + r(0, 0, 1) + r(0, 0, -1)) * (T(1) / T(6));
            if (own(a, b, c)) rO[idxMO(m, a, b, c)] = v;
        }
        M[p] = v;
    }
    __syncthreads();
    // Eq. (Erblu), as rs3_m2b
    const int mc = m / 2;
    if (tid < H * H * H) {
        const int p = tid;
        const int A = ox / 2 + p % H, B = oy / 2 + (p / H) % H, C = oz / 2 + p / (H * H);
        if (grp_in(A, mc) && grp_in(B, mc) && grp_in(C, mc)) {
            const int i = 2 * A - (ox - 1), j = 2 * B - (oy - 1), k = 2 * C - (oz - 1);
            auto e = [&](int da, int db, int dc) { return M[((k + dc) * MW + (j + db)) * MW + (i + da)]; };
            rB[idxG(mc, A, B, C)] = (8 * e(0, 0, 0)
                                     + e(1, 1, 1) + e(1, 1, -1)
                                     + e(1, -1, 1) + e(1, -1, -1)
                                     + e(-1, 1, 1) + e(-1, 1, -1)
                                     + e(-1, -1, 1) + e(-1, -1, -1)) * T(0.0625);
        }
    }
}

// Jacobi: magenta (Eqs. Emprolm, Emprolb) from the blue correction, red
// (Eqs. Erprolr, Erprolm) from the new magenta values, green (Eqs. Egprolg,
// Egprolr) from the new red values.  cm: magenta coefficient; c1, c2: red;
// cg: green.
template <typename T>
struct GrpUp {
    const T *rG, *rR, *rE, *rO, *vB;
    T *vG, *vR, *vE, *vO;
    T cm, c1, c2, cg;
};

template <typename T>
__global__ void __launch_bounds__(kGrpThreads) k3_up_group(int m, GrpUp<T> L, int nt, const Ctl* ctl)
{
    DMG_GATE(ctl);
    // boxes (fine indices): blue half indices [4t-3, 4t+6]; magenta centres
    // (odd) [8t-5, 8t+11], corners (even) [8t-4, 8t+10]; red [8t-3, 8t+10]
    // (corners over [8t-2, 8t+9]); green F [8t-1, 8t+8]; green C: the tile
    constexpr int BW = kGrpT / 2 + 6, OW = kGrpT / 2 + 5, EW = kGrpT / 2 + 4, RW = kGrpT + 6, FW = kGrpT + 2;
    constexpr int NT = kGrpThreads, NB = BW * BW * BW, NO = OW * OW * OW, NE = EW * EW * EW, NR = RW * RW * RW,
                  NF = FW * FW * FW, NC = kGrpT * kGrpT * kGrpT;
    __shared__ T Bv[NB];
    __shared__ T Mo[NO];
    __shared__ T Me[NE];
    __shared__ T Rv[NR];
    __shared__ T Gf[NF];
    const int bid = xcd_block();
    const int tx = bid % nt, ty = (bid / nt) % nt, tz = bid / (nt * nt);
    const int ox = kGrpT * tx, oy = kGrpT * ty, oz = kGrpT * tz;
    const int tid = threadIdx.x;
    const int mc = m / 2;
    auto own = [&](int a, int b, int c) {
        return a >= ox && a < ox + kGrpT && b >= oy && b < oy + kGrpT && c >= oz && c < oz + kGrpT;
    };
    auto inside = [&](int a, int b, int c) { return grp_in(a, m) && grp_in(b, m) && grp_in(c, m); };
    const int bx = ox / 2 - 3, by = oy / 2 - 3, bz = oz / 2 - 3;
    // point p of each step's box
    auto pO = [&](int p, int& a, int& b, int& c) {
        a = ox - 5 + 2 * (p % OW); b = oy - 5 + 2 * ((p / OW) % OW); c = oz - 5 + 2 * (p / (OW * OW));
    };
    auto pE = [&](int p, int& a, int& b, int& c) {
        a = ox - 4 + 2 * (p % EW); b = oy - 4 + 2 * ((p / EW) % EW); c = oz - 4 + 2 * (p / (EW * EW));
    };
    auto pR = [&](int p, int& a, int& b, int& c) {
        a = ox - 3 + p % RW; b = oy - 3 + (p / RW) % RW; c = oz - 3 + p / (RW * RW);
    };
    auto pF = [&](int p, int& a, int& b, int& c) {
        a = ox - 1 + p % FW; b = oy - 1 + (p / FW) % FW; c = oz - 1 + p / (FW * FW);
    };
    auto pC = [&](int p, int& a, int& b, int& c) {
        a = ox + p % kGrpT; b = oy + (p / kGrpT) % kGrpT; c = oz + p / (kGrpT * kGrpT);
    };
    auto isface = [](int a, int b, int c) { return (a & 1) + (b & 1) + (c & 1) == 2; };
    // every global input of the workgroup, loaded up front
    T lb[grp_per(NB)], lo[grp_per(NO)], le[grp_per(NE)], lr[grp_per(NR)], lf[grp_per(NF)], lc[grp_per(NC)];
#pragma unroll
    for (int k = 0; k < grp_per(NB); k++) {
        const int p = tid + k * NT;
        const int A = bx + p % BW, B = by + (p / BW) % BW, C = bz + p / (BW * BW);
        lb[k] = (p < NB && A >= 0 && A <= mc && B >= 0 && B <= mc && C >= 0 && C <= mc) ? L.vB[idxG(mc, A, B, C)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < grp_per(NO); k++) {
        const int p = tid + k * NT;
        int a, b, c;
        pO(p, a, b, c);
        lo[k] = (p < NO && inside(a, b, c)) ? L.rO[idxMO(m, a, b, c)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < grp_per(NE); k++) {
        const int p = tid + k * NT;
        int a, b, c;
        pE(p, a, b, c);
        le[k] = (p < NE && inside(a, b, c)) ? L.rE[idxME(m, a, b, c)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < grp_per(NR); k++) {   // face centres over the box, corners over the box less its border
        const int p = tid + k * NT;
        int a, b, c;
        pR(p, a, b, c);
        lr[k] = (p < NR && !((a + b + c) & 1) && inside(a, b, c)) ? L.rR[idxR(m, a, b, c)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < grp_per(NF); k++) {
        const int p = tid + k * NT;
        int a, b, c;
        pF(p, a, b, c);
        lf[k] = (p < NF && ((a + b + c) & 1) && inside(a, b, c)) ? L.rG[idxG(m, a, b, c)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < grp_per(NC); k++) {
        const int p = tid + k * NT;
        int a, b, c;
        pC(p, a, b, c);
        lc[k] = (p < NC && !((a + b + c) & 1) && inside(a, b, c)) ? L.rG[idxG(m, a, b, c)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < grp_per(NB); k++)
        if (tid + k * NT < NB) Bv[tid + k * NT] = lb[k];
    __syncthreads();
    // magenta centres, as jac3_magF
#pragma unroll
    for (int kk = 0; kk < grp_per(NO); kk++) {
        const int p = tid + kk * NT;
        if (p >= NO) break;
        int a, b, c;
        pO(p, a, b, c);
        T v = T(0);
        if (inside(a, b, c)) {
            const int q = ((((c - 1) >> 1) - bz) * BW + (((b - 1) >> 1) - by)) * BW + (((a - 1) >> 1) - bx);
            const int w = BW, w2 = BW * BW;
            v = (-L.cm * lo[kk]
                 + Bv[q + 1 + w + w2] + Bv[q + 1 + w] + Bv[q + 1 + w2] + Bv[q + 1]
                 + Bv[q + w + w2] + Bv[q + w] + Bv[q + w2] + Bv[q]) * T(0.125);
            if (own(a, b, c)) L.vO[idxMO(m, a, b, c)] = v;
        }
        Mo[p] = v;
    }
    __syncthreads();
    // magenta corners, as jac3_magC
#pragma unroll
    for (int kk = 0; kk < grp_per(NE); kk++) {
        const int p = tid + kk * NT;
        if (p >= NE) break;
        const int i = p % EW, j = (p / EW) % EW, k = p / (EW * EW);
        int a, b, c;
        pE(p, a, b, c);
        T v = T(0);
        if (inside(a, b, c)) {
            // centre (a+da, b+db, c+dc) of Mo: a+1 -> i+1, a-1 -> i
            auto o = [&](int da, int db, int dc) {
                return Mo[((k + (dc + 1) / 2) * OW + (j + (db + 1) / 2)) * OW + (i + (da + 1) / 2)];
            };
            T sm = o(1, 1, 1) + o(1, 1, -1) + o(1, -1, 1) + o(1, -1, -1) + o(-1, 1, 1) + o(-1, 1, -1) + o(-1, -1, 1) +
                   o(-1, -1, -1);
            v = (-L.cm * le[kk] + sm) * T(0.125);
            if (own(a, b, c)) L.vE[idxME(m, a, b, c)] = v;
        }
        Me[p] = v;
    }
    __syncthreads();
    // magenta value at fine (a, b, c): a corner (all even) or a centre (all odd)
    auto mE = [&](int a, int b, int c) {
        return Me[(((c - (oz - 4)) >> 1) * EW + ((b - (oy - 4)) >> 1)) * EW + ((a - (ox - 4)) >> 1)];
    };
    auto mO = [&](int a, int b, int c) {
        return Mo[(((c - (oz - 5)) >> 1) * OW + ((b - (oy - 5)) >> 1)) * OW + ((a - (ox - 5)) >> 1)];
    };
    // red face centres, as jac3_redF (other slots: 0 for now)
#pragma unroll
    for (int kk = 0; kk < grp_per(NR); kk++) {
        const int p = tid + kk * NT;
        if (p >= NR) break;
        int a, b, c;
        pR(p, a, b, c);
        T v = T(0);
        if (isface(a, b, c) && inside(a, b, c)) {
            T sm;
            if (!(c & 1))
                sm = 2 * (mO(a, b, c + 1) + mO(a, b, c - 1))
                     + mE(a + 1, b + 1, c) + mE(a + 1, b - 1, c)
                     + mE(a - 1, b - 1, c) + mE(a - 1, b + 1, c);
            else if (!(a & 1))
                sm = 2 * (mO(a + 1, b, c) + mO(a - 1, b, c))
                     + mE(a, b + 1, c + 1) + mE(a, b + 1, c - 1)
                     + mE(a, b - 1, c - 1) + mE(a, b - 1, c + 1);
            else
                sm = 2 * (mO(a, b + 1, c) + mO(a, b - 1, c))
                     + mE(a + 1, b, c + 1) + mE(a - 1, b, c + 1)
                     + mE(a - 1, b, c - 1) + mE(a + 1, b, c - 1);
            v = (-L.c1 * lr[kk] + sm) * T(0.125);
            if (own(a, b, c)) L.vR[idxR(m, a, b, c)] = v;
        }
        Rv[p] = v;
    }
    __syncthreads();
    // red corners over [8t-2, 8t+9], as jac3_redC: they read face centres
    // only, so they are written into the same array
#pragma unroll
    for (int kk = 0; kk < grp_per(NR); kk++) {
        const int p = tid + kk * NT;
        if (p >= NR) break;
        const int i = p % RW, j = (p / RW) % RW, k = p / (RW * RW);
        int a, b, c;
        pR(p, a, b, c);
        if (!((a | b | c) & 1) && i >= 1 && i < RW - 1 && j >= 1 && j < RW - 1 && k >= 1 && k < RW - 1 &&
            inside(a, b, c)) {
            auto f = [&](int da, int db, int dc) { return Rv[p + (dc * RW + db) * RW + da]; };
            T sm = f(1, 1, 0) + f(1, -1, 0) + f(-1, -1, 0) + f(-1, 1, 0)
                 + f(1, 0, 1) + f(1, 0, -1) + f(-1, 0, -1) + f(-1, 0, 1)
                 + f(0, 1, 1) + f(0, 1, -1) + f(0, -1, -1) + f(0, -1, 1);
            const T v = (-L.c2 * lr[kk] + sm) * (T(1) / T(12));
            if (own(a, b, c)) L.vR[idxR(m, a, b, c)] = v;
            Rv[p] = v;
        }
    }
    __syncthreads();
    // green F points (a+b+c odd) over [8t-1, 8t+8], as jac3_greenF
#pragma unroll
    for (int kk = 0; kk < grp_per(NF); kk++) {
        const int p = tid + kk * NT;
        if (p >= NF) break;
        const int i = p % FW, j = (p / FW) % FW, k = p / (FW * FW);
        int a, b, c;
        pF(p, a, b, c);
        T v = T(0);
        if (((a + b + c) & 1) && inside(a, b, c)) {
            const int q = ((k + 2) * RW + (j + 2)) * RW + (i + 2), w = RW, w2 = RW * RW;
            T sm = Rv[q + 1] + Rv[q - 1] + Rv[q + w] + Rv[q - w] + Rv[q + w2] + Rv[q - w2];
            v = (-L.cg * lf[kk] + sm) * (T(1) / T(6));
            if (own(a, b, c)) L.vG[idxG(m, a, b, c)] = v;
        }
        Gf[p] = v;
    }
    __syncthreads();
    // green C points of the tile, as jac3_greenC
#pragma unroll
    for (int kk = 0; kk < grp_per(NC); kk++) {
        const int p = tid + kk * NT;
        if (p >= NC) break;
        int a, b, c;
        pC(p, a, b, c);
        if (((a + b + c) & 1) || !inside(a, b, c)) continue;
        const int q = ((c - oz + 1) * FW + (b - oy + 1)) * FW + (a - ox + 1), w = FW, w2 = FW * FW;
        T sm = Gf[q + 1] + Gf[q - 1] + Gf[q + w] + Gf[q - w] + Gf[q + w2] + Gf[q - w2];
        L.vG[idxG(m, a, b, c)] = (-L.cg * lc[kk] + sm) * (T(1) / T(6));
    }
}

bool group3_ok(int m, bool up) { return m >= kGrpMinSide && m <= (up ? kGrpMaxUp : kGrpMaxDown); }

template <typename T>
void launch_down_group3(const Lev3<T>& G, const Lev3<T>& R, const Lev3<T>& M, const Lev3<T>& B, const Ctl* ctl,
                        hipStream_t s)
{
    const int nt = G.m / kGrpT;
    hipLaunchKernelGGL(k3_down_group<T>, dim3(nt * nt * nt), dim3(kGrpThreads), 0, s, G.m, G.r, R.r, M.r, M.r2, B.r,
                       nt, ctl);
}

template <typename T>
void launch_up_group3(const Lev3<T>& G, const Lev3<T>& R, const Lev3<T>& M, const Lev3<T>& B, const Ctl* ctl,
                      hipStream_t s)
{
    const int nt = G.m / kGrpT;
    GrpUp<T> L{G.r, R.r, M.r, M.r2, B.v, G.v, R.v, M.v, M.v2, M.c, R.c, R.c2, G.c};
    hipLaunchKernelGGL(k3_up_group<T>, dim3(nt * nt * nt), dim3(kGrpThreads), 0, s, G.m, L, nt, ctl);
}

// ------------------------------------------------- coarse persistent kernel
// Every level of side <= 8 (green, red and magenta of sides 8 and 4, then
// the green of side 2: at most 1585 points per kind) staged in LDS: the
// first level's residual is read once, each level step works in LDS with one
// barrier, and every level is written back at the end.
constexpr int kCoarse3Threads = 1024;
constexpr int kCoarse3Lds = 1585;

template <typename T>
__device__ inline int lev3_elems(const Lev3<T>& L)
{
    if (L.kind == 0) return (int)sizeG(L.m);
    if (L.kind == 1) return (int)sizeR(L.m);
    return (int)(sizeME(L.m) + sizeMO(L.m));
}

// the staged levels: r (magenta: corners, then centres at +sizeME) and v at
// +kCoarse3Lds; a zero correction below the coarsest level at the end
template <typename T>
struct S3 {
    T* lds;
    const int* off;
    const Coarse3<T>* a;
    __device__ T* R(int d) const { return lds + off[d]; }
    __device__ T* V(int d) const { return lds + kCoarse3Lds + off[d]; }
    __device__ T* R2(int d) const { return lds + off[d] + sizeME(a->lev[d].m); }
    __device__ T* V2(int d) const { return lds + kCoarse3Lds + off[d] + sizeME(a->lev[d].m); }
    __device__ T* Z() const { return lds + 2 * kCoarse3Lds; }
};
constexpr int kCoarse3LdsTotal = 2 * kCoarse3Lds + 64;

// offsets, zeroing and the first level's residual
template <typename T>
__device__ void coarse3_stage_in(const Coarse3<T>& a, T* lds, int* off)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) {
        int o = 0;
        for (int d = a.first; d <= a.last; d++) {
            off[d] = o;
            o += lev3_elems(a.lev[d]);
        }
        off[32] = o;
    }
    __syncthreads();
    const S3<T> S{lds, off, &a};
    for (int q = tid; q < off[32]; q += nt) {
        lds[q] = T(0);
        lds[kCoarse3Lds + q] = T(0);
    }
    if (tid < 64) S.Z()[tid] = T(0);
    __syncthreads();
    const Lev3<T>& L0 = a.lev[a.first];
    const int ne = L0.kind == 2 ? (int)sizeME(L0.m) : lev3_elems(L0);
    for (int q = tid; q < ne; q += nt) S.R(a.first)[q] = L0.r[q];
    if (L0.kind == 2)
        for (int q = tid; q < (int)sizeMO(L0.m); q += nt) S.R2(a.first)[q] = L0.r2[q];
    __syncthreads();
}

// restriction into d for d = lo+1 .. hi
template <typename T>
__device__ void coarse3_down(const Coarse3<T>& a, const S3<T>& S, int lo, int hi)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int d = lo + 1; d <= hi; d++) {
        const Lev3<T>& C = a.lev[d];
        const int m = a.lev[d - 1].m;
        const T* Fr = S.R(d - 1);
        if (C.kind == 1) {
            T* Cr = S.R(d);
            int w = m / 2 + 1;
            int tot = w * (m - 1) * (m - 1);
            for (int q = tid; q < tot; q += nt) {
                int col = q % w, b = (q / w) % (m - 1) + 1, c = q / (w * (m - 1)) + 1;
                int aa = 2 * col + ((b + c) & 1);
                if (aa >= 1 && aa < m) Cr[idxR(m, aa, b, c)] = rs3_g2r(Fr, m, aa, b, c);
            }
        } else if (C.kind == 2) {
            T* CrE = S.R(d);
            T* CrO = S.R2(d);
            int h = m / 2;
            for (int q = tid; q < h * h * h; q += nt) {
                int A = q % h, B = (q / h) % h, Cc = q / (h * h);
                CrO[idxMO(m, 2 * A + 1, 2 * B + 1, 2 * Cc + 1)] = rs3_r2mO(Fr, m, 2 * A + 1, 2 * B + 1, 2 * Cc + 1);
                if (A >= 1 && B >= 1 && Cc >= 1) CrE[idxME(m, 2 * A, 2 * B, 2 * Cc)] = rs3_r2mE(Fr, m, 2 * A, 2 * B, 2 * Cc);
            }
        } else {
            T* Cr = S.R(d);
            const T* FrO = S.R2(d - 1);
            int mc = m / 2, k = mc - 1;
            for (int q = tid; q < k * k * k; q += nt) {
                int A = q % k + 1, B = (q / k) % k + 1, Cc = q / (k * k) + 1;
                Cr[idxG(mc, A, B, Cc)] = rs3_m2b(Fr, FrO, m, A, B, Cc);
            }
        }
        __syncthreads();
    }
}

// Jacobi at d = hi down to lo (the coarsest from a zero correction).  Each
// level takes two passes with a barrier between them: its first-half-sweep
// points (magenta centres, red face centres, green F points) into LDS, then
// its second-half-sweep points summed from those stored values in the order
// of jac3_magC / jac3_redC / jac3_greenC (the same bits as recomputing them,
// with a dependent chain of 7-9 LDS reads per thread instead of 37-85).
template <typename T>
__device__ void coarse3_up(const Coarse3<T>& a, const S3<T>& S, int lo, int hi)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int d = hi; d >= lo; d--) {
        const Lev3<T>& L = a.lev[d];
        int m = L.m;
        if (L.kind == 2) {
            const T* vB = S.V(d + 1);
            const T* rE = S.R(d);
            const T* rO = S.R2(d);
            T* vE = S.V(d);
            T* vO = S.V2(d);
            int h = m / 2;
            for (int q = tid; q < h * h * h; q += nt) {
                int A = q % h, B = (q / h) % h, Cc = q / (h * h);
                int x = 2 * A + 1, y = 2 * B + 1, z = 2 * Cc + 1;
                vO[idxMO(m, x, y, z)] = jac3_magF(rO, vB, m, L.c, x, y, z);
            }
            __syncthreads();
            const int k = h - 1;   // interior corners (2A, 2B, 2C), A, B, C in [1, h-1]
            for (int q = tid; q < k * k * k; q += nt) {
                int x = 2 * (q % k + 1), y = 2 * ((q / k) % k + 1), z = 2 * (q / (k * k) + 1);
                auto o = [&](int dx, int dy, int dz) { return vO[idxMO(m, x + dx, y + dy, z + dz)]; };
                T sm = o(1, 1, 1) + o(1, 1, -1) + o(1, -1, 1) + o(1, -1, -1) + o(-1, 1, 1) + o(-1, 1, -1) +
                       o(-1, -1, 1) + o(-1, -1, -1);
                vE[idxME(m, x, y, z)] = (-L.c * rE[idxME(m, x, y, z)] + sm) * T(0.125);
            }
        } else if (L.kind == 1) {
            const T* mE = S.V(d + 1);
            const T* mO = S.V2(d + 1);
            const T* rR = S.R(d);
            T* vR = S.V(d);
            int h = m / 2;
            for (int q = tid; q < h * h * h; q += nt) {
                int A = q % h, B = (q / h) % h, Cc = q / (h * h);
                int x = 2 * A, y = 2 * B, z = 2 * Cc;
                if (Cc >= 1) vR[idxR(m, x + 1, y + 1, z)] = jac3_redF(rR, mE, mO, m, L.c, x + 1, y + 1, z);
                if (A >= 1) vR[idxR(m, x, y + 1, z + 1)] = jac3_redF(rR, mE, mO, m, L.c, x, y + 1, z + 1);
                if (B >= 1) vR[idxR(m, x + 1, y, z + 1)] = jac3_redF(rR, mE, mO, m, L.c, x + 1, y, z + 1);
            }
            __syncthreads();
            const int k = h - 1;   // interior corners
            for (int q = tid; q < k * k * k; q += nt) {
                int x = 2 * (q % k + 1), y = 2 * ((q / k) % k + 1), z = 2 * (q / (k * k) + 1);
                auto f = [&](int dx, int dy, int dz) { return vR[idxR(m, x + dx, y + dy, z + dz)]; };
                T sm = f(1, 1, 0) + f(1, -1, 0) + f(-1, -1, 0) + f(-1, 1, 0) + f(1, 0, 1) + f(1, 0, -1) +
                       f(-1, 0, -1) + f(-1, 0, 1) + f(0, 1, 1) + f(0, 1, -1) + f(0, -1, -1) + f(0, -1, 1);
                vR[idxR(m, x, y, z)] = (-L.c2 * rR[idxR(m, x, y, z)] + sm) * (T(1) / T(12));
            }
        } else {
            const T* vR = (d == a.last) ? S.Z() : S.V(d + 1);
            const T* rG = S.R(d);
            T* vG = S.V(d);
            int w = m / 2 + 1;
            int tot = w * (m - 1) * (m - 1);
            for (int q = tid; q < tot; q += nt) {
                int t = q % w, b = (q / w) % (m - 1) + 1, c = q / (w * (m - 1)) + 1;
                int aF = 2 * t + 1 - ((b + c) & 1);
                if (aF >= 1 && aF < m) vG[idxG(m, aF, b, c)] = jac3_greenF(rG, vR, m, L.c, aF, b, c);
            }
            __syncthreads();
            for (int q = tid; q < tot; q += nt) {
                int t = q % w, b = (q / w) % (m - 1) + 1, c = q / (w * (m - 1)) + 1;
                int aC = 2 * t + ((b + c) & 1);
                if (aC >= 1 && aC < m) {
                    // F neighbours off the interior are zero in LDS, as jac3_greenF returns there
                    const size_t p = idxG(m, aC, b, c), W1 = (size_t)(m + 1), W2 = W1 * W1;
                    T sm = vG[p + 1] + vG[p - 1] + vG[p + W1] + vG[p - W1] + vG[p + W2] + vG[p - W2];
                    vG[p] = (-L.c * rG[p] + sm) * (T(1) / T(6));
                }
            }
        }
        __syncthreads();
    }
}

// write back: residuals below the first level, every correction
template <typename T>
__device__ void coarse3_stage_out(const Coarse3<T>& a, const S3<T>& S)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int d = a.first; d <= a.last; d++) {
        const Lev3<T>& L = a.lev[d];
        const int n1 = L.kind == 2 ? (int)sizeME(L.m) : lev3_elems(L);
        for (int q = tid; q < n1; q += nt) {
            if (d > a.first) L.r[q] = S.R(d)[q];
            L.v[q] = S.V(d)[q];
        }
        if (L.kind == 2)
            for (int q = tid; q < (int)sizeMO(L.m); q += nt) {
                if (d > a.first) L.r2[q] = S.R2(d)[q];
                L.v2[q] = S.V2(d)[q];
            }
    }
}

template <typename T>
__global__ void __launch_bounds__(kCoarse3Threads) k3_coarse(Coarse3<T> a, const Ctl* ctl)
{
    DMG_GATE(ctl);
    __shared__ T lds[kCoarse3LdsTotal];
    __shared__ int off[33];
    coarse3_stage_in(a, lds, off);
    const S3<T> S{lds, off, &a};
    coarse3_down(a, S, a.first, a.last);
    coarse3_up(a, S, a.first, a.last);
    coarse3_stage_out(a, S);
}

// ------------------------------------------------- learned coarse correction
// The cut is the green level of side 8 (9^3 points): the first coarse level
// when the grid has a level below it.  The network's output at the red
// points (a+b+c even) fills the red level's correction, and the cut level's
// own Jacobi then runs unchanged.  Judge and state as in 2D (Ctl::net).

__device__ inline double block_sum3(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[w];
    return s;
}

// ||r - A v||^2 over the interior of a green level of side m (7-point
// Laplacian with spacing 1/m)
template <typename T>
__device__ double cut3_resid2(const T* r, const T* v, int m, double* red)
{
    double s = 0, m2 = (double)m * m;
    const int k = m - 1;
    for (int q = threadIdx.x; q < k * k * k; q += blockDim.x) {
        int a = q % k + 1, b = (q / k) % k + 1, c = q / (k * k) + 1;
        size_t o = idxG(m, a, b, c), w = (size_t)(m + 1), w2 = w * w;
        double av = ((double)v[o - 1] + (double)v[o + 1] + (double)v[o - w] + (double)v[o + w] + (double)v[o - w2] +
                     (double)v[o + w2] - 6.0 * (double)v[o]) * m2;
        double d = (double)r[o] - av;
        s += d * d;
    }
    return block_sum3(s, red);
}

// network on r_c (green 9^3, spacing H = 1/8): the red-point values of the
// estimate of A_c^{-1} r_c go to vR (R layout of side 8).  Returns ||r_c||^2.
template <typename T>
__device__ double net_cut_3d(const T* rc, T* vR, const bf16_t* __restrict__ wf, bf16_t* A, bf16_t* B, float* out0,
                             short* linq, double* red)
{
    using N = NetGeo<3>;
    net_zero(A, N::ACT);
    net_zero(B, N::ACT);
    net_fill_lin<3>(linq);
    double ss = 0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        double x = (double)rc[N::lin(q)];
        ss += x * x;
    }
    ss = block_sum3(ss, red);
    double rms = sqrt(ss / N::NIN);
    double sc = rms > 0 ? 1.0 / rms : 0.0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        int p = N::lin(q);
        A[p * kNetCh] = f2bf((float)((double)rc[p] * sc));
    }
    __syncthreads();
    const int WLY = N::WLY;
    net_conv_fwd<3, true>(A, B, nullptr, wf, linq);
    __syncthreads();
    net_conv_fwd<3, true>(B, A, nullptr, wf + WLY, linq);
    __syncthreads();
    net_conv_fwd<3, true>(A, B, nullptr, wf + 2 * WLY, linq);
    __syncthreads();
    net_conv_fwd<3, false>(B, nullptr, out0, wf + 3 * WLY, linq);
    __syncthreads();
    const double back = rms / ((N::G - 1) * (N::G - 1));
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        int x = q % N::IN + 1, y = (q / N::IN) % N::IN + 1, z = q / (N::IN * N::IN) + 1;
        if (((x + y + z) & 1) == 0) vR[idxR(N::G - 1, x, y, z)] = (T)((double)out0[q] * back);
    }
    __syncthreads();
    return ss;
}

// dynamic LDS of the learned kernel: staged levels, then (16-byte aligned)
// the two activation grids, the fp32 output, the point table and a copy of
// the red correction of side 8 (405 points)
template <typename T>
constexpr size_t coarse3_net_act_off() { return (sizeof(T) * kCoarse3LdsTotal + 15) / 16 * 16; }
template <typename T>
constexpr size_t coarse3_net_save_off()
{
    using N = NetGeo<3>;
    return (coarse3_net_act_off<T>() + 2 * sizeof(bf16_t) * N::ACT + N::TILES * 16 * sizeof(float) +
            N::LQ * sizeof(short) + 15) / 16 * 16;
}
template <typename T>
constexpr size_t coarse3_net_lds() { return coarse3_net_save_off<T>() + sizeof(T) * 405; }

template <typename T>
__global__ void __launch_bounds__(kCoarse3Threads) k3_coarse_net(Coarse3<T> a, Ctl* ctl, const bf16_t* __restrict__ wf)
{
    using N = NetGeo<3>;
    DMG_GATE(ctl);
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    bf16_t* A = reinterpret_cast<bf16_t*>(smem + coarse3_net_act_off<T>());
    bf16_t* B = A + N::ACT;
    float* out0 = reinterpret_cast<float*>(B + N::ACT);
    short* linq = reinterpret_cast<short*>(out0 + N::TILES * 16);
    T* vsave = reinterpret_cast<T*>(smem + coarse3_net_save_off<T>());
    __shared__ int off[33];
    __shared__ double red[kCoarse3Threads / 64];
    coarse3_stage_in(a, lds, off);
    const S3<T> S{lds, off, &a};
    const int cut = a.first;
    const bool has = a.lev[cut].kind == 0 && a.lev[cut].m == N::G - 1 && a.last > cut;
    const int state = has ? ctl->net : 0;
    if (state == 0) {
        coarse3_down(a, S, a.first, a.last);
        coarse3_up(a, S, a.first, a.last);
        coarse3_stage_out(a, S);
        return;
    }
    const int m = a.lev[cut].m;
    const int nR = (int)sizeR(m);   // 405 (side 8)
    double rn2 = net_cut_3d<T>(S.R(cut), S.V(cut + 1), wf, A, B, out0, linq, red);
    coarse3_up(a, S, cut, cut);
    double qn = cut3_resid2<T>(S.R(cut), S.V(cut), m, red);
    int next = state, used = 0;
    double theta = ctl->theta, qfirst = ctl->q_net;
    if (state == 1 || !(qn <= theta * theta * rn2)) {
        if (state == 1)
            for (int q = threadIdx.x; q < nR; q += blockDim.x) vsave[q] = S.V(cut + 1)[q];
        __syncthreads();
        coarse3_down(a, S, a.first, a.last);
        coarse3_up(a, S, a.first, a.last);
        double qp = cut3_resid2<T>(S.R(cut), S.V(cut), m, red);
        if (state == 1) {
            theta = rn2 > 0 ? sqrt(qp / rn2) : 0.0;
            qfirst = rn2 > 0 ? sqrt(qn / rn2) : 0.0;
            if (qn <= qp) {
                for (int q = threadIdx.x; q < nR; q += blockDim.x) S.V(cut + 1)[q] = vsave[q];
                __syncthreads();
                coarse3_up(a, S, cut, cut);
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
    coarse3_stage_out(a, S);
    if (threadIdx.x == 0) {
        ctl->net = next;
        ctl->theta = theta;
        ctl->q_net = qfirst;
        ctl->net_used += used;
        if (next == 0) ctl->net_off = 1;
    }
}

template <typename T>
void launch_coarse3(const Coarse3<T>& a, const Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(k3_coarse<T>, dim3(1), dim3(kCoarse3Threads), 0, s, a, ctl);
}

template <typename T>
void launch_coarse3_net(const Coarse3<T>& a, Ctl* ctl, const bf16_t* wf, hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k3_coarse_net<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)coarse3_net_lds<T>());
        attr = true;
    }
    hipLaunchKernelGGL(k3_coarse_net<T>, dim3(1), dim3(kCoarse3Threads), coarse3_net_lds<T>(), s, a, ctl, wf);
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
    template void launch_down_group3<T>(const Lev3<T>&, const Lev3<T>&, const Lev3<T>&, const Lev3<T>&,      \
                                        const Ctl*, hipStream_t);                                             \
    template void launch_up_group3<T>(const Lev3<T>&, const Lev3<T>&, const Lev3<T>&, const Lev3<T>&,        \
                                      const Ctl*, hipStream_t);                                               \
    template void launch_coarse3<T>(const Coarse3<T>&, const Ctl*, hipStream_t);                          \
    template void launch_coarse3_net<T>(const Coarse3<T>&, Ctl*, const bf16_t*, hipStream_t);             \
    template void launch_level_get3<T>(int, int, const T*, const T*, double*, hipStream_t);              \
    template void launch_resid3_fused<T>(int, const double*, const double*, T*, T*, double*, const Ctl*, hipStream_t, int);
DMG_INST3(double)
DMG_INST3(float)

}  // namespace dmg

// The conventional comparison V-cycle (Roberts, Sections 2.1-2.3 and 3.1-3.3)
// on the standard hierarchy of axis-aligned (cubic) grids of spacing h, 2h,
// 4h, ... down to one interior node: the finest residual, the nine-point (2D)
// or 27-point (3D) full-weighting restriction, and on the way up bilinear
// (trilinear) interpolation of the coarse correction followed by one Jacobi
// iteration (nu1 = 0, nu2 = 1) in red-black order -- the points with an odd
// index sum first, then the even ones from the new odd values -- with the
// parameter p (2D) / p_g (3D) on the residual term.  The finest step adds the
// correction to u.  It is the scheme the paper measures its diagonal grids
// against (Tables tbl:2d, tbl:3d, tbl:3dopt, rows "usual").
//
// Every level is a natural (m+1)^dim array (x fastest) of the level type T.
// The up step runs in one launch per level (tiles staged in LDS, below), so
// each level array is read and written once per step.  Sums follow the order the operators are written in (see the
// per-point functions), so FP64 results agree with the CPU reference to
// rounding of the reciprocals at most.
#include "dmg_b2d.hpp"
#include "dmg_launch.hpp"
#include "dmg_launch3.hpp"
#include "dmg_usual.hpp"

#include <algorithm>
#include <string.h>

namespace dmg {

namespace {

// ------------------------------------------------------ per-point arithmetic

// nine-point full weighting: (4 centre + 2 (E + N + W + S) + NE + NW + SW + SE) / 16
template <typename T>
__device__ inline T fw2_core(T c, T e, T n, T w, T s, T ne, T nw, T sw, T se)
{
#pragma clang fp contract(off)
    return (4 * c + 2 * (e + n + w + s) + ne + nw + sw + se) * T(0.0625);
}

// 27-point full weighting: (8 centre + 4 faces + 2 edges + corners) / 64
template <typename T>
__device__ inline T fw3_core(T c, T faces, T edges, T corners)
{
#pragma clang fp contract(off)
    return (8 * c + 4 * faces + 2 * edges + corners) * T(0.015625);
}

// one Jacobi value of Lap v = r (2 dim axis neighbours, in the order +x, -x,
// +y, -y, +z, -z in 3D; -x, -y, +x, +y in 2D, as written for each)
template <typename T>
__device__ inline T rb2_core(T c, T r, T w, T s, T e, T n)
{
#pragma clang fp contract(off)
    return (-c * r + w + s + e + n) * T(0.25);
}
template <typename T>
__device__ inline T rb3_core(T c, T r, T xp, T xm, T yp, T ym, T zp, T zm)
{
#pragma clang fp contract(off)
    return (-c * r + xp + xm + yp + ym + zp + zm) / T(6);
}
template <typename T>
__device__ inline T avg4(T a, T b, T c, T d)
{
#pragma clang fp contract(off)
    return (a + b + c + d) * T(0.25);
}

// ------------------------------------------------------------- restriction

template <typename T>
__global__ void __launch_bounds__(256) ku2_fw(int m, const T* __restrict__ r, T* __restrict__ rc,
                                              const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    const int mc = m / 2;
    const int A = blockIdx.x * blockDim.x + threadIdx.x + 1, B = blockIdx.y + 1;
    if (A > mc - 1) return;
    const size_t w = (size_t)m + 1;
    const T* p = r + (size_t)(2 * B) * w + 2 * A;
    rc[(size_t)B * (mc + 1) + A] = fw2_core(p[0], p[1], p[w], p[-1], p[-(long)w], p[w + 1], p[w - 1],
                                            p[-(long)w - 1], p[-(long)w + 1]);
}

template <typename T>
__global__ void __launch_bounds__(128) ku3_fw(int m, const T* __restrict__ r, T* __restrict__ rc,
                                              const Ctl* __restrict__ ctl)
{
#pragma clang fp contract(off)
    if (ctl->done) return;
    const int mc = m / 2;
    const int A = blockIdx.x * blockDim.x + threadIdx.x + 1, B = blockIdx.y + 1, C = blockIdx.z + 1;
    if (A > mc - 1) return;
    const long w = m + 1, w2 = w * w;
    const T* p = r + (size_t)(2 * C) * w2 + (size_t)(2 * B) * w + 2 * A;
    auto at = [&](int di, int dj, int dk) { return p[dk * w2 + dj * w + di]; };
    const T faces = at(1, 0, 0) + at(-1, 0, 0) + at(0, 1, 0) + at(0, -1, 0) + at(0, 0, 1) + at(0, 0, -1);
    const T edges = at(1, 1, 0) + at(1, -1, 0) + at(-1, 1, 0) + at(-1, -1, 0) + at(1, 0, 1) + at(1, 0, -1) +
                    at(-1, 0, 1) + at(-1, 0, -1) + at(0, 1, 1) + at(0, 1, -1) + at(0, -1, 1) + at(0, -1, -1);
    const T corners = at(1, 1, 1) + at(1, 1, -1) + at(1, -1, 1) + at(1, -1, -1) + at(-1, 1, 1) + at(-1, 1, -1) +
                      at(-1, -1, 1) + at(-1, -1, -1);
    rc[((size_t)C * (mc + 1) + B) * (mc + 1) + A] = fw3_core(p[0], faces, edges, corners);
}

// --------------------------------------------------------------- up steps
// A workgroup owns a tile of fine points.  It stages the coarse correction
// under the tile (plus a ring) in LDS, then fills one LDS array X over the
// tile plus a two-point ring: the interpolated coarse values at the even
// points (the only ones the odd colour reads), then, in the same array, the
// odd colour's new values at the odd points of the tile plus a one-point ring
// (the two sets of points are disjoint); the even colour is then computed on
// the tile from X.  The ring's odd values are recomputed by both neighbouring
// tiles instead of exchanged.

constexpr int kU2X = 64, kU2Y = 16;              // 2D tile of fine points
constexpr int kU3X = 32, kU3Y = 8, kU3Z = 4;     // 3D tile

template <typename T, bool FINEST>
__global__ void __launch_bounds__(256) ku2_up(int m, T c, const T* __restrict__ vc, const T* __restrict__ r,
                                              T* __restrict__ v, double* __restrict__ u, const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    constexpr int CX = kU2X / 2 + 3, CY = kU2Y / 2 + 3;   // coarse points under the tile and its ring
    constexpr int XX = kU2X + 4, XY = kU2Y + 4;
    constexpr int FX = XX - 2, FY = XY - 2;               // the tile and a one-point ring
    constexpr int NT = 256, NV = (CX * CY + NT - 1) / NT, NF = (FX * FY + NT - 1) / NT, NO = kU2X * kU2Y / NT;
    __shared__ T vcl[CY][CX];
    __shared__ T X[XY][XX];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kU2X, y0 = blockIdx.y * kU2Y;
    const int A0 = x0 / 2 - 1, B0 = y0 / 2 - 1, mc = m / 2, wc = mc + 1;
    const size_t w = (size_t)m + 1;
    auto interior = [&](int a, int b) { return a >= 1 && a <= m - 1 && b >= 1 && b <= m - 1; };
    // every global load of the tile first: the residuals of both colours, u,
    // the coarse values (they then arrive together instead of one loop
    // iteration at a time)
    T ro[NO];
    double uo[NO];
#pragma unroll
    for (int k = 0; k < NO; k++) {
        const int q = tid + k * NT, a = x0 + q % kU2X, b = y0 + q / kU2X;
        ro[k] = T(0);
        uo[k] = 0;
        if (interior(a, b)) {
            ro[k] = r[(size_t)b * w + a];
            if constexpr (FINEST) uo[k] = u[(size_t)b * w + a];
        }
    }
    T cv[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const int q = tid + k * NT, A = A0 + q % CX, B = B0 + q / CX;
        cv[k] = (q < CX * CY && A >= 0 && A <= mc && B >= 0 && B <= mc) ? vc[(size_t)B * wc + A] : T(0);
    }
    T rf[NF];
#pragma unroll
    for (int k = 0; k < NF; k++) {
        const int q = tid + k * NT, a = x0 - 1 + q % FX, b = y0 - 1 + q / FX;
        rf[k] = (q < FX * FY && ((a + b) & 1) && interior(a, b)) ? r[(size_t)b * w + a] : T(0);
    }
#pragma unroll
    for (int k = 0; k < NV; k++) {
        const int q = tid + k * NT;
        if (q < CX * CY) vcl[q / CX][q % CX] = cv[k];
    }
    __syncthreads();
    // interpolation at the even points: the coarse value, or the mean of the
    // four corners of the coarse cell (both indices odd); 0 off the interior
    for (int q = tid; q < XX * XY; q += NT) {
        const int lx = q % XX, ly = q / XX;
        const int a = x0 - 2 + lx, b = y0 - 2 + ly;
        if ((a + b) & 1) continue;
        T val = 0;
        if (interior(a, b)) {
            const int ca = (a >> 1) - A0, cb = (b >> 1) - B0;
            val = (a & 1) ? avg4(vcl[cb][ca], vcl[cb][ca + 1], vcl[cb + 1][ca + 1], vcl[cb + 1][ca]) : vcl[cb][ca];
        }
        X[ly][lx] = val;
    }
    __syncthreads();
    // the odd colour on the tile and a one-point ring
#pragma unroll
    for (int k = 0; k < NF; k++) {
        const int q = tid + k * NT;
        const int lx = q % FX + 1, ly = q / FX + 1;
        const int a = x0 - 2 + lx, b = y0 - 2 + ly;
        if (q >= FX * FY || !((a + b) & 1)) continue;
        X[ly][lx] = interior(a, b) ? rb2_core(c, rf[k], X[ly][lx - 1], X[ly - 1][lx], X[ly][lx + 1], X[ly + 1][lx]) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NO; k++) {
        const int q = tid + k * NT;
        const int lx = q % kU2X + 2, ly = q / kU2X + 2;
        const int a = x0 - 2 + lx, b = y0 - 2 + ly;
        if (!interior(a, b)) continue;
        const size_t o = (size_t)b * w + a;
        const T val = ((a + b) & 1) ? X[ly][lx]
                                    : rb2_core(c, ro[k], X[ly][lx - 1], X[ly - 1][lx], X[ly][lx + 1], X[ly + 1][lx]);
        if constexpr (FINEST) u[o] = uo[k] + (double)val;
        else v[o] = val;
    }
}

template <typename T, bool FINEST>
__global__ void __launch_bounds__(256) ku3_up(int m, T c, const T* __restrict__ vc, const T* __restrict__ r,
                                              T* __restrict__ v, double* __restrict__ u, const Ctl* __restrict__ ctl)
{
    if (ctl->done) return;
    constexpr int CX = kU3X / 2 + 3, CY = kU3Y / 2 + 3, CZ = kU3Z / 2 + 3;
    constexpr int XX = kU3X + 4, XY = kU3Y + 4, XZ = kU3Z + 4;
    constexpr int FX = XX - 2, FY = XY - 2, FZ = XZ - 2;
    constexpr int NT = 256, NV = (CX * CY * CZ + NT - 1) / NT, NF = (FX * FY * FZ + NT - 1) / NT;
    constexpr int NO = kU3X * kU3Y * kU3Z / NT;
    __shared__ T vcl[CZ][CY][CX];
    __shared__ T X[XZ][XY][XX];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kU3X, y0 = blockIdx.y * kU3Y, z0 = blockIdx.z * kU3Z;
    const int A0 = x0 / 2 - 1, B0 = y0 / 2 - 1, C0 = z0 / 2 - 1, mc = m / 2, wc = mc + 1;
    const size_t w = (size_t)m + 1, w2 = w * w;
    auto interior = [&](int i, int j, int k) {
        return i >= 1 && i <= m - 1 && j >= 1 && j <= m - 1 && k >= 1 && k <= m - 1;
    };
    T ro[NO];
    double uo[NO];
#pragma unroll
    for (int e = 0; e < NO; e++) {
        const int q = tid + e * NT;
        const int i = x0 + q % kU3X, j = y0 + (q / kU3X) % kU3Y, k = z0 + q / (kU3X * kU3Y);
        ro[e] = T(0);
        uo[e] = 0;
        if (interior(i, j, k)) {
            const size_t o = (size_t)k * w2 + (size_t)j * w + i;
            ro[e] = r[o];
            if constexpr (FINEST) uo[e] = u[o];
        }
    }
    T cv[NV];
#pragma unroll
    for (int e = 0; e < NV; e++) {
        const int q = tid + e * NT;
        const int A = A0 + q % CX, B = B0 + (q / CX) % CY, C = C0 + q / (CX * CY);
        cv[e] = (q < CX * CY * CZ && A >= 0 && A <= mc && B >= 0 && B <= mc && C >= 0 && C <= mc)
                    ? vc[((size_t)C * wc + B) * wc + A] : T(0);
    }
    T rf[NF];
#pragma unroll
    for (int e = 0; e < NF; e++) {
        const int q = tid + e * NT;
        const int i = x0 - 1 + q % FX, j = y0 - 1 + (q / FX) % FY, k = z0 - 1 + q / (FX * FY);
        rf[e] = (q < FX * FY * FZ && ((i + j + k) & 1) && interior(i, j, k)) ? r[(size_t)k * w2 + (size_t)j * w + i]
                                                                            : T(0);
    }
#pragma unroll
    for (int e = 0; e < NV; e++) {
        const int q = tid + e * NT;
        if (q < CX * CY * CZ) vcl[q / (CX * CY)][(q / CX) % CY][q % CX] = cv[e];
    }
    __syncthreads();
    // trilinear interpolation at the even points (all indices even: the
    // coarse value; two odd: the mean of the four coarse corners in the plane
    // of the odd axes, summed with z slowest and x fastest); 0 off the interior
    for (int q = tid; q < XX * XY * XZ; q += NT) {
        const int lx = q % XX, ly = (q / XX) % XY, lz = q / (XX * XY);
        const int i = x0 - 2 + lx, j = y0 - 2 + ly, k = z0 - 2 + lz;
        if ((i + j + k) & 1) continue;
        T val = 0;
        if (interior(i, j, k)) {
            const int ci = (i >> 1) - A0, cj = (j >> 1) - B0, ck = (k >> 1) - C0;
            if (!(i & 1) && !(j & 1) && !(k & 1)) val = vcl[ck][cj][ci];
            else if (!(k & 1)) val = avg4(vcl[ck][cj][ci], vcl[ck][cj][ci + 1], vcl[ck][cj + 1][ci], vcl[ck][cj + 1][ci + 1]);
            else if (!(j & 1)) val = avg4(vcl[ck][cj][ci], vcl[ck][cj][ci + 1], vcl[ck + 1][cj][ci], vcl[ck + 1][cj][ci + 1]);
            else val = avg4(vcl[ck][cj][ci], vcl[ck][cj + 1][ci], vcl[ck + 1][cj][ci], vcl[ck + 1][cj + 1][ci]);
        }
        X[lz][ly][lx] = val;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NF; e++) {
        const int q = tid + e * NT;
        const int lx = q % FX + 1, ly = (q / FX) % FY + 1, lz = q / (FX * FY) + 1;
        const int i = x0 - 2 + lx, j = y0 - 2 + ly, k = z0 - 2 + lz;
        if (q >= FX * FY * FZ || !((i + j + k) & 1)) continue;
        X[lz][ly][lx] = interior(i, j, k)
                            ? rb3_core(c, rf[e], X[lz][ly][lx + 1], X[lz][ly][lx - 1], X[lz][ly + 1][lx],
                                       X[lz][ly - 1][lx], X[lz + 1][ly][lx], X[lz - 1][ly][lx])
                            : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NO; e++) {
        const int q = tid + e * NT;
        const int lx = q % kU3X + 2, ly = (q / kU3X) % kU3Y + 2, lz = q / (kU3X * kU3Y) + 2;
        const int i = x0 - 2 + lx, j = y0 - 2 + ly, k = z0 - 2 + lz;
        if (!interior(i, j, k)) continue;
        const size_t o = (size_t)k * w2 + (size_t)j * w + i;
        const T val = ((i + j + k) & 1) ? X[lz][ly][lx]
                                        : rb3_core(c, ro[e], X[lz][ly][lx + 1], X[lz][ly][lx - 1], X[lz][ly + 1][lx],
                                                   X[lz][ly - 1][lx], X[lz + 1][ly][lx], X[lz - 1][ly][lx]);
        if constexpr (FINEST) u[o] = uo[e] + (double)val;
        else v[o] = val;
    }
}

// ----------------------------------------------------------------- launchers

template <typename T>
void launch_fw(int dim, int m, const T* r, T* rc, const Ctl* ctl, hipStream_t s)
{
    const int mc = m / 2;
    if (mc < 2) return;   // a coarse grid of side 1 has no interior
    if (dim == 2)
        hipLaunchKernelGGL(ku2_fw<T>, dim3((mc - 1 + 255) / 256, mc - 1), dim3(256), 0, s, m, r, rc, ctl);
    else
        hipLaunchKernelGGL(ku3_fw<T>, dim3((mc - 1 + 127) / 128, mc - 1, mc - 1), dim3(128), 0, s, m, r, rc, ctl);
}

template <typename T, bool FINEST>
void launch_up(int dim, int m, T c, const T* vc, const T* r, T* v, double* u, const Ctl* ctl, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL((ku2_up<T, FINEST>), dim3((m + kU2X) / kU2X, (m + kU2Y) / kU2Y), dim3(256), 0, s, m, c, vc, r,
                           v, u, ctl);
    else
        hipLaunchKernelGGL((ku3_up<T, FINEST>), dim3((m + kU3X) / kU3X, (m + kU3Y) / kU3Y, (m + kU3Z) / kU3Z), dim3(256),
                           0, s, m, c, vc, r, v, u, ctl);
}

// ---------------------------------------------------------------- the plan

template <typename T>
T* at(PlanU& P, size_t off) { return reinterpret_cast<T*>(P.ws + off); }

double vol(int dim, int m) { return dim == 2 ? (double)(m + 1) * (m + 1) : (double)(m + 1) * (m + 1) * (m + 1); }
double inner(int dim, int m) { return dim == 2 ? (double)(m - 1) * (m - 1) : (double)(m - 1) * (m - 1) * (m - 1); }

template <typename T>
void enq_cycle(PlanU& P, double* u, const Ctl* ctl)
{
    const int dim = P.dim, n = P.n, D = P.D;
    const double es = sizeof(T);
    hipStream_t s = P.stream;
    auto R = [&](int d) { return d == 0 ? at<T>(P, P.r0) : at<T>(P, P.r[d]); };
    for (int d = 1; d <= D; d++) {
        const int m = n >> (d - 1);
        Timed t(&P.tm, MG_K_RESTRICT, es * (inner(dim, m) + inner(dim, m / 2)));
        launch_fw<T>(dim, m, R(d - 1), R(d), ctl, s);
    }
    T* zero = at<T>(P, P.zero);
    for (int d = D; d >= 1; d--) {
        const int m = n >> d;
        Timed t(&P.tm, MG_K_JACOBI, es * (2 * inner(dim, m) + (m >= 4 ? inner(dim, m / 2) : 0)));
        launch_up<T, false>(dim, m, (T)P.c[d], d == D ? zero : at<T>(P, P.v[d + 1]), R(d), at<T>(P, P.v[d]), nullptr,
                            ctl, s);
    }
    Timed t(&P.tm, MG_K_FINEST, es * (inner(dim, n) + (n >= 4 ? inner(dim, n / 2) : 0)) + 16 * inner(dim, n));
    launch_up<T, true>(dim, n, (T)P.c[0], D >= 1 ? at<T>(P, P.v[1]) : zero, R(0), nullptr, u, ctl, s);
}

void enq_cycle_any(PlanU& P, double* u, const Ctl* ctl)
{
    if (P.prec == MG_FP64) enq_cycle<double>(P, u, ctl);
    else enq_cycle<float>(P, u, ctl);
}

void enq_residual(PlanU& P, const double* u, const double* f, const Ctl* ctl)
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

void enq_finalize(PlanU& P, int kind, Ctl* ctl, HostState* host = nullptr)
{
    Timed t(&P.tm, MG_K_NORM, 8.0 * P.nparts);
    launch_finalize(kind, at<double>(P, P.partial), P.nparts, ctl, P.stream, host);
}

// order 4: the right-hand side combination of f (Eqs. Efos2 / Efos4), once per call
const double* rhs(PlanU& P, const double* f)
{
    if (P.rorder != 4) return f;
    double* g = at<double>(P, P.g);
    if (P.dim == 2) launch_b_rhs4(P.n, f, g, P.stream);
    else launch_rhs4_3d(P.n, f, g, P.stream);
    return g;
}

}  // namespace

int planu_layout(PlanU& P, int dim, int n, int prec, double p)
{
    if (dim != 2 && dim != 3) return MG_ERR_ARG;
    const int K = ilog2(n);
    if (K < 1 || K > (dim == 2 ? 15 : 11)) return MG_ERR_SIZE;
    P.rorder = (prec & MG_ORDER4) ? 4 : 2;
    prec &= ~(MG_ORDER4 | MG_USUAL);
    if (prec != MG_FP64 && prec != MG_FP32_REFINED) return MG_ERR_ARG;
    P.dim = dim;
    P.n = n;
    P.prec = prec;
    P.p = p;
    P.D = K - 1;
    const size_t es = prec == MG_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = alignUp(off + bytes);
        return o;
    };
    P.ctl = take(sizeof(Ctl));
    P.nparts = residual_parts(dim, n);   // the residual and the norm of f use the same grid
    P.partial = take(sizeof(double) * (size_t)P.nparts);
    P.zero = take(sizeof(double) * 64);
    P.r0 = take(es * (size_t)vol(dim, n));
    if (P.rorder == 4) P.g = take(sizeof(double) * (size_t)vol(dim, n));
    const double h = 1.0 / n;
    for (int d = 0; d <= P.D; d++) {
        const double sh = (double)(1 << d) * h;   // sigma * h
        P.c[d] = p * sh * sh;
        if (d >= 1) {
            P.r[d] = take(es * (size_t)vol(dim, n >> d));
            P.v[d] = take(es * (size_t)vol(dim, n >> d));
        }
    }
    P.total = off;
    return MG_OK;
}

int planu_setup(PlanU& P, void* ws, size_t ws_bytes, hipStream_t stream)
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
    // boundary entries of every level stay 0
    return hip_status(hipMemsetAsync(P.ws, 0, P.total, P.stream));
}

void planu_destroy(PlanU& P)
{
    P.tm.destroy();
    if (P.live) (void)hipStreamSynchronize(P.stream);
    if (P.hctl) (void)hipHostFree(P.hctl);
    if (P.hstate) (void)hipHostFree(P.hstate);
}

int planu_vcycle(PlanU& P, double* u, const double* f, double* relres)
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

int planu_solve(PlanU& P, double* u, const double* f, double rtol, int max_cycles, int* cycles_out, double* rel_res_out,
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
    // as the 3D plan: iteration it+1 is queued before the host reads what
    // iteration it decided (later launches of a finished solve return at once)
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

int planu_level_get(PlanU& P, int depth, int which, double* dst)
{
    if (depth < 0 || depth > P.D || (which != 0 && which != 1) || (which == 1 && depth == 0)) return MG_ERR_ARG;
    const int m = P.n >> depth;
    const size_t off = which == 0 ? (depth == 0 ? P.r0 : P.r[depth]) : P.v[depth];
    if (P.dim == 2) {
        if (P.prec == MG_FP64) launch_b_level_get<double>(0, m, at<double>(P, off), dst, P.stream);
        else launch_b_level_get<float>(0, m, at<float>(P, off), dst, P.stream);
    } else {
        if (P.prec == MG_FP64) launch_level_get3<double>(0, m, at<double>(P, off), nullptr, dst, P.stream);
        else launch_level_get3<float>(0, m, at<float>(P, off), nullptr, dst, P.stream);
    }
    return last_launch();
}

}  // namespace dmg

// 3D level descriptors, per-point stencils and launchers of libdmg
// (Roberts, Section 3: green cubic -> red FCC -> magenta BCC -> blue cubic).
// Indices are in units of the group's green stride sigma, as the paper
// indexes a whole group with the subscripts of its finest grid (Section 3.1).
#pragma once
#include "dmg_common.hpp"

namespace dmg {

template <typename T>
struct Lev3 {
    int m = 0;
    int kind = 0;           // 0 green (G layout), 1 red (R layout), 2 magenta (E + O arrays)
    T* r = nullptr;         // green/red residual, or magenta corners
    T* v = nullptr;
    T* r2 = nullptr;        // magenta cube centres
    T* v2 = nullptr;
    T c = 0, c2 = 0;        // Jacobi coefficients (red: c = 2 p_r1 (sh)^2, c2 = 4 p_r2 (sh)^2)
};

template <typename T>
struct Coarse3 {
    int first, last;
    Lev3<T> lev[32];
    T* zero;
};

// ------------------------------------------------------------ restriction

// Eq. (Erred): green (G, side m) -> red at (a,b,c), a+b+c even.
template <typename T>
__device__ inline T rs3_g2r(const T* __restrict__ r, int m, int a, int b, int c)
{
    size_t q = idxG(m, a, b, c), w = (size_t)(m + 1), w2 = w * w;
    return (6 * r[q] + r[q + 1] + r[q - 1] + r[q + w] + r[q - w] + r[q + w2] + r[q - w2]) * (T(1) / T(12));
}

// Eq. (Ermagc): red (R, side m) -> magenta corner (a,b,c all even).
template <typename T>
__device__ inline T rs3_r2mE(const T* __restrict__ r, int m, int a, int b, int c)
{
    return (12 * r[idxR(m, a, b, c)]
            + r[idxR(m, a + 1, b + 1, c)] + r[idxR(m, a + 1, b - 1, c)]
            + r[idxR(m, a - 1, b - 1, c)] + r[idxR(m, a - 1, b + 1, c)]
            + r[idxR(m, a + 1, b, c + 1)] + r[idxR(m, a + 1, b, c - 1)]
            + r[idxR(m, a - 1, b, c - 1)] + r[idxR(m, a - 1, b, c + 1)]
            + r[idxR(m, a, b + 1, c + 1)] + r[idxR(m, a, b + 1, c - 1)]
            + r[idxR(m, a, b - 1, c - 1)] + r[idxR(m, a, b - 1, c + 1)]) * (T(1) / T(24));
}

// Eq. (Ermagm): red -> magenta cube centre (a,b,c all odd), no centre term.
template <typename T>
__device__ inline T rs3_r2mO(const T* __restrict__ r, int m, int a, int b, int c)
{
    return (r[idxR(m, a + 1, b, c)] + r[idxR(m, a - 1, b, c)] + r[idxR(m, a, b + 1, c)]
            + r[idxR(m, a, b - 1, c)] + r[idxR(m, a, b, c + 1)] + r[idxR(m, a, b, c - 1)]) * (T(1) / T(6));
}

// Eq. (Erblu): magenta (E, O of side m) -> blue = green of side m/2 at (A,B,C).
template <typename T>
__device__ inline T rs3_m2b(const T* __restrict__ rE, const T* __restrict__ rO, int m, int A, int B, int C)
{
    int a = 2 * A, b = 2 * B, c = 2 * C;
    return (8 * rE[idxME(m, a, b, c)]
            + rO[idxMO(m, a + 1, b + 1, c + 1)] + rO[idxMO(m, a + 1, b + 1, c - 1)]
            + rO[idxMO(m, a + 1, b - 1, c + 1)] + rO[idxMO(m, a + 1, b - 1, c - 1)]
            + rO[idxMO(m, a - 1, b + 1, c + 1)] + rO[idxMO(m, a - 1, b + 1, c - 1)]
            + rO[idxMO(m, a - 1, b - 1, c + 1)] + rO[idxMO(m, a - 1, b - 1, c - 1)]) * T(0.0625);
}

// ----------------------------------------------------------------- Jacobi

// Eq. (Emprolm): magenta cube centre (a,b,c odd) from the blue grid vB
// (G layout, side m/2).
template <typename T>
__device__ inline T jac3_magF(const T* __restrict__ rO, const T* __restrict__ vB, int m, T cc, int a, int b, int c)
{
    int mc = m / 2;
    int i0 = (a - 1) >> 1, j0 = (b - 1) >> 1, k0 = (c - 1) >> 1;
    size_t w = (size_t)(mc + 1), w2 = w * w;
    size_t q = idxG(mc, i0, j0, k0);  // (i0, j0, k0)
    return (-cc * rO[idxMO(m, a, b, c)]
            + vB[q + 1 + w + w2] + vB[q + 1 + w] + vB[q + 1 + w2] + vB[q + 1]
            + vB[q + w + w2] + vB[q + w] + vB[q + w2] + vB[q]) * T(0.125);
}

// Eq. (Emprolb): magenta corner (a,b,c even, interior) from its eight new
// cube-centre neighbours.
template <typename T>
__device__ inline T jac3_magC(const T* __restrict__ rE, const T* __restrict__ rO, const T* __restrict__ vB, int m,
                              T cc, int a, int b, int c)
{
    T s = jac3_magF(rO, vB, m, cc, a + 1, b + 1, c + 1) + jac3_magF(rO, vB, m, cc, a + 1, b + 1, c - 1)
        + jac3_magF(rO, vB, m, cc, a + 1, b - 1, c + 1) + jac3_magF(rO, vB, m, cc, a + 1, b - 1, c - 1)
        + jac3_magF(rO, vB, m, cc, a - 1, b + 1, c + 1) + jac3_magF(rO, vB, m, cc, a - 1, b + 1, c - 1)
        + jac3_magF(rO, vB, m, cc, a - 1, b - 1, c + 1) + jac3_magF(rO, vB, m, cc, a - 1, b - 1, c - 1);
    return (-cc * rE[idxME(m, a, b, c)] + s) * T(0.125);
}

// Eq. (Erprolr) and its cyclic permutations: red face centre (two indices
// odd, interior) from the magenta grid of the same side: the two cube
// centres along the even axis (weight 2) and the four corners in the plane
// normal to it.
template <typename T>
__device__ inline T jac3_redF(const T* __restrict__ rR, const T* __restrict__ vE, const T* __restrict__ vO, int m,
                              T cc, int a, int b, int c)
{
    T s;
    if (!(c & 1))
        s = 2 * (vO[idxMO(m, a, b, c + 1)] + vO[idxMO(m, a, b, c - 1)])
            + vE[idxME(m, a + 1, b + 1, c)] + vE[idxME(m, a + 1, b - 1, c)]
            + vE[idxME(m, a - 1, b - 1, c)] + vE[idxME(m, a - 1, b + 1, c)];
    else if (!(a & 1))
        s = 2 * (vO[idxMO(m, a + 1, b, c)] + vO[idxMO(m, a - 1, b, c)])
            + vE[idxME(m, a, b + 1, c + 1)] + vE[idxME(m, a, b + 1, c - 1)]
            + vE[idxME(m, a, b - 1, c - 1)] + vE[idxME(m, a, b - 1, c + 1)];
    else
        s = 2 * (vO[idxMO(m, a, b + 1, c)] + vO[idxMO(m, a, b - 1, c)])
            + vE[idxME(m, a + 1, b, c + 1)] + vE[idxME(m, a - 1, b, c + 1)]
            + vE[idxME(m, a - 1, b, c - 1)] + vE[idxME(m, a + 1, b, c - 1)];
    return (-cc * rR[idxR(m, a, b, c)] + s) * T(0.125);
}

// Eq. (Erprolm): red corner (all even, interior) from its twelve new face-centre neighbours.
template <typename T>
__device__ __forceinline__ T jac3_redC(const T* __restrict__ rR, const T* __restrict__ vE, const T* __restrict__ vO, int m,
                              T c1, T c2, int a, int b, int c)
{
    T s = jac3_redF(rR, vE, vO, m, c1, a + 1, b + 1, c) + jac3_redF(rR, vE, vO, m, c1, a + 1, b - 1, c)
        + jac3_redF(rR, vE, vO, m, c1, a - 1, b - 1, c) + jac3_redF(rR, vE, vO, m, c1, a - 1, b + 1, c)
        + jac3_redF(rR, vE, vO, m, c1, a + 1, b, c + 1) + jac3_redF(rR, vE, vO, m, c1, a + 1, b, c - 1)
        + jac3_redF(rR, vE, vO, m, c1, a - 1, b, c - 1) + jac3_redF(rR, vE, vO, m, c1, a - 1, b, c + 1)
        + jac3_redF(rR, vE, vO, m, c1, a, b + 1, c + 1) + jac3_redF(rR, vE, vO, m, c1, a, b + 1, c - 1)
        + jac3_redF(rR, vE, vO, m, c1, a, b - 1, c - 1) + jac3_redF(rR, vE, vO, m, c1, a, b - 1, c + 1);
    return (-c2 * rR[idxR(m, a, b, c)] + s) * (T(1) / T(12));
}

// Eq. (Egprolg): green point with a+b+c odd from the red grid vR (same side).
template <typename T>
__device__ inline T jac3_greenF(const T* __restrict__ rG, const T* __restrict__ vR, int m, T cc, int a, int b, int c)
{
    if (a <= 0 || a >= m || b <= 0 || b >= m || c <= 0 || c >= m) return T(0);
    T s = vR[idxR(m, a + 1, b, c)] + vR[idxR(m, a - 1, b, c)] + vR[idxR(m, a, b + 1, c)]
        + vR[idxR(m, a, b - 1, c)] + vR[idxR(m, a, b, c + 1)] + vR[idxR(m, a, b, c - 1)];
    return (-cc * rG[idxG(m, a, b, c)] + s) * (T(1) / T(6));
}

// Eq. (Egprolr): red point (a+b+c even, interior) from its six new neighbours.
template <typename T>
__device__ inline T jac3_greenC(const T* __restrict__ rG, const T* __restrict__ vR, int m, T cc, int a, int b, int c)
{
    T s = jac3_greenF(rG, vR, m, cc, a + 1, b, c) + jac3_greenF(rG, vR, m, cc, a - 1, b, c)
        + jac3_greenF(rG, vR, m, cc, a, b + 1, c) + jac3_greenF(rG, vR, m, cc, a, b - 1, c)
        + jac3_greenF(rG, vR, m, cc, a, b, c + 1) + jac3_greenF(rG, vR, m, cc, a, b, c - 1);
    return (-cc * rG[idxG(m, a, b, c)] + s) * (T(1) / T(6));
}

// -------------------------------------------------------------- launchers
template <typename T>
void launch_rs3(const Lev3<T>& fine, const Lev3<T>& coarse, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_jac3(const Lev3<T>& L, const Lev3<T>& coarser, T* zero, const Ctl* ctl, hipStream_t s);
template <typename T>
void launch_jac3_finest(int n, T c, const T* r0, const T* vR, double* u, const Ctl* ctl, hipStream_t s);
// one level group (green G -> red R -> magenta M -> blue B, side 16 .. 64)
// in one launch each way: the three restrictions from G's residual, or the
// three Jacobi steps from B's correction
bool group3_ok(int m, bool up);
template <typename T>
void launch_down_group3(const Lev3<T>& G, const Lev3<T>& R, const Lev3<T>& M, const Lev3<T>& B, const Ctl* ctl,
                        hipStream_t s);
template <typename T>
void launch_up_group3(const Lev3<T>& G, const Lev3<T>& R, const Lev3<T>& M, const Lev3<T>& B, const Ctl* ctl,
                      hipStream_t s);
template <typename T>
void launch_coarse3(const Coarse3<T>& a, const Ctl* ctl, hipStream_t s);
// the coarse kernel with the learned correction at the green level of side 8 (wf: packed forward weights)
template <typename T>
void launch_coarse3_net(const Coarse3<T>& a, Ctl* ctl, const unsigned short* wf, hipStream_t s);
template <typename T>
void launch_level_get3(int kind, int m, const T* src, const T* src2, double* dst, hipStream_t s);
// residual of the finest green grid fused with Eq. (Erred) onto the red grid of
// the same side (n >= 128); writes resid3_fused_parts(n) norm partials
int resid3_fused_parts(int n);
// (order 4: f is the right-hand side combination of Eq. Efos4 and the
// operator the 19-point one)
template <typename T>
void launch_resid3_fused(int n, const double* u, const double* f, T* r0, T* rR, double* partial, const Ctl* ctl,
                         hipStream_t s, int order = 2);
// g = the right-hand side combination of the fourth-order residual (Eq. Efos4)
void launch_rhs4_3d(int n, const double* f, double* g, hipStream_t s);

}  // namespace dmg

// Shared definitions of libdmg: level layouts in HBM, the solve control
// block and the per-point stencils of the diagonally oriented multigrid
// (Roberts, Sections 2 and 3).  Every kernel variant (one level per launch,
// several coarse levels per persistent launch, batched) calls the same
// point functions, so they compute bit-identical values.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dmg {

// ---------------------------------------------------------------- layouts
//
// 2D level of side m (m = n / sigma, indices a = x/sigma, b = y/sigma):
//   axis grid      -> A layout: (m+1) x (m+1), natural, x fastest.
//   diagonal grid  -> D layout: the points with (a+b) even, compacted
//                     along x: row b holds a = (b&1), (b&1)+2, ...;
//                     element (a,b) at b*(m/2+1) + (a>>1).
// 3D level of side m:
//   green grid     -> G layout: (m+1)^3 natural.
//   red grid       -> R layout: points with (a+b+c) even, compacted along
//                     x: element (a,b,c) at (c*(m+1) + b)*(m/2+1) + (a>>1).
//   magenta grid   -> two arrays: corners E (all indices even) as a
//                     (m/2+1)^3 natural array of (a/2,b/2,c/2), and cube
//                     centres O (all odd) as an (m/2)^3 natural array of
//                     ((a-1)/2, (b-1)/2, (c-1)/2).
// Boundary entries are stored and hold 0 (zero Dirichlet correction), so
// the stencils need no boundary tests except where a point's neighbour
// may lie outside the level's own array.

__host__ __device__ inline size_t idxA(int m, int a, int b) { return (size_t)b * (m + 1) + a; }
__host__ __device__ inline size_t idxD(int m, int a, int b) { return (size_t)b * (m / 2 + 1) + (a >> 1); }
__host__ __device__ inline size_t idxG(int m, int a, int b, int c)
{
    return ((size_t)c * (m + 1) + b) * (m + 1) + a;
}
__host__ __device__ inline size_t idxR(int m, int a, int b, int c)
{
    return ((size_t)c * (m + 1) + b) * (m / 2 + 1) + (a >> 1);
}
__host__ __device__ inline size_t idxME(int m, int a, int b, int c)
{
    int h = m / 2;
    return ((size_t)(c >> 1) * (h + 1) + (b >> 1)) * (h + 1) + (a >> 1);
}
__host__ __device__ inline size_t idxMO(int m, int a, int b, int c)
{
    int h = m / 2;
    return ((size_t)(c >> 1) * h + (b >> 1)) * h + (a >> 1);
}

__host__ __device__ inline size_t sizeA(int m) { return (size_t)(m + 1) * (m + 1); }
__host__ __device__ inline size_t sizeD(int m) { return (size_t)(m + 1) * (m / 2 + 1); }
__host__ __device__ inline size_t sizeG(int m) { return (size_t)(m + 1) * (m + 1) * (m + 1); }
__host__ __device__ inline size_t sizeR(int m) { return (size_t)(m + 1) * (m + 1) * (m / 2 + 1); }
__host__ __device__ inline size_t sizeME(int m) { return (size_t)(m / 2 + 1) * (m / 2 + 1) * (m / 2 + 1); }
__host__ __device__ inline size_t sizeMO(int m) { return (size_t)(m / 2) * (m / 2) * (m / 2); }

// ---------------------------------------------------------- control block
// Lives at the start of the workspace.  The convergence decision of the
// outer iteration (Section 1) is taken on the device, so a solve can
// enqueue cycles without a host round trip: every kernel of a cycle returns
// at once when `done` is set.
constexpr int kMaxCycles = 1000;

struct Ctl {
    int done;        // 1: stop; every later kernel of the solve returns at once
    int status;      // MG_* code of the decision
    int cycles;      // cycles run when done was set
    int grow;        // consecutive cycles with a growing residual
    int mode;        // 0: single cycle (never sets done); 1: solve
    int max_cycles;
    int k;           // residual evaluations done so far
    int net;         // learned coarse correction: 0 off, 1 first (judged) cycle, 2 on
    double rtol;
    double fnorm;    // ||f||_2 over interior nodes
    double rr0, prev;
    double last;     // relative residual of the latest evaluation
    double theta;    // the plain sub-cycle's cut-level residual reduction on the first cycle
    double q_net;    // the network's cut-level residual reduction on the first cycle
    int net_used;    // cycles whose coarse correction came from the network
    int net_off;     // 1 once the judge switched the network off
    double hist[kMaxCycles + 1];
};
// leading fields copied back to the host after a solve
constexpr size_t kCtlHead = offsetof(Ctl, hist);

// what a solve loop needs after each residual evaluation, written by the
// finalize kernel into pinned host memory
struct HostState {
    int done;
    int k;         // evaluations done
    double last;
};

constexpr size_t kAlign = 256;
__host__ __device__ inline size_t alignUp(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------ 2D stencils
// Argument order of every sum follows the paper's printed equations.

// The 2D point functions below serve the levels of side < 512 (one thread
// per point, the coarse kernel, the fused mid-level kernels), so their
// offsets fit in 32 bits.  Their arithmetic lives in three cores on loaded
// operands, compiled without fused multiply-add contraction: every caller
// (global or LDS operands, any kernel) then rounds each product and sum the
// same way, as the equations are written.

// Eqs. (Erest2r), (Erest2b): (4 r_c + four neighbours) / 8, summed in order
template <typename T>
__device__ inline T rs2_core(T c, T n0, T n1, T n2, T n3)
{
#pragma clang fp contract(off)
    return (4 * c + n0 + n1 + n2 + n3) * T(0.125);
}
// Eq. (Eajacr): (-cc r + four coarse values) / 4, accumulated in order
template <typename T>
__device__ inline T jac2_chain(T cc, T r, T n0, T n1, T n2, T n3)
{
#pragma clang fp contract(off)
    return (-cc * r + n0 + n1 + n2 + n3) * T(0.25);
}
// Eq. (Eajacb) and the axis-grid steps: the four neighbours summed first
template <typename T>
__device__ inline T jac2_sum(T cc, T r, T n0, T n1, T n2, T n3)
{
#pragma clang fp contract(off)
    T s = n0 + n1 + n2 + n3;
    return (-cc * r + s) * T(0.25);
}

// Eq. (Erest2r): axis grid (A, side m) -> diagonal grid (D, side m) at (a,b), a+b even.
template <typename T>
__device__ inline T rs2_a2d(const T* __restrict__ rA, int m, int a, int b)
{
    const int w = m + 1, c = b * w + a;
    return rs2_core(rA[c], rA[c - 1], rA[c - w], rA[c + 1], rA[c + w]);
}

// Eq. (Erest2b): diagonal grid (D, side m) -> axis grid of side m/2 at (2A, 2B).
template <typename T>
__device__ inline T rs2_d2a(const T* __restrict__ rD, int m, int A, int B)
{
    const int w = m / 2 + 1;
    const int c = 2 * B * w + A;         // row b = 2B (even), column a>>1 = A
    const int lo = c - w, hi = c + w;    // rows b-1, b+1 (odd): columns (a-1)>>1 = A-1 and (a+1)>>1 = A
    return rs2_core(rD[c], rD[lo - 1], rD[lo], rD[hi], rD[hi - 1]);
}

// Eq. (Eajacr): Jacobi value at a diagonal-grid point (a,b), a and b odd,
// from the axis grid vA2 of side m/2 (its coarser level).
template <typename T>
__device__ inline T jac2_diagF(const T* __restrict__ rD, const T* __restrict__ vA2, int m, T cc, int a, int b)
{
    const int w = m / 2 + 1;             // row length of vA2 (side m/2) and of the D layout
    const int q = ((b - 1) >> 1) * w + ((a - 1) >> 1);
    // v_{i-1,j-1} + v_{i+1,j-1} + v_{i+1,j+1} + v_{i-1,j+1}
    return jac2_chain(cc, rD[b * w + (a >> 1)], vA2[q], vA2[q + 1], vA2[q + w + 1], vA2[q + w]);
}

// Eq. (Eajacb): diagonal-grid point (a,b), a and b even, interior, from the
// new values at its four diagonal neighbours (recomputed here).
template <typename T>
__device__ inline T jac2_diagC(const T* __restrict__ rD, const T* __restrict__ vA2, int m, T cc, int a, int b)
{
    return jac2_sum(cc, rD[b * (m / 2 + 1) + (a >> 1)], jac2_diagF(rD, vA2, m, cc, a - 1, b - 1),
                    jac2_diagF(rD, vA2, m, cc, a + 1, b - 1), jac2_diagF(rD, vA2, m, cc, a + 1, b + 1),
                    jac2_diagF(rD, vA2, m, cc, a - 1, b + 1));
}

// Eq. (Eajacb) from stored new values: vD already holds the level's F
// points (a and b odd); same operands and order as jac2_diagC.
template <typename T>
__device__ inline T jac2_diagC_stored(const T* __restrict__ rD, const T* vD, int m, T cc, int a, int b)
{
    const int w = m / 2 + 1, c = b * w + (a >> 1);   // (a-1)>>1 = (a>>1) - 1 and (a+1)>>1 = a>>1 on odd rows
    return jac2_sum(cc, rD[c], vD[c - w - 1], vD[c - w], vD[c + w], vD[c + w - 1]);
}

// Axis-grid analogue ("similarly for a green grid", Section 2.4): point
// (a,b) with a+b odd from the diagonal grid vD of the same side.
template <typename T>
__device__ inline T jac2_axisF(const T* __restrict__ rA, const T* __restrict__ vD, int m, T cc, int a, int b)
{
    if (a <= 0 || a >= m || b <= 0 || b >= m) return T(0);
    const int w = m / 2 + 1, rowb = b * w;
    // neighbours (a-1,b), (a,b-1), (a+1,b), (a,b+1): all have an even index sum
    return jac2_sum(cc, rA[b * (m + 1) + a], vD[rowb + ((a - 1) >> 1)], vD[rowb - w + (a >> 1)],
                    vD[rowb + ((a + 1) >> 1)], vD[rowb + w + (a >> 1)]);
}

// Point (a,b) with a+b even, interior, from the new values at its four axis
// neighbours.
template <typename T>
__device__ inline T jac2_axisC(const T* __restrict__ rA, const T* __restrict__ vD, int m, T cc, int a, int b)
{
    return jac2_sum(cc, rA[b * (m + 1) + a], jac2_axisF(rA, vD, m, cc, a - 1, b), jac2_axisF(rA, vD, m, cc, a, b - 1),
                    jac2_axisF(rA, vD, m, cc, a + 1, b), jac2_axisF(rA, vD, m, cc, a, b + 1));
}

// The same from stored new values: vA already holds the level's F points
// (a+b odd; the boundary entries hold 0, as jac2_axisF returns there).
template <typename T>
__device__ inline T jac2_axisC_stored(const T* __restrict__ rA, const T* vA, int m, T cc, int a, int b)
{
    const int w = m + 1, c = b * w + a;
    return jac2_sum(cc, rA[c], vA[c - 1], vA[c - w], vA[c + 1], vA[c + w]);
}

}  // namespace dmg

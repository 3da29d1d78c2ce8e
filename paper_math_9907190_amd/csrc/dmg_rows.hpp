// Shared launch geometry of the row-marching kernels.
#pragma once
#include "dmg_common.hpp"

namespace dmg {

constexpr int kMaxRows = 32;         // longest strip a wave marches through
constexpr int kChunk = 2;            // default depth: rows whose loads are issued together
constexpr int kTargetWaves = 4096;   // ~16 waves per CU on 256 CUs
constexpr int kWavesPerBlock = 4;
constexpr int kRowBlock = 64 * kWavesPerBlock;
constexpr int kPairsPerWave = 62;    // lanes 1..62 write; lanes 0 and 63 are halo
constexpr int kColsPerWave = 63;     // one-sided halo (lane 0 only)
constexpr int kXcds = 8;             // MI355X: 8 accelerator dies, one L2 each

// Blocks are dispatched to the XCDs round-robin (block b runs on XCD b % 8).
// Renumber them so that each XCD gets a contiguous range of logical blocks
// (a bijection of [0, gridDim.x)): neighbouring tiles then run on the same
// die, so the halo they share stays in one L2.
__device__ inline int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = b % kXcds;
    return x * per + (x < rem ? x : rem) + b / kXcds;
}

// consecutive waves march neighbouring column bands of the same strip.  The
// id is the same in every lane of a wave, which the compiler cannot see from
// threadIdx.x; reading it from the first lane makes it (and the strip, band
// and row indices derived from it) scalar, so the per-row range checks of a
// march are scalar compares and branches instead of vector compares and
// execution-mask updates.
__device__ inline int rows_wave_id(int nwaves)
{
    (void)nwaves;
    return __builtin_amdgcn_readfirstlane(xcd_block() * kWavesPerBlock + (int)(threadIdx.x >> 6));
}

// Two adjacent elements (columns 2t, 2t+1 of a row) moved as one access.
// Rows of odd length leave every other pair 8-byte (not 16-byte) aligned;
// gfx950 global loads and stores only need dword alignment.
template <typename T>
struct alignas(sizeof(T)) P2 {
    T x, y;
};

// Neighbour-lane reads as DPP moves across the whole wave (wave_shr:1 and
// wave_shl:1 of the GFX9 DPP controls): lane i takes lane i-1's value
// (lane_up) or lane i+1's (lane_down), and lane 0, resp. lane 63, reads 0
// (bound_ctrl).  One VALU move instead of an LDS permute: no LDS round trip
// in the dependent chains of the row kernels.  The kernels that use them
// never take a value at lane 0 or 63 that came from beyond the wave (their
// halo lanes).
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ inline float lane_dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ inline double lane_dpp(double x)
{
    return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true));
}
template <typename T>
__device__ inline T lane_up(T x) { return lane_dpp<kDppWaveShr1>(x); }
template <typename T>
__device__ inline T lane_down(T x) { return lane_dpp<kDppWaveShl1>(x); }

// Sum over the block (fixed order: wave shuffle tree, then waves in order).
__device__ inline double rows_block_sum(double x)
{
    __shared__ double red[kWavesPerBlock];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kWavesPerBlock; i++) s += red[i];
    return s;
}

// Double-buffered march over rows jbeg, jbeg+CH, ... <= jlast: the loads of
// the next CH rows are in flight while the current CH rows are computed.
template <int CH, typename Ck, typename Load, typename Proc>
__device__ inline void rows_march(int jbeg, int jlast, Load&& load, Proc&& proc)
{
    Ck A, B;
    int jb = jbeg;
    load(jb, A);
    while (true) {
        load(jb + CH, B);
        proc(jb, A);
        jb += CH;
        if (jb > jlast) break;
        load(jb + CH, A);
        proc(jb, B);
        jb += CH;
        if (jb > jlast) break;
    }
}

// f(Int<0>{}), ..., f(Int<N-1>{}): a row loop whose index is a compile-time
// constant in the body, so that per-row choices (a row's parity) fold away
template <int I>
struct Int {
    static constexpr int value = I;
};
template <int I, int N, typename F>
__device__ inline void static_for(F&& f)
{
    if constexpr (I < N) {
        f(Int<I>{});
        static_for<I + 1, N>(f);
    }
}

// rows_march<1> over jbeg (even), jbeg+1, ... <= jlast with the row's parity
// as a compile-time argument (Int<0> or Int<1>) of load and proc: even and
// odd rows keep buffers of their own, so that what one parity never loads
// folds away.
template <typename Ck, typename Load, typename Proc>
__device__ inline void rows_march_parity(int jbeg, int jlast, Load&& load, Proc&& proc)
{
    Ck E, O;
    int jj = jbeg;
    load(Int<0>{}, jj, E);
    while (true) {
        load(Int<1>{}, jj + 1, O);
        proc(Int<0>{}, jj, E);
        if (++jj > jlast) break;
        load(Int<0>{}, jj + 1, E);
        proc(Int<1>{}, jj, O);
        if (++jj > jlast) break;
    }
}

// Global-memory views.  Pointers that reach a kernel through an item table
// in memory are generic addresses, which the compiler can only access with
// FLAT instructions; those count against both the vector-memory and the LDS
// counters and may complete out of order, so every wait for one load is a
// wait for all of them (vmcnt(0) lgkmcnt(0)), and a row kernel's loads of
// the next rows are never in flight during the current row's arithmetic.
// Accesses through gmem() pointers are global loads and stores: they count
// in order and a wait covers only the load it needs.
#define DMG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline DMG_GLOBAL T* gmem(T* p)
{
    return (DMG_GLOBAL T*)p;
}
// a pair as one vector access (element-aligned, like P2)
template <typename T>
__device__ inline P2<T> ld_pair(const DMG_GLOBAL T* p)
{
    typedef T V __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    const V v = *(const DMG_GLOBAL V*)p;
    return P2<T>{v.x, v.y};
}
template <typename T>
__device__ inline void st_pair(DMG_GLOBAL T* p, T x, T y)
{
    typedef T V __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    const V v = {x, y};
    *(DMG_GLOBAL V*)p = v;
}

// Streaming pair accesses for arrays that are not reused before the cache
// would evict them anyway (f, and r0 between the residual and the finest
// Jacobi): non-temporal hints keep them from displacing u and the level
// arrays the next kernels read.
template <typename T>
__device__ inline P2<T> ld_pair_nt(const T* p)
{
    typedef T V __attribute__((ext_vector_type(2)));
    V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    return P2<T>{v.x, v.y};
}
template <typename T>
__device__ inline void st_pair_nt(T* p, T x, T y)
{
    typedef T V __attribute__((ext_vector_type(2)));
    V v = {x, y};
    __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}
template <typename T>
__device__ inline P2<T> ld_pair_nt(const DMG_GLOBAL T* p)
{
    typedef T V __attribute__((ext_vector_type(2)));
    V v = __builtin_nontemporal_load((const DMG_GLOBAL V*)p);
    return P2<T>{v.x, v.y};
}
template <typename T>
__device__ inline void st_pair_nt(DMG_GLOBAL T* p, T x, T y)
{
    typedef T V __attribute__((ext_vector_type(2)));
    V v = {x, y};
    __builtin_nontemporal_store(v, (DMG_GLOBAL V*)p);
}

}  // namespace dmg

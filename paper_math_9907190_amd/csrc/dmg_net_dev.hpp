// Device side of the learned coarse correction: four convolutions of 3x3
// (2D) or 3x3x3 (3D) taps with 16 channels, bf16 operands with fp32
// accumulation on gfx950's 16x16x32 bf16 matrix cores, one workgroup per
// sample.
//
// A sample is a grid of G^dim points (G = 17 in 2D, 9 in 3D) whose boundary
// is the zero Dirichlet padding.  Activations live in LDS as bf16
// [point][16 channels]; only interior points are ever written, so the
// boundary stays zero.  The interior points are numbered 0..NIN-1 (x
// fastest) and processed in tiles of 16; a tile's 16 points are the columns
// of one 16x16 matrix product per pair of taps (k = 32: the 16 channels of
// tap 2s, then those of tap 2s+1; an odd last tap pairs with zero weights):
//
//   forward      Y^T[co][pt]  += W_t^T[co][ci] * X^T[ci][pt + off_t]
//   input grad   dX^T[ci][pt] += W_t[ci][co]   * dY^T[co][pt - off_t]
//   weight grad  dW_t[ci][co] += X[pt + off_t][ci]^T * dY[pt][co]  (k = points, 32 at a time)
//
// Operand layout of one 64-lane product (lane l, g = l/16, c = l%16):
// A[c][8g+j], B[8g+j][c] for j = 0..7 and D[4g+j][c] for j = 0..3.  In the
// forward and input-gradient products a lane therefore reads eight
// consecutive channels of one point (16 bytes) of tap 2s (g < 2) or 2s+1
// (g >= 2), and the weights are pre-packed per lane: the forward form holds
// W[t][ci][c], the input-gradient form W[t][c][co], with t and ci (co) from
// 8g+j as above.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmg {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

constexpr int kNetCh = 16;
constexpr int kNetLayers = 4;
constexpr int kNetThreads = 256;
constexpr int kNetCut = 6;   // aligned level replaced from below by the network

template <int DIM>
struct NetGeo {
    static constexpr int G = DIM == 2 ? 17 : 9;
    static constexpr int T = DIM == 2 ? 9 : 27;
    static constexpr int IN = G - 2;
    static constexpr int PTS = DIM == 2 ? G * G : G * G * G;
    static constexpr int NIN = DIM == 2 ? IN * IN : IN * IN * IN;
    static constexpr int TILES = (NIN + 15) / 16;
    static constexpr int LQ = (NIN + 31) / 32 * 32;                // point list length (k-chunks of 32)
    static constexpr int TP = (T + 1) / 2;                         // tap pairs per layer
    static constexpr int NW = kNetLayers * T * kNetCh * kNetCh;   // logical weights [layer][tap][ci][co]
    static constexpr int GLY = T * kNetCh * kNetCh;                // logical weights per layer
    static constexpr int WLY = TP * 64 * 8;                        // packed bf16 per layer and operand form
    static constexpr int PACK = kNetLayers * WLY;                  // packed bf16 per operand form (odd T: padded)
    static constexpr int ACT = PTS * kNetCh;                       // bf16 per activation grid
    __host__ __device__ static constexpr int off(int t)
    {
        return (t % 3 - 1) + G * ((t / 3) % 3 - 1) + (DIM == 3 ? G * G * (t / 9 - 1) : 0);
    }
    // interior ordinal -> linear grid index
    __host__ __device__ static int lin(int q)
    {
        int x = q % IN + 1, r = q / IN;
        if (DIM == 2) return (r + 1) * G + x;
        return ((r / IN + 1) * G + (r % IN + 1)) * G + x;
    }
};

// round to nearest even; NaN stays NaN
__host__ __device__ inline bf16_t f2bf(float x)
{
    union { float f; uint32_t u; } v;
    v.f = x;
    if ((v.u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((v.u >> 16) | 0x40u);
    v.u += 0x7fffu + ((v.u >> 16) & 1u);
    return (bf16_t)(v.u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t b)
{
    union { float f; uint32_t u; } v;
    v.u = (uint32_t)b << 16;
    return v.f;
}

__device__ inline bf16x8 ld8(const bf16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// linq[q] for q < LQ: linear index of interior point q; the padding entries
// repeat the last interior point (their products are computed and discarded).
template <int DIM>
__device__ inline void net_fill_lin(short* linq)
{
    using N = NetGeo<DIM>;
    for (int q = threadIdx.x; q < N::LQ; q += blockDim.x) linq[q] = (short)N::lin(q < N::NIN ? q : N::NIN - 1);
}

__device__ inline void net_zero(bf16_t* p, int count)
{
    uint4* q = reinterpret_cast<uint4*>(p);
    for (int i = threadIdx.x; i < count / 8; i += blockDim.x) q[i] = make_uint4(0, 0, 0, 0);
}

// the tap whose channels lane group g (= lane / 16) holds in pair s; the
// padded second half of an odd last pair reads the first tap again (its
// weights are zero)
template <int DIM>
__device__ inline int net_tap(int s, int g)
{
    const int t = 2 * s + (g >> 1);
    return t < NetGeo<DIM>::T ? t : t - 1;
}

// One forward layer.  X, Y: LDS activations; wl: this layer's packed forward
// weights (global).  RELU for the hidden layers; out0 (LDS, fp32, by
// interior ordinal) receives channel 0 of the last layer.
template <int DIM, bool RELU>
__device__ void net_conv_fwd(const bf16_t* __restrict__ X, bf16_t* __restrict__ Y, float* __restrict__ out0,
                             const bf16_t* __restrict__ wl, const short* __restrict__ linq)
{
    using N = NetGeo<DIM>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    bf16x8 w[N::TP];
#pragma unroll
    for (int s = 0; s < N::TP; s++) w[s] = ld8(wl + (s * 64 + lane) * 8);
    for (int tile = wave; tile < N::TILES; tile += nwave) {
        const int q = tile * 16 + c;
        const int p = linq[q];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < N::TP; s++)
            acc = mfma32(w[s], ld8(X + (p + N::off(net_tap<DIM>(s, g))) * kNetCh + 8 * (g & 1)), acc);
        if (q < N::NIN) {
            if (out0 && g == 0) out0[q] = acc[0];
            if (Y) {
                s16x4 o;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    float v = acc[j];
                    if (RELU) v = v > 0.f ? v : 0.f;
                    o[j] = (short)f2bf(v);
                }
                *reinterpret_cast<s16x4*>(Y + p * kNetCh + 4 * g) = o;
            }
        }
    }
}

// Gradient with respect to this layer's input, masked by the ReLU that
// produced it (X > 0): dX = sum_t W_t dY(. - off_t).
template <int DIM>
__device__ void net_conv_bwd_data(const bf16_t* __restrict__ dY, const bf16_t* __restrict__ X, bf16_t* __restrict__ dX,
                                  const bf16_t* __restrict__ wl, const short* __restrict__ linq)
{
    using N = NetGeo<DIM>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    bf16x8 w[N::TP];
#pragma unroll
    for (int s = 0; s < N::TP; s++) w[s] = ld8(wl + (s * 64 + lane) * 8);
    for (int tile = wave; tile < N::TILES; tile += nwave) {
        const int q = tile * 16 + c;
        const int p = linq[q];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < N::TP; s++)
            acc = mfma32(w[s], ld8(dY + (p - N::off(net_tap<DIM>(s, g))) * kNetCh + 8 * (g & 1)), acc);
        if (q < N::NIN) {
            const s16x4 x = *reinterpret_cast<const s16x4*>(X + p * kNetCh + 4 * g);
            s16x4 o;
#pragma unroll
            for (int j = 0; j < 4; j++) o[j] = (short)(((bf16_t)x[j] != 0 && ((bf16_t)x[j] & 0x8000u) == 0) ? f2bf(acc[j]) : 0);
            *reinterpret_cast<s16x4*>(dX + p * kNetCh + 4 * g) = o;
        }
    }
}

// Weight gradient of this layer for one sample, written as fp32
// [tap][ci][co] to gw (global).  Taps are spread over the waves; the
// contraction runs over the interior points in chunks of 16.
template <int DIM>
__device__ void net_conv_bwd_weight(const bf16_t* __restrict__ X, const bf16_t* __restrict__ dY, float* __restrict__ gw,
                                    const short* __restrict__ linq)
{
    using N = NetGeo<DIM>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    for (int t = wave; t < N::T; t += nwave) {
        const int o = N::off(t);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int ch = 0; ch < N::LQ / 32; ch++) {
            s16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int q = ch * 32 + 8 * g + j;
                const int p = linq[q];
                a[j] = (short)X[(p + o) * kNetCh + c];
                b[j] = q < N::NIN ? (short)dY[p * kNetCh + c] : (short)0;
            }
            acc = mfma32(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) gw[(t * kNetCh + 4 * g + j) * kNetCh + c] = acc[j];
    }
}

// Weight packing: logical index (layer, tap, ci, co) -> position in the
// forward form and in the input-gradient form (T taps per layer, paired:
// tap t is k-half t & 1 of pair t / 2).
__host__ __device__ inline int net_pack_fwd(int T, int layer, int tap, int ci, int co)
{
    const int k = (tap & 1) * kNetCh + ci;
    return ((layer * ((T + 1) / 2) + (tap >> 1)) * 64 + (k >> 3) * 16 + co) * 8 + (k & 7);
}
__host__ __device__ inline int net_pack_bwd(int T, int layer, int tap, int ci, int co)
{
    const int k = (tap & 1) * kNetCh + co;
    return ((layer * ((T + 1) / 2) + (tap >> 1)) * 64 + (k >> 3) * 16 + ci) * 8 + (k & 7);
}

}  // namespace dmg

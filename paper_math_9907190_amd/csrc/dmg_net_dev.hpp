// Device side of the learned coarse correction: four convolutions of 3x3
// (2D) or 3x3x3 (3D) taps with 16 channels, bf16 operands with fp32
// accumulation on the 16x16x16 bf16 matrix cores, one workgroup per sample.
//
// A sample is a grid of G^dim points (G = 17 in 2D, 9 in 3D) whose boundary
// is the zero Dirichlet padding.  Activations live in LDS as bf16
// [point][16 channels]; only interior points are ever written, so the
// boundary stays zero.  The interior points are numbered 0..NIN-1 (x
// fastest) and processed in tiles of 16; a tile's 16 points are the columns
// of one 16x16 matrix product per tap:
//
//   forward      Y^T[co][pt]  += W_t^T[co][ci] * X^T[ci][pt + off_t]
//   input grad   dX^T[ci][pt] += W_t[ci][co]   * dY^T[co][pt - off_t]
//   weight grad  dW_t[ci][co] += X[pt + off_t][ci]^T * dY[pt][co]  (k = points)
//
// Operand layout of one 64-lane product (lane l, g = l/16, c = l%16):
// A[c][4g+j], B[4g+j][c], D[4g+j][c] for j = 0..3.  So in the forward and
// input-gradient products a lane reads and writes four consecutive channels
// of one point (8 bytes), and the weights are pre-packed per lane: the
// forward form holds W[t][4g+j][c], the input-gradient form W[t][c][4g+j].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
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
    static constexpr int NW = kNetLayers * T * kNetCh * kNetCh;   // logical weights [layer][tap][ci][co]
    static constexpr int PACK = kNetLayers * T * 64 * 4;           // packed bf16 per operand form (= NW)
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

__device__ inline bf16x4 ld4(const bf16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// linq[q] for q < TILES*16: linear index of interior point q; the padding
// entries of the last tile repeat the last interior point (its products are
// computed and discarded).
template <int DIM>
__device__ inline void net_fill_lin(short* linq)
{
    using N = NetGeo<DIM>;
    for (int q = threadIdx.x; q < N::TILES * 16; q += blockDim.x) linq[q] = (short)N::lin(q < N::NIN ? q : N::NIN - 1);
}

__device__ inline void net_zero(bf16_t* p, int count)
{
    uint4* q = reinterpret_cast<uint4*>(p);
    for (int i = threadIdx.x; i < count / 8; i += blockDim.x) q[i] = make_uint4(0, 0, 0, 0);
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
    bf16x4 w[N::T];
#pragma unroll
    for (int t = 0; t < N::T; t++) w[t] = ld4(wl + (t * 64 + lane) * 4);
    for (int tile = wave; tile < N::TILES; tile += nwave) {
        const int q = tile * 16 + c;
        const int p = linq[q];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < N::T; t++) acc = mfma16(w[t], ld4(X + (p + N::off(t)) * kNetCh + 4 * g), acc);
        if (q < N::NIN) {
            if (out0 && g == 0) out0[q] = acc[0];
            if (Y) {
                bf16x4 o;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    float v = acc[j];
                    if (RELU) v = v > 0.f ? v : 0.f;
                    o[j] = (short)f2bf(v);
                }
                *reinterpret_cast<bf16x4*>(Y + p * kNetCh + 4 * g) = o;
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
    bf16x4 w[N::T];
#pragma unroll
    for (int t = 0; t < N::T; t++) w[t] = ld4(wl + (t * 64 + lane) * 4);
    for (int tile = wave; tile < N::TILES; tile += nwave) {
        const int q = tile * 16 + c;
        const int p = linq[q];
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < N::T; t++) acc = mfma16(w[t], ld4(dY + (p - N::off(t)) * kNetCh + 4 * g), acc);
        if (q < N::NIN) {
            bf16x4 x = ld4(X + p * kNetCh + 4 * g);
            bf16x4 o;
#pragma unroll
            for (int j = 0; j < 4; j++) o[j] = (short)(((bf16_t)x[j] != 0 && ((bf16_t)x[j] & 0x8000u) == 0) ? f2bf(acc[j]) : 0);
            *reinterpret_cast<bf16x4*>(dX + p * kNetCh + 4 * g) = o;
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
        for (int ch = 0; ch < N::TILES; ch++) {
            bf16x4 a, b;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int q = ch * 16 + 4 * g + j;
                const int p = linq[q];
                a[j] = (short)X[(p + o) * kNetCh + c];
                b[j] = q < N::NIN ? (short)dY[p * kNetCh + c] : (short)0;
            }
            acc = mfma16(a, b, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) gw[(t * kNetCh + 4 * g + j) * kNetCh + c] = acc[j];
    }
}

// Weight packing: logical index (layer, tap, ci, co) -> position in the
// forward form and in the input-gradient form.
__host__ __device__ inline int net_pack_fwd(int lt, int ci, int co) { return (lt * 64 + (ci >> 2) * 16 + co) * 4 + (ci & 3); }
__host__ __device__ inline int net_pack_bwd(int lt, int ci, int co) { return (lt * 64 + (co >> 2) * 16 + ci) * 4 + (co & 3); }

}  // namespace dmg

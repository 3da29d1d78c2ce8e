// Training and stand-alone inference of the learned coarse correction: the
// network of dmg_net_dev.hpp trained with mean-squared error and Adam
// (Kingma and Ba) on (residual, error) pairs of the cut level, all on the
// GPU.  FP32 master weights and Adam moments; bf16 copies of the weights in
// the two packed operand forms feed the matrix cores.
//
// Normalisation of a pair (r, e): s = rms of r over the interior points;
// the network sees r / s and is trained towards e / (s H^2), where H = 1/(G-1)
// is the cut level's spacing, so an inference output y stands for y s H^2.
#include "dmg_host.hpp"
#include "dmg_net.hpp"
#include "dmg_net_dev.hpp"

#include <math.h>
#include <new>
#include <string.h>
#include <vector>

namespace dmg {

template <int DIM>
constexpr double net_h2() { return 1.0 / ((NetGeo<DIM>::G - 1) * (NetGeo<DIM>::G - 1)); }

template <int DIM>
constexpr size_t net_lds_train()
{
    using N = NetGeo<DIM>;
    return 6 * (size_t)N::ACT * sizeof(bf16_t) + 2 * N::TILES * 16 * sizeof(float) + N::LQ * sizeof(short);
}
template <int DIM>
constexpr size_t net_lds_fwd()
{
    using N = NetGeo<DIM>;
    return 2 * (size_t)N::ACT * sizeof(bf16_t) + N::TILES * 16 * sizeof(float) + N::LQ * sizeof(short);
}

__device__ inline double block_sum(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[w];
    __syncthreads();
    return s;
}

// sample index of block b in a step: an affine permutation of 0..npairs-1
__device__ inline int net_sample(int b, long long base, long long pa, long long pb, int npairs)
{
    if (npairs <= 0) return b;
    return (int)((pa * (base + b) + pb) % npairs);
}

// Loads sample s into X0 (channel 0) and tgt; returns the input scale.
// judge: tgt receives the (scaled) input itself in single precision.
template <int DIM>
__device__ double net_load(const double* __restrict__ in, const double* __restrict__ target, int normalize,
                           bf16_t* X0, float* tgt, double* red, bool judge = false)
{
    using N = NetGeo<DIM>;
    double ss = 0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        double v = in[N::lin(q)];
        ss += v * v;
    }
    double rms = sqrt(block_sum(ss, red) / N::NIN);
    double sc = normalize ? (rms > 0 ? 1.0 / rms : 0.0) : 1.0;
    double st = normalize ? (rms > 0 ? 1.0 / (rms * net_h2<DIM>()) : 0.0) : 1.0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        int p = N::lin(q);
        X0[p * kNetCh] = f2bf((float)(in[p] * sc));
        if (tgt) tgt[q] = judge ? (float)(in[p] * sc) : (float)(target[p] * st);
    }
    return normalize ? rms * net_h2<DIM>() : 1.0;
}

// The cut-level objective (judge != 0): the network output y at the grid's
// even points (the points the cut level shares with the level below) goes
// through the cut level's own red-black Jacobi step for Lap v = x, with its
// over-relaxation parameter pj on the residual (odd points first, then the
// even ones from the new odd values; the network's units, spacing 1), and
// the loss is the sum of rho^2 over the interior, rho = x - L v: the
// squared reduction of the cut level's residual by the correction the coarse
// kernel would use.  Its gradient with respect to y (the step is linear) goes
// into d0 at the even points; d1 serves as scratch and is cleared again.
template <int DIM>
__device__ double net_judge_loss(const float* out0, const float* xin, const short* linq, float pj, float inv_cnt,
                                 bf16_t* d0, bf16_t* d1, int grad, double* red)
{
    using N = NetGeo<DIM>;
    constexpr int G = N::G, PTS = N::PTS;
    constexpr float d2 = 2.f * DIM, inv2d = 1.f / (2.f * DIM);
    float* Y = reinterpret_cast<float*>(d1);
    float* X = Y + PTS;
    float* V = X + PTS;
    float* R = V + PTS;
    float* F = R + PTS;
    auto par = [](int p) { return (p % G + (p / G) % G + p / (G * G)) & 1; };
    auto nsum = [](const float* a, int p) {
        float s = a[p - 1] + a[p + 1] + a[p - G] + a[p + G];
        if (DIM == 3) s += a[p - G * G] + a[p + G * G];
        return s;
    };
    for (int p = threadIdx.x; p < 5 * PTS; p += blockDim.x) Y[p] = 0.f;
    __syncthreads();
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        const int p = linq[q];
        X[p] = xin[q];
        if (!par(p)) Y[p] = out0[q];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        const int p = linq[q];
        if (par(p)) V[p] = (nsum(Y, p) - pj * X[p]) * inv2d;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        const int p = linq[q];
        if (!par(p)) V[p] = (nsum(V, p) - pj * X[p]) * inv2d;
    }
    __syncthreads();
    double l = 0;
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
        const int p = linq[q];
        const float rho = X[p] - (nsum(V, p) - d2 * V[p]);
        R[p] = rho;
        l += (double)rho * rho;
    }
    l = block_sum(l, red);
    if (grad) {
        // d loss / d v = -L (2 rho inv_cnt) (L symmetric, zero boundary), into Y
        for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
            const int p = linq[q];
            Y[p] = -(nsum(R, p) - d2 * R[p]) * 2.f * inv_cnt;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {   // odd points feed their even neighbours
            const int p = linq[q];
            if (par(p)) F[p] = Y[p] + nsum(Y, p) * inv2d;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {   // onto the network's even outputs
            const int p = linq[q];
            if (!par(p)) d0[p * kNetCh] = f2bf(nsum(F, p) * inv2d);
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < 5 * PTS; p += blockDim.x) Y[p] = 0.f;   // d1 is zero again
    __syncthreads();
    return l;
}

// One sample per workgroup: forward, loss, and (grad != 0) the weight
// gradient of this sample into gpart[block][NW].  judge: the cut-level
// objective above instead of the mean squared error (e is not read).
template <int DIM>
__global__ void __launch_bounds__(kNetThreads) kn_train(const double* __restrict__ r, const double* __restrict__ e,
                                                        long long base, long long pa, long long pb, int npairs,
                                                        int normalize, float inv_cnt, const bf16_t* __restrict__ wf,
                                                        const bf16_t* __restrict__ wb, float* __restrict__ gpart,
                                                        double* __restrict__ lpart, int grad, int judge, float pj)
{
    using N = NetGeo<DIM>;
    extern __shared__ __align__(16) unsigned char smem[];
    bf16_t* act = reinterpret_cast<bf16_t*>(smem);   // X0..X3, then the two gradient buffers
    bf16_t* d0 = act + 4 * N::ACT;
    bf16_t* d1 = d0 + N::ACT;
    float* out0 = reinterpret_cast<float*>(d1 + N::ACT);
    float* tgt = out0 + N::TILES * 16;
    short* linq = reinterpret_cast<short*>(tgt + N::TILES * 16);
    __shared__ double red[kNetThreads / 64];

    const int s = net_sample(blockIdx.x, base, pa, pb, npairs);
    net_zero(act, 6 * N::ACT);
    net_fill_lin<DIM>(linq);
    __syncthreads();
    net_load<DIM>(r + (size_t)s * N::PTS, judge ? nullptr : e + (size_t)s * N::PTS, normalize, act, tgt, red,
                  judge != 0);
    __syncthreads();
    const int WLY = N::WLY, GLY = N::GLY;
    net_conv_fwd<DIM, true>(act, act + N::ACT, nullptr, wf, linq);
    __syncthreads();
    net_conv_fwd<DIM, true>(act + N::ACT, act + 2 * N::ACT, nullptr, wf + WLY, linq);
    __syncthreads();
    net_conv_fwd<DIM, true>(act + 2 * N::ACT, act + 3 * N::ACT, nullptr, wf + 2 * WLY, linq);
    __syncthreads();
    net_conv_fwd<DIM, false>(act + 3 * N::ACT, nullptr, out0, wf + 3 * WLY, linq);
    __syncthreads();
    double l = 0;
    if (judge) {
        l = net_judge_loss<DIM>(out0, tgt, linq, pj, inv_cnt, d0, d1, grad, red);
    } else {
        for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) {
            float d = out0[q] - tgt[q];
            l += (double)d * d;
            if (grad) d0[linq[q] * kNetCh] = f2bf(2.f * d * inv_cnt);
        }
        l = block_sum(l, red);
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = l;
    if (!grad) return;
    float* gw = gpart + (size_t)blockIdx.x * N::NW;
    net_conv_bwd_weight<DIM>(act + 3 * N::ACT, d0, gw + 3 * GLY, linq);
    net_conv_bwd_data<DIM>(d0, act + 3 * N::ACT, d1, wb + 3 * WLY, linq);
    __syncthreads();
    net_conv_bwd_weight<DIM>(act + 2 * N::ACT, d1, gw + 2 * GLY, linq);
    net_conv_bwd_data<DIM>(d1, act + 2 * N::ACT, d0, wb + 2 * WLY, linq);
    __syncthreads();
    net_conv_bwd_weight<DIM>(act + N::ACT, d0, gw + GLY, linq);
    net_conv_bwd_data<DIM>(d0, act + N::ACT, d1, wb + WLY, linq);
    __syncthreads();
    net_conv_bwd_weight<DIM>(act, d1, gw, linq);
}

// Inference on a batch: out = network(in) (scaled back when normalize).
template <int DIM>
__global__ void __launch_bounds__(kNetThreads) kn_forward(const double* __restrict__ in, double* __restrict__ out,
                                                          int normalize, const bf16_t* __restrict__ wf)
{
    using N = NetGeo<DIM>;
    extern __shared__ __align__(16) unsigned char smem[];
    bf16_t* A = reinterpret_cast<bf16_t*>(smem);
    bf16_t* B = A + N::ACT;
    float* out0 = reinterpret_cast<float*>(B + N::ACT);
    short* linq = reinterpret_cast<short*>(out0 + N::TILES * 16);
    __shared__ double red[kNetThreads / 64];
    const size_t s = blockIdx.x;
    net_zero(A, 2 * N::ACT);
    net_fill_lin<DIM>(linq);
    __syncthreads();
    double back = net_load<DIM>(in + s * N::PTS, nullptr, normalize, A, nullptr, red);
    __syncthreads();
    const int WLY = N::WLY;
    net_conv_fwd<DIM, true>(A, B, nullptr, wf, linq);
    __syncthreads();
    net_conv_fwd<DIM, true>(B, A, nullptr, wf + WLY, linq);
    __syncthreads();
    net_conv_fwd<DIM, true>(A, B, nullptr, wf + 2 * WLY, linq);
    __syncthreads();
    net_conv_fwd<DIM, false>(B, nullptr, out0, wf + 3 * WLY, linq);
    __syncthreads();
    double* o = out + s * N::PTS;
    for (int p = threadIdx.x; p < N::PTS; p += blockDim.x) o[p] = 0.0;
    __syncthreads();
    for (int q = threadIdx.x; q < N::NIN; q += blockDim.x) o[N::lin(q)] = (double)out0[q] * back;
}

// Sum of the per-sample gradients in a fixed order, then (update) one Adam
// step on the master weights and the packed bf16 copies.  Thread 0 adds the
// batch loss to *loss_acc.
template <int DIM>
__global__ void __launch_bounds__(256) kn_adam(const float* __restrict__ gpart, int B, float* __restrict__ w,
                                               float* __restrict__ m, float* __restrict__ v, int step, float lr,
                                               float b1, float b2, float eps, bf16_t* __restrict__ wf,
                                               bf16_t* __restrict__ wb, float* __restrict__ gout, int update,
                                               const double* __restrict__ lpart, double* __restrict__ loss_acc,
                                               double inv_cnt)
{
    using N = NetGeo<DIM>;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && loss_acc) {
        double s = 0;
        for (int b = 0; b < B; b++) s += lpart[b];
        *loss_acc += s * inv_cnt;
    }
    if (i >= N::NW) return;
    double gs = 0;
    for (int b = 0; b < B; b++) gs += gpart[(size_t)b * N::NW + i];
    const int lt = i >> 8, ci = (i >> 4) & 15, co = i & 15, layer = lt / N::T, tap = lt % N::T;
    if ((layer == 0 && ci != 0) || (layer == kNetLayers - 1 && co != 0)) gs = 0;
    const float g = (float)gs;
    if (gout) gout[i] = g;
    if (!update) return;
    float mi = b1 * m[i] + (1.f - b1) * g;
    float vi = b2 * v[i] + (1.f - b2) * g * g;
    float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    m[i] = mi;
    v[i] = vi;
    w[i] = wi;
    bf16_t h = f2bf(wi);
    wf[net_pack_fwd(N::T, layer, tap, ci, co)] = h;
    wb[net_pack_bwd(N::T, layer, tap, ci, co)] = h;
}

template <int DIM>
void net_set_lds_limits()
{
    (void)hipFuncSetAttribute((const void*)kn_train<DIM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)net_lds_train<DIM>());
    (void)hipFuncSetAttribute((const void*)kn_forward<DIM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)net_lds_fwd<DIM>());
}

}  // namespace dmg

using namespace dmg;

constexpr int kMaxEpochs = 4096;

struct mg_net {
    int dim = 2, max_batch = 0, device = 0, nw = 0, step = 0;
    int judge = 0;      // loss: 0 mean squared error to the target, 1 the cut-level objective
    float pj = 1.f;     // the cut level's over-relaxation parameter (judge)
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t off_w = 0, off_m = 0, off_v = 0, off_wf = 0, off_wb = 0, off_gpart = 0, off_lpart = 0, off_gout = 0,
           off_loss = 0, total = 0;
    template <typename T>
    T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

int net_nw(int dim) { return dim == 2 ? NetGeo<2>::NW : NetGeo<3>::NW; }
int net_nin(int dim) { return dim == 2 ? NetGeo<2>::NIN : NetGeo<3>::NIN; }
int net_taps(int dim) { return dim == 2 ? 9 : 27; }
int net_pack_len(int dim) { return dim == 2 ? NetGeo<2>::PACK : NetGeo<3>::PACK; }

void net_layout(mg_net& N)
{
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = alignUp(off + b); return o; };
    size_t nw = (size_t)N.nw;
    N.off_w = take(4 * nw);
    N.off_m = take(4 * nw);
    N.off_v = take(4 * nw);
    N.off_wf = take(2 * (size_t)net_pack_len(N.dim));   // packed forms; odd tap counts pad with zeros
    N.off_wb = take(2 * (size_t)net_pack_len(N.dim));
    N.off_gpart = take(4 * nw * (size_t)N.max_batch);
    N.off_lpart = take(8 * (size_t)N.max_batch);
    N.off_gout = take(4 * nw);
    N.off_loss = take(8 * (size_t)kMaxEpochs);
    N.total = off;
}

int launch_train(mg_net& N, const double* r, const double* e, int B, long long base, long long pa, long long pb,
                 int npairs, int normalize, float inv_cnt, int grad)
{
    if (N.dim == 2)
        hipLaunchKernelGGL(kn_train<2>, dim3(B), dim3(kNetThreads), net_lds_train<2>(), N.stream, r, e, base, pa, pb, npairs,
                           normalize, inv_cnt, N.at<bf16_t>(N.off_wf), N.at<bf16_t>(N.off_wb), N.at<float>(N.off_gpart),
                           N.at<double>(N.off_lpart), grad, N.judge, N.pj);
    else
        hipLaunchKernelGGL(kn_train<3>, dim3(B), dim3(kNetThreads), net_lds_train<3>(), N.stream, r, e, base, pa, pb, npairs,
                           normalize, inv_cnt, N.at<bf16_t>(N.off_wf), N.at<bf16_t>(N.off_wb), N.at<float>(N.off_gpart),
                           N.at<double>(N.off_lpart), grad, N.judge, N.pj);
    return last_launch();
}

int launch_adam(mg_net& N, int B, float lr, int update, double* loss_acc, double inv_cnt)
{
    int blocks = (N.nw + 255) / 256;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    if (N.dim == 2)
        hipLaunchKernelGGL(kn_adam<2>, dim3(blocks), dim3(256), 0, N.stream, N.at<float>(N.off_gpart), B, N.at<float>(N.off_w),
                           N.at<float>(N.off_m), N.at<float>(N.off_v), N.step, lr, b1, b2, eps, N.at<bf16_t>(N.off_wf),
                           N.at<bf16_t>(N.off_wb), N.at<float>(N.off_gout), update, N.at<double>(N.off_lpart), loss_acc,
                           inv_cnt);
    else
        hipLaunchKernelGGL(kn_adam<3>, dim3(blocks), dim3(256), 0, N.stream, N.at<float>(N.off_gpart), B, N.at<float>(N.off_w),
                           N.at<float>(N.off_m), N.at<float>(N.off_v), N.step, lr, b1, b2, eps, N.at<bf16_t>(N.off_wf),
                           N.at<bf16_t>(N.off_wb), N.at<float>(N.off_gout), update, N.at<double>(N.off_lpart), loss_acc,
                           inv_cnt);
    return last_launch();
}

uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

long long gcdll(long long a, long long b) { while (b) { long long t = a % b; a = b; b = t; } return a; }

}  // namespace

namespace dmg {

// host packing of fp32 weights [layer][tap][ci][co] into the two bf16 forms
// (each of net_pack_len(dim) entries; the padding entries are set to zero)
void net_pack_host(int dim, const float* w, bf16_t* wf, bf16_t* wb)
{
    const int T = net_taps(dim), len = net_pack_len(dim);
    if (wf) memset(wf, 0, sizeof(bf16_t) * len);
    if (wb) memset(wb, 0, sizeof(bf16_t) * len);
    for (int layer = 0; layer < kNetLayers; layer++)
        for (int tap = 0; tap < T; tap++)
            for (int ci = 0; ci < kNetCh; ci++)
                for (int co = 0; co < kNetCh; co++) {
                    bf16_t h = f2bf(w[((layer * T + tap) * kNetCh + ci) * kNetCh + co]);
                    if (wf) wf[net_pack_fwd(T, layer, tap, ci, co)] = h;
                    if (wb) wb[net_pack_bwd(T, layer, tap, ci, co)] = h;
                }
}

int net_weight_count(int dim) { return (dim == 2 || dim == 3) ? net_nw(dim) : 0; }

}  // namespace dmg

extern "C" {

int mg_net_workspace_bytes(int dim, int max_batch, size_t* bytes)
{
    if (!bytes || (dim != 2 && dim != 3) || max_batch < 1) return MG_ERR_ARG;
    mg_net N;
    N.dim = dim;
    N.nw = net_nw(dim);
    N.max_batch = max_batch;
    net_layout(N);
    *bytes = N.total;
    return MG_OK;
}

int mg_net_create(mg_net** out, int dim, int max_batch, void* workspace, size_t ws_bytes, void* hip_stream)
{
    if (!out) return MG_ERR_ARG;
    *out = nullptr;
    if ((dim != 2 && dim != 3) || max_batch < 1) return MG_ERR_ARG;
    mg_net* N = new (std::nothrow) mg_net;
    if (!N) return MG_ERR_ALLOC;
    N->dim = dim;
    N->nw = net_nw(dim);
    N->max_batch = max_batch;
    net_layout(*N);
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || ws_bytes < N->total) { delete N; return MG_ERR_WS; }
    N->ws = (char*)workspace;
    N->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&N->device) != hipSuccess) { delete N; return MG_ERR_HIP; }
    if (dim == 2) net_set_lds_limits<2>(); else net_set_lds_limits<3>();
    if (hipMemsetAsync(N->ws, 0, N->total, N->stream) != hipSuccess || hipStreamSynchronize(N->stream) != hipSuccess) {
        delete N;
        return MG_ERR_HIP;
    }
    *out = N;
    return MG_OK;
}

int mg_net_set_weights(mg_net* N, const float* w)
{
    if (!N || !w) return MG_ERR_ARG;
    DevGuard g(N->device);
    std::vector<float> wm(w, w + N->nw);
    int T = net_taps(N->dim);
    for (int lt = 0; lt < kNetLayers * T; lt++)   // the padded channels are not parameters
        for (int ci = 0; ci < kNetCh; ci++)
            for (int co = 0; co < kNetCh; co++) {
                int layer = lt / T;
                if ((layer == 0 && ci) || (layer == kNetLayers - 1 && co)) wm[(lt * kNetCh + ci) * kNetCh + co] = 0.f;
            }
    const size_t np = (size_t)net_pack_len(N->dim);
    std::vector<bf16_t> wf(np), wb(np);
    net_pack_host(N->dim, wm.data(), wf.data(), wb.data());
    size_t nb = sizeof(float) * N->nw;
    if (hipMemcpyAsync(N->at<float>(N->off_w), wm.data(), nb, hipMemcpyHostToDevice, N->stream) != hipSuccess ||
        hipMemsetAsync(N->at<float>(N->off_m), 0, nb, N->stream) != hipSuccess ||
        hipMemsetAsync(N->at<float>(N->off_v), 0, nb, N->stream) != hipSuccess ||
        hipMemcpyAsync(N->at<bf16_t>(N->off_wf), wf.data(), sizeof(bf16_t) * np, hipMemcpyHostToDevice, N->stream) != hipSuccess ||
        hipMemcpyAsync(N->at<bf16_t>(N->off_wb), wb.data(), sizeof(bf16_t) * np, hipMemcpyHostToDevice, N->stream) != hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess)
        return MG_ERR_HIP;
    N->step = 0;
    return MG_OK;
}

int mg_net_get_weights(mg_net* N, float* w)
{
    if (!N || !w) return MG_ERR_ARG;
    DevGuard g(N->device);
    if (hipMemcpyAsync(w, N->at<float>(N->off_w), sizeof(float) * N->nw, hipMemcpyDeviceToHost, N->stream) != hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess)
        return MG_ERR_HIP;
    return MG_OK;
}

int mg_net_init(mg_net* N, unsigned long long seed)
{
    if (!N) return MG_ERR_ARG;
    // He initialisation: N(0, 2 / fan_in), fan_in = taps x active input channels
    std::vector<float> w(N->nw, 0.f);
    uint64_t s = seed;
    int T = net_taps(N->dim);
    for (int i = 0; i < N->nw; i++) {
        int lt = i >> 8, ci = (i >> 4) & 15, co = i & 15, layer = lt / T;
        if ((layer == 0 && ci) || (layer == kNetLayers - 1 && co)) continue;
        double u1 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double u2 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        double fan = (double)T * (layer == 0 ? 1 : kNetCh);
        w[i] = (float)(z * sqrt(2.0 / fan));
    }
    return mg_net_set_weights(N, w.data());
}

int mg_net_forward(mg_net* N, const double* in, double* out, int batch, int normalize)
{
    if (!N || !in || !out || batch < 0) return MG_ERR_ARG;
    if (batch == 0) return MG_OK;
    DevGuard g(N->device);
    if (N->dim == 2)
        hipLaunchKernelGGL(kn_forward<2>, dim3(batch), dim3(kNetThreads), net_lds_fwd<2>(), N->stream, in, out, normalize,
                           N->at<bf16_t>(N->off_wf));
    else
        hipLaunchKernelGGL(kn_forward<3>, dim3(batch), dim3(kNetThreads), net_lds_fwd<3>(), N->stream, in, out, normalize,
                           N->at<bf16_t>(N->off_wf));
    return last_launch();
}

int mg_net_set_loss(mg_net* N, int kind, double pj)
{
    if (!N || (kind != MG_NET_LOSS_MSE && kind != MG_NET_LOSS_CUT)) return MG_ERR_ARG;
    if (kind == MG_NET_LOSS_CUT && !(pj > 0.0 && pj < 1e3)) return MG_ERR_ARG;
    N->judge = kind == MG_NET_LOSS_CUT;
    N->pj = kind == MG_NET_LOSS_CUT ? (float)pj : 1.f;
    return MG_OK;
}

int mg_net_loss_grad(mg_net* N, const double* in, const double* target, int batch, int normalize, float* grad,
                     double* loss)
{
    if (!N || !in || (!target && !N->judge) || batch < 1 || batch > N->max_batch) return MG_ERR_ARG;
    DevGuard g(N->device);
    double inv = 1.0 / ((double)batch * net_nin(N->dim));
    int e = launch_train(*N, in, target, batch, 0, 1, 0, 0, normalize, (float)inv, 1);
    if (e) return e;
    double* lacc = N->at<double>(N->off_loss);
    if (hipMemsetAsync(lacc, 0, sizeof(double), N->stream) != hipSuccess) return MG_ERR_HIP;
    if ((e = launch_adam(*N, batch, 0.f, 0, lacc, inv))) return e;
    if (grad && hipMemcpyAsync(grad, N->at<float>(N->off_gout), sizeof(float) * N->nw, hipMemcpyDeviceToHost,
                               N->stream) != hipSuccess)
        return MG_ERR_HIP;
    double l = 0;
    if (hipMemcpyAsync(&l, lacc, sizeof(double), hipMemcpyDeviceToHost, N->stream) != hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess)
        return MG_ERR_HIP;
    if (loss) *loss = l;
    return MG_OK;
}

int mg_net_train(mg_net* N, const double* r, const double* e, int npairs, int epochs, int batch, float lr,
                 unsigned long long seed, double* epoch_loss)
{
    if (!N || !r || (!e && !N->judge) || npairs < 1 || epochs < 0 || epochs > kMaxEpochs || batch < 1 || batch > N->max_batch ||
        batch > npairs || !(lr > 0.f))
        return MG_ERR_ARG;
    DevGuard g(N->device);
    double* lacc = N->at<double>(N->off_loss);
    if (hipMemsetAsync(lacc, 0, sizeof(double) * (size_t)(epochs > 0 ? epochs : 1), N->stream) != hipSuccess)
        return MG_ERR_HIP;
    const int steps = npairs / batch;
    const double inv = 1.0 / ((double)batch * net_nin(N->dim));
    uint64_t s = seed;
    for (int ep = 0; ep < epochs; ep++) {
        // this epoch's order: k -> (pa k + pb) mod npairs with pa coprime to npairs
        long long pa = 1, pb = 0;
        if (npairs > 1) {
            do { pa = 1 + (long long)(splitmix64(s) % (uint64_t)(npairs - 1)); } while (gcdll(pa, npairs) != 1);
            pb = (long long)(splitmix64(s) % (uint64_t)npairs);
        }
        for (int k = 0; k < steps; k++) {
            int err = launch_train(*N, r, e, batch, (long long)k * batch, pa, pb, npairs, 1, (float)inv, 1);
            if (err) return err;
            N->step++;
            if ((err = launch_adam(*N, batch, lr, 1, lacc + ep, inv)))
                return err;
        }
    }
    if (epoch_loss && epochs > 0) {
        std::vector<double> h(epochs);
        if (hipMemcpyAsync(h.data(), lacc, sizeof(double) * epochs, hipMemcpyDeviceToHost, N->stream) != hipSuccess ||
            hipStreamSynchronize(N->stream) != hipSuccess)
            return MG_ERR_HIP;
        for (int ep = 0; ep < epochs; ep++) epoch_loss[ep] = steps ? h[ep] / steps : 0.0;
    } else if (hipStreamSynchronize(N->stream) != hipSuccess) {
        return MG_ERR_HIP;
    }
    return MG_OK;
}

int mg_net_destroy(mg_net* N)
{
    if (!N) return MG_OK;
    {
        DevGuard g(N->device);
        (void)hipStreamSynchronize(N->stream);
    }
    delete N;
    return MG_OK;
}

}  // extern "C"

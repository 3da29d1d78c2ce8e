// Host runtime of libdmg: the level plan, workspace carving, launch
// sequencing of one V-cycle and the outer iteration, and the exported C ABI
// declared in include/dmg.h.
//
// One V-cycle (Roberts, Section 1): residual on the finest grid, restriction
// level by level (Sections 2.1 / 3.1), all coarse levels in one persistent
// workgroup, Jacobi prolongation level by level back up (Sections 2.2, 2.5 /
// 3.2, 3.5), the finest Jacobi fused with u += v.
#include "../../include/dmg.h"
#include "dmg_launch.hpp"
#include "dmg_launch3.hpp"

#include <new>
#include <stdlib.h>
#include <string.h>

using namespace dmg;

namespace {

// levels with side <= kCoarseSide (2D) / kCoarseSide3 (3D) go to the persistent kernel
constexpr int kCoarseSide = 32;
constexpr int kCoarseSide3 = 8;

int ilog2(int n)
{
    if (n < 2) return -1;
    int k = 0;
    while ((1 << k) < n) k++;
    return ((1 << k) == n) ? k : -1;
}

struct Level {
    int m = 0;
    int kind = 0;  // 2D: 0 axis, 1 diagonal.  3D: 0 green, 1 red, 2 magenta
    size_t r = 0, v = 0;    // byte offsets; magenta: corner (E) arrays
    size_t r2 = 0, v2 = 0;  // magenta: cube-centre (O) arrays
    double c = 0, c2 = 0;   // Jacobi residual coefficients
};

struct Layout {
    int dim = 0, n = 0, prec = 0, D = 0, dc = 0;
    size_t ctl = 0, partial = 0, zero = 0, r0 = 0, total = 0;
    int nparts = 0;
    Level lev[kMaxLev];
};

int level_count(int dim, int n)
{
    int K = ilog2(n);
    return (dim == 2 ? 2 : 3) * (K - 1) + 1;
}

int side_of(int dim, int n, int d) { return n >> (d / dim); }

int check_size(int dim, int n)
{
    if (dim != 2 && dim != 3) return MG_ERR_ARG;
    int K = ilog2(n);
    if (K < 1) return MG_ERR_SIZE;
    if (dim == 2 && K > 15) return MG_ERR_SIZE;
    if (dim == 3 && K > 11) return MG_ERR_SIZE;
    return MG_OK;
}

int make_layout(int dim, int n, int prec, const double* p, Layout& L)
{
    int e = check_size(dim, n);
    if (e) return e;
    if (prec != MG_FP64 && prec != MG_FP32_REFINED) return MG_ERR_ARG;
    size_t es = prec == MG_FP64 ? sizeof(double) : sizeof(float);
    L.dim = dim;
    L.n = n;
    L.prec = prec;
    L.D = level_count(dim, n) - 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = alignUp(off + bytes);
        return o;
    };
    L.ctl = take(sizeof(Ctl));
    L.nparts = residual_parts(dim, n);
    L.partial = take(sizeof(double) * (size_t)L.nparts);
    L.zero = take(sizeof(double) * 64);
    L.r0 = take(es * (dim == 2 ? sizeA(n) : sizeG(n)));
    double h = 1.0 / n;
    for (int d = 0; d <= L.D; d++) {
        Level& v = L.lev[d];
        v.m = side_of(dim, n, d);
        v.kind = d % dim;
        double sh = (double)(n / v.m) * h;  // sigma * h
        if (dim == 2) {
            double pp = p ? p[0] : 1.0;
            v.c = v.kind ? 2 * pp * sh * sh : pp * sh * sh;
            if (d >= 1) {
                size_t cnt = v.kind ? sizeD(v.m) : sizeA(v.m);
                v.r = take(es * cnt);
                v.v = take(es * cnt);
            }
        } else {
            double pm = p ? p[0] : 1, pr1 = p ? p[1] : 1, pr2 = p ? p[2] : 1, pg = p ? p[3] : 1;
            if (v.kind == 0) v.c = pg * sh * sh;
            else if (v.kind == 1) { v.c = 2 * pr1 * sh * sh; v.c2 = 4 * pr2 * sh * sh; }
            else v.c = 4 * pm * sh * sh;
            if (d >= 1) {
                if (v.kind == 0) { v.r = take(es * sizeG(v.m)); v.v = take(es * sizeG(v.m)); }
                else if (v.kind == 1) { v.r = take(es * sizeR(v.m)); v.v = take(es * sizeR(v.m)); }
                else {
                    v.r = take(es * sizeME(v.m)); v.v = take(es * sizeME(v.m));
                    v.r2 = take(es * sizeMO(v.m)); v.v2 = take(es * sizeMO(v.m));
                }
            }
        }
    }
    // first depth handled by the coarse persistent kernel (0: no coarse kernel)
    L.dc = 0;
    if (L.D >= 1) {
        int lim = dim == 2 ? kCoarseSide : kCoarseSide3;
        for (int d = 1; d <= L.D; d++)
            if (L.lev[d].m <= lim) { L.dc = d; break; }
        if (dim == 3 && L.dc > 1) {
            // start the persistent part on a green level so that it runs whole groups
            while (L.dc % 3 != 0 && L.dc > 1) L.dc--;
        }
    }
    L.total = off;
    return MG_OK;
}

}  // namespace

struct mg_plan {
    Layout L;
    double p[4];
    hipStream_t stream;
    int device;
    char* ws;
    size_t ws_bytes;
    Ctl* hctl;  // pinned host copy of the control block
};

namespace {

template <typename T>
T* at(mg_plan* P, size_t off) { return reinterpret_cast<T*>(P->ws + off); }

struct DevGuard {
    int old = -1;
    bool ok = true;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) { ok = false; return; }
        if (old != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DevGuard()
    {
        if (old >= 0) { int cur; if (hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old); }
    }
};

template <typename T>
void enqueue_cycle_2d(mg_plan* P, double* u, const Ctl* ctl)
{
    Layout& L = P->L;
    hipStream_t s = P->stream;
    int D = L.D, dc = L.dc;
    T* r0 = at<T>(P, L.r0);
    auto R = [&](int d) -> T* { return d == 0 ? r0 : at<T>(P, L.lev[d].r); };
    auto V = [&](int d) -> T* { return at<T>(P, L.lev[d].v); };
    int last_rs = dc ? dc : D;
    for (int d = 1; d <= last_rs; d++) launch_rs2<T>((d - 1) % 2, L.lev[d - 1].m, R(d - 1), R(d), ctl, s);
    if (dc) {
        Coarse2<T> a;
        a.first = dc;
        a.last = D;
        for (int d = dc; d <= D; d++) {
            a.lev[d].m = L.lev[d].m;
            a.lev[d].diag = L.lev[d].kind;
            a.lev[d].r = R(d);
            a.lev[d].v = V(d);
            a.lev[d].c = (T)L.lev[d].c;
        }
        a.zeroD = at<T>(P, L.zero);
        launch_coarse2<T>(a, ctl, s);
    }
    for (int d = (dc ? dc - 1 : D); d >= 1; d--) {
        const T* vc = (d == D) ? at<T>(P, L.zero) : V(d + 1);
        launch_jac2<T>(L.lev[d].kind, L.lev[d].m, (T)L.lev[d].c, R(d), vc, V(d), ctl, s);
    }
    const T* v1 = D >= 1 ? V(1) : at<T>(P, L.zero);
    launch_jac2_finest<T>(L.n, (T)L.lev[0].c, r0, v1, u, ctl, s);
}

template <typename T>
void enqueue_cycle(mg_plan* P, double* u, const double* f, const Ctl* ctl, bool resid)
{
    Layout& L = P->L;
    if (resid)
        launch_residual<T>(L.dim, L.n, u, f, at<T>(P, L.r0), at<double>(P, L.partial), L.nparts, ctl, P->stream);
    if (L.dim == 2) enqueue_cycle_2d<T>(P, u, ctl);
    else enqueue_cycle_3d<T>(P, u, ctl);
}

int hip_status(hipError_t e) { return e == hipSuccess ? MG_OK : MG_ERR_HIP; }

int last_launch() { return hip_status(hipGetLastError()); }

}  // namespace

// 3D sequencing lives here too so it can reach the plan internals.
namespace {
template <typename T>
void enqueue_cycle_3d_impl(mg_plan* P, double* u, const Ctl* ctl)
{
    Layout& L = P->L;
    hipStream_t s = P->stream;
    int D = L.D, dc = L.dc;
    T* r0 = at<T>(P, L.r0);
    auto lv = [&](int d) {
        Lev3<T> x;
        const Level& q = L.lev[d];
        x.m = q.m;
        x.kind = q.kind;
        x.r = d == 0 ? r0 : at<T>(P, q.r);
        x.v = d == 0 ? nullptr : at<T>(P, q.v);
        x.r2 = q.kind == 2 ? at<T>(P, q.r2) : nullptr;
        x.v2 = q.kind == 2 ? at<T>(P, q.v2) : nullptr;
        x.c = (T)q.c;
        x.c2 = (T)q.c2;
        return x;
    };
    int last_rs = dc ? dc : D;
    for (int d = 1; d <= last_rs; d++) launch_rs3<T>(lv(d - 1), lv(d), ctl, s);
    if (dc) {
        Coarse3<T> a;
        a.first = dc;
        a.last = D;
        for (int d = dc; d <= D; d++) a.lev[d] = lv(d);
        a.zero = at<T>(P, L.zero);
        launch_coarse3<T>(a, ctl, s);
    }
    for (int d = (dc ? dc - 1 : D); d >= 1; d--) {
        Lev3<T> c = (d == D) ? Lev3<T>{} : lv(d + 1);
        launch_jac3<T>(lv(d), c, at<T>(P, L.zero), ctl, s);
    }
    Lev3<T> c1 = D >= 1 ? lv(1) : Lev3<T>{};
    launch_jac3_finest<T>(L.n, (T)L.lev[0].c, r0, D >= 1 ? c1.v : at<T>(P, L.zero), u, ctl, s);
}
}  // namespace

template <typename T>
void enqueue_cycle_3d(mg_plan* P, double* u, const Ctl* ctl) { enqueue_cycle_3d_impl<T>(P, u, ctl); }

extern "C" {

const char* mg_strerror(int code)
{
    switch (code) {
    case MG_OK: return "ok";
    case MG_ERR_ARG: return "invalid argument";
    case MG_ERR_SIZE: return "n must be a power of two in the supported range";
    case MG_ERR_WS: return "workspace null, misaligned or too small";
    case MG_ERR_ALLOC: return "host allocation failed";
    case MG_ERR_HIP: return "HIP runtime error";
    case MG_ERR_NONFINITE: return "residual is not finite";
    case MG_ERR_DIVERGED: return "iteration diverged";
    case MG_ERR_NOT_CONVERGED: return "not converged within max_cycles";
    default: return "unknown error code";
    }
}

int mg_level_info(int dim, int n, int depth, int* num_levels, int* side)
{
    int e = check_size(dim, n);
    if (e) return e;
    int nl = level_count(dim, n);
    if (num_levels) *num_levels = nl;
    if (side) {
        if (depth < 0 || depth >= nl) return MG_ERR_ARG;
        *side = side_of(dim, n, depth);
    }
    return MG_OK;
}

int mg_workspace_bytes(int dim, int n, int precision, size_t* bytes)
{
    if (!bytes) return MG_ERR_ARG;
    Layout L;
    int e = make_layout(dim, n, precision, nullptr, L);
    if (e) return e;
    *bytes = L.total;
    return MG_OK;
}

int mg_setup(mg_plan** out, int dim, int n, int precision, const double* p, int np, void* workspace,
             size_t ws_bytes, void* hip_stream)
{
    if (!out || !p) return MG_ERR_ARG;
    *out = nullptr;
    if ((dim == 2 && np != 1) || (dim == 3 && np != 4)) return MG_ERR_ARG;
    for (int i = 0; i < np; i++)
        if (!(p[i] > 0 && p[i] < 1e6)) return MG_ERR_ARG;
    mg_plan* P = new (std::nothrow) mg_plan;
    if (!P) return MG_ERR_ALLOC;
    int e = make_layout(dim, n, precision, p, P->L);
    if (e) { delete P; return e; }
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || ws_bytes < P->L.total) { delete P; return MG_ERR_WS; }
    for (int i = 0; i < 4; i++) P->p[i] = i < np ? p[i] : 0;
    P->stream = (hipStream_t)hip_stream;
    P->ws = (char*)workspace;
    P->ws_bytes = ws_bytes;
    P->hctl = nullptr;
    if (hipGetDevice(&P->device) != hipSuccess) { delete P; return MG_ERR_HIP; }
    if (hipHostMalloc((void**)&P->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
        delete P;
        return MG_ERR_HIP;
    }
    // zero the whole workspace once: boundary entries of every level stay 0
    if (hipMemsetAsync(P->ws, 0, P->L.total, P->stream) != hipSuccess) {
        (void)hipHostFree(P->hctl);
        delete P;
        return MG_ERR_HIP;
    }
    *out = P;
    return MG_OK;
}

int mg_destroy(mg_plan* P)
{
    if (!P) return MG_ERR_ARG;
    if (P->hctl) (void)hipHostFree(P->hctl);
    delete P;
    return MG_OK;
}

int mg_vcycle(mg_plan* P, double* u, const double* f, double* rel_res_before)
{
    if (!P || !u || !f) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    Layout& L = P->L;
    Ctl* ctl = at<Ctl>(P, L.ctl);
    double* part = at<double>(P, L.partial);
    launch_ctl_reset(ctl, 0, 0, 0.0, P->stream);
    if (rel_res_before) {
        launch_sumsq(L.dim, L.n, f, part, L.nparts, ctl, P->stream);
        launch_finalize(0, 0, part, L.nparts, ctl, P->stream);
    }
    bool dbl = L.prec == MG_FP64;
    if (dbl) launch_residual<double>(L.dim, L.n, u, f, at<double>(P, L.r0), part, L.nparts, ctl, P->stream);
    else launch_residual<float>(L.dim, L.n, u, f, at<float>(P, L.r0), part, L.nparts, ctl, P->stream);
    if (rel_res_before) launch_finalize(1, 0, part, L.nparts, ctl, P->stream);
    if (dbl) enqueue_cycle<double>(P, u, f, ctl, false);
    else enqueue_cycle<float>(P, u, f, ctl, false);
    int e = last_launch();
    if (e) return e;
    if (rel_res_before) {
        if (hipMemcpyAsync(P->hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P->stream) != hipSuccess)
            return MG_ERR_HIP;
        if (hipStreamSynchronize(P->stream) != hipSuccess) return MG_ERR_HIP;
        *rel_res_before = P->hctl->last;
    }
    return MG_OK;
}

int mg_solve(mg_plan* P, double* u, const double* f, double rtol, int max_cycles, int* cycles_out,
             double* rel_res_out, double* history)
{
    if (!P || !u || !f || !(rtol >= 0) || max_cycles < 0 || max_cycles > kMaxCycles) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    Layout& L = P->L;
    Ctl* ctl = at<Ctl>(P, L.ctl);
    double* part = at<double>(P, L.partial);
    hipStream_t s = P->stream;
    bool dbl = L.prec == MG_FP64;
    launch_ctl_reset(ctl, 1, max_cycles, rtol, s);
    launch_sumsq(L.dim, L.n, f, part, L.nparts, ctl, s);
    launch_finalize(0, 0, part, L.nparts, ctl, s);
    size_t head = offsetof(Ctl, rtol);
    for (int k = 0; k <= max_cycles; k++) {
        if (dbl) launch_residual<double>(L.dim, L.n, u, f, at<double>(P, L.r0), part, L.nparts, ctl, s);
        else launch_residual<float>(L.dim, L.n, u, f, at<float>(P, L.r0), part, L.nparts, ctl, s);
        launch_finalize(1, k, part, L.nparts, ctl, s);
        if (k == max_cycles) break;
        if (dbl) enqueue_cycle<double>(P, u, f, ctl, false);
        else enqueue_cycle<float>(P, u, f, ctl, false);
        int e = last_launch();
        if (e) return e;
        // the device decides; the host only stops enqueueing once it sees `done`
        if (hipMemcpyAsync(P->hctl, ctl, head, hipMemcpyDeviceToHost, s) != hipSuccess) return MG_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
        if (P->hctl->done) break;
    }
    if (hipMemcpyAsync(P->hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess) return MG_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
    const Ctl& H = *P->hctl;
    int cyc = H.done ? H.cycles : max_cycles;
    if (cycles_out) *cycles_out = cyc;
    if (rel_res_out) *rel_res_out = H.last;
    if (history)
        for (int k = 0; k <= cyc; k++) history[k] = H.hist[k];
    return H.done ? H.status : MG_ERR_NOT_CONVERGED;
}

int mg_level_get(mg_plan* P, int depth, int which, double* dst)
{
    if (!P || !dst) return MG_ERR_ARG;
    Layout& L = P->L;
    if (depth < 0 || depth > L.D || (which != 0 && which != 1) || (which == 1 && depth == 0)) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    const Level& q = L.lev[depth];
    size_t src = which == 0 ? (depth == 0 ? L.r0 : q.r) : q.v;
    size_t src2 = which == 0 ? q.r2 : q.v2;
    if (L.dim == 2) {
        if (L.prec == MG_FP64) launch_level_get2<double>(q.kind, q.m, at<double>(P, src), dst, P->stream);
        else launch_level_get2<float>(q.kind, q.m, at<float>(P, src), dst, P->stream);
    } else {
        if (L.prec == MG_FP64)
            launch_level_get3<double>(q.kind, q.m, at<double>(P, src), q.kind == 2 ? at<double>(P, src2) : nullptr,
                                      dst, P->stream);
        else
            launch_level_get3<float>(q.kind, q.m, at<float>(P, src), q.kind == 2 ? at<float>(P, src2) : nullptr,
                                     dst, P->stream);
    }
    return last_launch();
}

}  // extern "C"

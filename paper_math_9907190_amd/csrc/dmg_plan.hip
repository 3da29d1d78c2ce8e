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
#include "dmg_rows.hpp"

#include <new>
#include <stdlib.h>
#include <string.h>

using namespace dmg;

namespace {

// levels with side <= kCoarseSide (2D) / kCoarseSide3 (3D) go to the persistent kernel
constexpr int kCoarseSide = 32;
constexpr int kCoarseSide3 = 8;
// 2D levels of at least this side use the row-marching kernels; smaller ones
// are latency-bound and use one thread per point (a single round of loads)
constexpr int kRowsMinSide = 512;

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
    int nparts_f = 0;   // partial sums written by the norm of f
    int nparts_r = 0;   // partial sums written by the residual kernel
    bool fused_rs1 = false;  // 2D: the residual kernel also restricts to level 1
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
    L.fused_rs1 = (dim == 2 && L.D >= 1);
    L.nparts_f = residual_parts(dim, n);
    L.nparts_r = L.fused_rs1 ? rows_resid_parts(n) : L.nparts_f;
    L.partial = take(sizeof(double) * (size_t)(L.nparts_f > L.nparts_r ? L.nparts_f : L.nparts_r));
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

constexpr int kTimedMax = 64;

struct mg_plan {
    Layout L;
    double p[4];
    hipStream_t stream;
    int device;
    char* ws;
    size_t ws_bytes;
    Ctl* hctl;  // pinned host copy of the control block
    // measurement of one kernel family (mg_timing_enable)
    int tfam = -1;
    int tpend = 0;
    bool tev = false;
    hipEvent_t tbeg[kTimedMax], tend[kTimedMax];
    double tms = 0, tbytes = 0;
    long long tcount = 0;
};

namespace {

template <typename T>
T* at(mg_plan* P, size_t off) { return reinterpret_cast<T*>(P->ws + off); }

void timing_flush(mg_plan* P)
{
    for (int i = 0; i < P->tpend; i++) {
        float ms = 0;
        if (hipEventSynchronize(P->tend[i]) == hipSuccess && hipEventElapsedTime(&ms, P->tbeg[i], P->tend[i]) == hipSuccess)
            P->tms += ms;
    }
    P->tpend = 0;
}

// Brackets one launch with events when its family is the measured one.
struct Timed {
    mg_plan* P;
    bool on;
    Timed(mg_plan* p, int fam, double bytes) : P(p), on(p->tev && p->tfam == fam)
    {
        if (!on) return;
        if (P->tpend == kTimedMax) timing_flush(P);
        (void)hipEventRecord(P->tbeg[P->tpend], P->stream);
        P->tbytes += bytes;
        P->tcount++;
    }
    ~Timed()
    {
        if (on) (void)hipEventRecord(P->tend[P->tpend++], P->stream);
    }
};

// Algorithmic HBM bytes of one launch: every element of an input array the
// launch reads, and every element it writes, counted once.
double bytes_rs2(int diag_in, int m, size_t es)
{
    int M = m / 2;
    if (!diag_in) return (double)es * (sizeA(m) + (double)M * M + (double)(M - 1) * (M - 1));
    return (double)es * (sizeD(m) + (double)(M - 1) * (M - 1));
}
double bytes_jac2(int diag, int m, size_t es)
{
    int M = m / 2;
    if (diag) {
        double pts = (double)M * M + (double)(M - 1) * (M - 1);
        return (double)es * (2 * pts + sizeA(M));
    }
    return (double)es * (2.0 * (m - 1) * (m - 1) + sizeD(m));
}
double bytes_rs3(int coarse_kind, int m, size_t es)
{
    double M = m / 2;
    if (coarse_kind == 1) return (double)es * (sizeG(m) + (double)(m - 1) * (m - 1) * (m - 1) / 2);
    if (coarse_kind == 2) return (double)es * (sizeR(m) + (M - 1) * (M - 1) * (M - 1) + M * M * M);
    return (double)es * (sizeME(m) + sizeMO(m) + (M - 1) * (M - 1) * (M - 1));
}
double bytes_jac3(int kind, int m, size_t es)
{
    double M = m / 2, c = (double)(m - 1) * (m - 1) * (m - 1);
    if (kind == 2) return (double)es * (2 * ((M - 1) * (M - 1) * (M - 1) + M * M * M) + sizeG(m / 2));
    if (kind == 1) return (double)es * (2 * ((M - 1) * (M - 1) * (M - 1) + 3 * M * M * (M - 1)) + sizeME(m) + sizeMO(m));
    return (double)es * (2 * c + sizeR(m));
}
double bytes_residual(int dim, int n, size_t es, bool fused_rs1)
{
    double inter = dim == 2 ? (double)(n - 1) * (n - 1) : (double)(n - 1) * (n - 1) * (n - 1);
    double all = dim == 2 ? (double)sizeA(n) : (double)sizeG(n);
    double b = 8 * all + 8 * inter + es * inter;
    if (fused_rs1) {
        double M = n / 2;
        b += es * (M * M + (M - 1) * (M - 1));  // the level-1 residual it also writes
    }
    return b;
}
double bytes_finest(int dim, int n, size_t es)
{
    double inter = dim == 2 ? (double)(n - 1) * (n - 1) : (double)(n - 1) * (n - 1) * (n - 1);
    double vc = dim == 2 ? (double)sizeD(n) : (double)sizeR(n);
    return es * (inter + vc) + 16 * inter;
}

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
    const size_t es = sizeof(T);
    int last_rs = dc ? dc : D;
    for (int d = L.fused_rs1 ? 2 : 1; d <= last_rs; d++) {
        Timed t(P, MG_K_RESTRICT, bytes_rs2((d - 1) % 2, L.lev[d - 1].m, es));
        if (L.lev[d - 1].m >= kRowsMinSide) launch_rs2_rows<T>((d - 1) % 2, L.lev[d - 1].m, R(d - 1), R(d), ctl, s);
        else launch_rs2<T>((d - 1) % 2, L.lev[d - 1].m, R(d - 1), R(d), ctl, s);
    }
    if (dc) {
        double cb = 0;
        for (int d = dc + 1; d <= D; d++) cb += bytes_rs2((d - 1) % 2, L.lev[d - 1].m, es);
        for (int d = dc; d <= D; d++) cb += bytes_jac2(L.lev[d].kind, L.lev[d].m, es);
        Timed t(P, MG_K_COARSE, cb);
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
        Timed t(P, MG_K_JACOBI, bytes_jac2(L.lev[d].kind, L.lev[d].m, es));
        if (L.lev[d].m >= kRowsMinSide) launch_jac2_rows<T>(L.lev[d].kind, L.lev[d].m, (T)L.lev[d].c, R(d), vc, V(d), ctl, s);
        else launch_jac2<T>(L.lev[d].kind, L.lev[d].m, (T)L.lev[d].c, R(d), vc, V(d), ctl, s);
    }
    const T* v1 = D >= 1 ? V(1) : at<T>(P, L.zero);
    Timed t(P, MG_K_FINEST, bytes_finest(2, L.n, es));
    launch_jac2_finest_rows<T>(L.n, (T)L.lev[0].c, r0, v1, u, ctl, s);
}

template <typename T>
void enqueue_cycle(mg_plan* P, double* u, const Ctl* ctl)
{
    if (P->L.dim == 2) enqueue_cycle_2d<T>(P, u, ctl);
    else enqueue_cycle_3d<T>(P, u, ctl);
}

void enqueue_residual(mg_plan* P, const double* u, const double* f, const Ctl* ctl)
{
    Layout& L = P->L;
    bool dbl = L.prec == MG_FP64;
    double* part = at<double>(P, L.partial);
    Timed t(P, MG_K_RESIDUAL, bytes_residual(L.dim, L.n, dbl ? 8 : 4, L.fused_rs1));
    if (L.fused_rs1) {
        if (dbl) launch_resid_a2d<double>(L.n, u, f, at<double>(P, L.r0), at<double>(P, L.lev[1].r), part, ctl, P->stream);
        else launch_resid_a2d<float>(L.n, u, f, at<float>(P, L.r0), at<float>(P, L.lev[1].r), part, ctl, P->stream);
    } else {
        if (dbl) launch_residual<double>(L.dim, L.n, u, f, at<double>(P, L.r0), part, L.nparts_r, ctl, P->stream);
        else launch_residual<float>(L.dim, L.n, u, f, at<float>(P, L.r0), part, L.nparts_r, ctl, P->stream);
    }
}

// kind 0: norm of f (partials of the sumsq kernel); kind 1: residual norm
void enqueue_finalize(mg_plan* P, int kind, int k, Ctl* ctl)
{
    int np = kind == 0 ? P->L.nparts_f : P->L.nparts_r;
    Timed t(P, MG_K_NORM, 8.0 * np);
    launch_finalize(kind, k, at<double>(P, P->L.partial), np, ctl, P->stream);
}

void enqueue_cycle_any(mg_plan* P, double* u, const Ctl* ctl)
{
    if (P->L.prec == MG_FP64) enqueue_cycle<double>(P, u, ctl);
    else enqueue_cycle<float>(P, u, ctl);
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
    const size_t es = sizeof(T);
    int last_rs = dc ? dc : D;
    for (int d = 1; d <= last_rs; d++) {
        Timed t(P, MG_K_RESTRICT, bytes_rs3(L.lev[d].kind, L.lev[d - 1].m, es));
        launch_rs3<T>(lv(d - 1), lv(d), ctl, s);
    }
    if (dc) {
        double cb = 0;
        for (int d = dc + 1; d <= D; d++) cb += bytes_rs3(L.lev[d].kind, L.lev[d - 1].m, es);
        for (int d = dc; d <= D; d++) cb += bytes_jac3(L.lev[d].kind, L.lev[d].m, es);
        Timed t(P, MG_K_COARSE, cb);
        Coarse3<T> a;
        a.first = dc;
        a.last = D;
        for (int d = dc; d <= D; d++) a.lev[d] = lv(d);
        a.zero = at<T>(P, L.zero);
        launch_coarse3<T>(a, ctl, s);
    }
    for (int d = (dc ? dc - 1 : D); d >= 1; d--) {
        Lev3<T> c = (d == D) ? Lev3<T>{} : lv(d + 1);
        Timed t(P, MG_K_JACOBI, bytes_jac3(L.lev[d].kind, L.lev[d].m, es));
        launch_jac3<T>(lv(d), c, at<T>(P, L.zero), ctl, s);
    }
    Lev3<T> c1 = D >= 1 ? lv(1) : Lev3<T>{};
    Timed t(P, MG_K_FINEST, bytes_finest(3, L.n, es));
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
    if (P->tev) {
        timing_flush(P);
        for (int i = 0; i < kTimedMax; i++) {
            (void)hipEventDestroy(P->tbeg[i]);
            (void)hipEventDestroy(P->tend[i]);
        }
    }
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
        launch_sumsq(L.dim, L.n, f, part, L.nparts_f, ctl, P->stream);
        enqueue_finalize(P, 0, 0, ctl);
    }
    enqueue_residual(P, u, f, ctl);
    if (rel_res_before) enqueue_finalize(P, 1, 0, ctl);
    enqueue_cycle_any(P, u, ctl);
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
    launch_ctl_reset(ctl, 1, max_cycles, rtol, s);
    launch_sumsq(L.dim, L.n, f, part, L.nparts_f, ctl, s);
    enqueue_finalize(P, 0, 0, ctl);
    enqueue_residual(P, u, f, ctl);
    enqueue_finalize(P, 1, 0, ctl);
    size_t head = offsetof(Ctl, rtol);
    // The device takes the decision after every residual evaluation; the
    // host launches the next cycle only once it has seen that the last
    // evaluation did not stop the solve, so no launch is wasted.
    for (int k = 0;; k++) {
        if (hipMemcpyAsync(P->hctl, ctl, head, hipMemcpyDeviceToHost, s) != hipSuccess) return MG_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return MG_ERR_HIP;
        if (P->hctl->done || k >= max_cycles) break;
        enqueue_cycle_any(P, u, ctl);
        enqueue_residual(P, u, f, ctl);
        enqueue_finalize(P, 1, k + 1, ctl);
        int e = last_launch();
        if (e) return e;
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

int mg_timing_enable(mg_plan* P, int family)
{
    if (!P || family < -1 || family >= MG_K_FAMILIES) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (family >= 0 && !P->tev) {
        for (int i = 0; i < kTimedMax; i++)
            if (hipEventCreate(&P->tbeg[i]) != hipSuccess || hipEventCreate(&P->tend[i]) != hipSuccess)
                return MG_ERR_HIP;
        P->tev = true;
    }
    if (P->tev) timing_flush(P);
    P->tfam = family;
    P->tms = P->tbytes = 0;
    P->tcount = 0;
    return MG_OK;
}

int mg_timing_read(mg_plan* P, double* ms, long long* launches, double* bytes)
{
    if (!P) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->tev) timing_flush(P);
    if (ms) *ms = P->tms;
    if (launches) *launches = P->tcount;
    if (bytes) *bytes = P->tbytes;
    P->tms = P->tbytes = 0;
    P->tcount = 0;
    return MG_OK;
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

// Host runtime of the 3D solver (Roberts, Section 3): level plan, workspace
// carving and launch sequencing of one V-cycle: residual on the finest
// green grid, restriction green -> red -> magenta -> blue group by group
// (a group of side 16 .. 64 in one launch), every level of side <= 8 in
// one persistent workgroup, Jacobi back up (magenta-blue, red-magenta,
// green-red; again one launch per group of side 16 .. 64), the finest fused
// with u += v.
#include "dmg_launch.hpp"
#include "dmg_launch3.hpp"
#include "dmg_net.hpp"
#include "dmg_plan3d.hpp"

#include <algorithm>
#include <string.h>
#include <vector>

namespace dmg {

namespace {

constexpr int kCoarseSide3 = 8;  // levels of side <= 8 run in the persistent kernel

template <typename T>
T* at(Plan3& P, size_t off) { return reinterpret_cast<T*>(P.ws + off); }

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
double bytes_resid3(int n, size_t es)
{
    double inter = (double)(n - 1) * (n - 1) * (n - 1);
    return 8 * (double)sizeG(n) + 8 * inter + es * inter;
}
double bytes_finest3(int n, size_t es)
{
    double inter = (double)(n - 1) * (n - 1) * (n - 1);
    return es * (inter + (double)sizeR(n)) + 16 * inter;
}

// A level group (green at depth g > 0, then red, magenta, and the blue =
// green at g+3) runs each way in one launch when its side allows: down when
// the restrictions into g+1 .. g+3 are launched here (g+3 <= last_rs), up
// when the Jacobi steps of g+2 .. g are (g+2 <= first_jac).
bool group_down(const Plan3& P, int g, int last_rs)
{
    return g >= 3 && g % 3 == 0 && g + 3 <= last_rs && group3_ok(P.lev[g].m, false);
}
bool group_up(const Plan3& P, int g, int first_jac)
{
    return g >= 3 && g % 3 == 0 && g + 2 <= first_jac && g + 3 <= P.D && group3_ok(P.lev[g].m, true);
}
// algorithmic bytes: green residual read; red, magenta and blue residuals written
double bytes_down_group3(int m, size_t es)
{
    double M = m / 2, c = (double)(m - 1) * (m - 1) * (m - 1);
    return (double)es * (c + c / 2 + (M - 1) * (M - 1) * (M - 1) + M * M * M + (M - 1) * (M - 1) * (M - 1));
}
// blue correction and the three residuals read; the three corrections written
double bytes_up_group3(int m, size_t es)
{
    double M = m / 2, c = (double)(m - 1) * (m - 1) * (m - 1);
    double mag = (M - 1) * (M - 1) * (M - 1) + M * M * M;
    return (double)es * (sizeG(m / 2) + 2 * (c + c / 2 + mag));
}

template <typename T>
void enqueue_cycle3(Plan3& P, double* u, const Ctl* ctl)
{
    hipStream_t s = P.stream;
    int D = P.D, dc = P.dc;
    const size_t es = sizeof(T);
    T* r0 = at<T>(P, P.r0);
    auto lv = [&](int d) {
        Lev3<T> x;
        const Level3& q = P.lev[d];
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
    for (int d = P.fused_resid ? 2 : 1; d <= last_rs; d++) {   // the fused residual produced level 1
        if (group_down(P, d - 1, last_rs)) {   // the group's three restrictions in one launch
            Timed t(&P.tm, MG_K_RESTRICT, bytes_down_group3(P.lev[d - 1].m, es));
            launch_down_group3<T>(lv(d - 1), lv(d), lv(d + 1), lv(d + 2), ctl, s);
            d += 2;
            continue;
        }
        Timed t(&P.tm, MG_K_RESTRICT, bytes_rs3(P.lev[d].kind, P.lev[d - 1].m, es));
        launch_rs3<T>(lv(d - 1), lv(d), ctl, s);
    }
    if (dc) {
        double cb = 0;
        for (int d = dc + 1; d <= D; d++) cb += bytes_rs3(P.lev[d].kind, P.lev[d - 1].m, es);
        for (int d = dc; d <= D; d++) cb += bytes_jac3(P.lev[d].kind, P.lev[d].m, es);
        Timed t(&P.tm, MG_K_COARSE, cb);
        Coarse3<T> a;
        a.first = dc;
        a.last = D;
        for (int d = dc; d <= D; d++) a.lev[d] = lv(d);
        a.zero = at<T>(P, P.zero);
        if (P.has_net) launch_coarse3_net<T>(a, at<Ctl>(P, P.ctl), at<bf16_t>(P, P.net), s);
        else launch_coarse3<T>(a, ctl, s);
    }
    const int first_jac = dc ? dc - 1 : D;
    for (int d = first_jac; d >= 1; d--) {
        if (d >= 2 && group_up(P, d - 2, first_jac)) {   // magenta d, red d-1, green d-2 in one launch
            Timed t(&P.tm, MG_K_JACOBI, bytes_up_group3(P.lev[d - 2].m, es));
            launch_up_group3<T>(lv(d - 2), lv(d - 1), lv(d), lv(d + 1), ctl, s);
            d -= 2;
            continue;
        }
        Lev3<T> c = (d == D) ? Lev3<T>{} : lv(d + 1);
        Timed t(&P.tm, MG_K_JACOBI, bytes_jac3(P.lev[d].kind, P.lev[d].m, es));
        launch_jac3<T>(lv(d), c, at<T>(P, P.zero), ctl, s);
    }
    Lev3<T> c1 = D >= 1 ? lv(1) : Lev3<T>{};
    Timed t(&P.tm, MG_K_FINEST, bytes_finest3(P.n, es));
    launch_jac3_finest<T>(P.n, (T)P.lev[0].c, r0, D >= 1 ? c1.v : at<T>(P, P.zero), u, ctl, s);
}

void enqueue_cycle_any(Plan3& P, double* u, const Ctl* ctl)
{
    if (P.prec == MG_FP64) enqueue_cycle3<double>(P, u, ctl);
    else enqueue_cycle3<float>(P, u, ctl);
}

void enqueue_residual(Plan3& P, const double* u, const double* f, const Ctl* ctl)
{
    bool dbl = P.prec == MG_FP64;
    double* part = at<double>(P, P.partial);
    size_t es = dbl ? 8 : 4;
    if (P.fused_resid) {
        Timed t(&P.tm, MG_K_RESIDUAL, bytes_resid3(P.n, es) + es * (double)sizeR(P.n) / 2);
        if (dbl) launch_resid3_fused<double>(P.n, u, f, at<double>(P, P.r0), at<double>(P, P.lev[1].r), part, ctl, P.stream, P.rorder);
        else launch_resid3_fused<float>(P.n, u, f, at<float>(P, P.r0), at<float>(P, P.lev[1].r), part, ctl, P.stream, P.rorder);
        return;
    }
    Timed t(&P.tm, MG_K_RESIDUAL, bytes_resid3(P.n, es));
    if (dbl) launch_residual<double>(3, P.n, u, f, at<double>(P, P.r0), part, P.nparts, ctl, P.stream, P.rorder);
    else launch_residual<float>(3, P.n, u, f, at<float>(P, P.r0), part, P.nparts, ctl, P.stream, P.rorder);
}

void enqueue_finalize(Plan3& P, int kind, Ctl* ctl, HostState* host = nullptr)
{
    const int np = kind == 0 ? P.nparts : P.nparts_res;
    Timed t(&P.tm, MG_K_NORM, 8.0 * np);
    launch_finalize(kind, at<double>(P, P.partial), np, ctl, P.stream, host);
}

}  // namespace

int plan3_layout(Plan3& P, int n, int prec, const double* p)
{
    int K = ilog2(n);
    if (K < 1 || K > 11) return MG_ERR_SIZE;
    P.rorder = (prec & MG_ORDER4) ? 4 : 2;
    prec &= ~MG_ORDER4;
    if (prec != MG_FP64 && prec != MG_FP32_REFINED) return MG_ERR_ARG;
    size_t es = prec == MG_FP64 ? sizeof(double) : sizeof(float);
    P.n = n;
    P.prec = prec;
    P.D = 3 * (K - 1);
    if (p)
        for (int i = 0; i < 4; i++) P.p[i] = p[i];
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = alignUp(off + bytes);
        return o;
    };
    P.ctl = take(sizeof(Ctl));
    P.nparts = residual_parts(3, n);
    P.fused_resid = resid3_fused_parts(n) > 0;
    P.nparts_res = P.fused_resid ? resid3_fused_parts(n) : P.nparts;
    P.partial = take(sizeof(double) * (size_t)std::max(P.nparts, P.nparts_res));
    P.zero = take(sizeof(double) * 64);
    P.r0 = take(es * sizeG(n));
    if (P.rorder == 4) P.g = take(sizeof(double) * sizeG(n));
    P.net = take(sizeof(bf16_t) * (size_t)NetGeo<3>::PACK);
    double h = 1.0 / n;
    for (int d = 0; d <= P.D; d++) {
        Level3& v = P.lev[d];
        v.m = n >> (d / 3);
        v.kind = d % 3;
        double sh = (double)(n / v.m) * h;  // sigma * h
        double pm = P.p[0], pr1 = P.p[1], pr2 = P.p[2], pg = P.p[3];
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
    // first depth run by the persistent kernel (0: none), on a green level
    P.dc = 0;
    if (P.D >= 1) {
        for (int d = 1; d <= P.D; d++)
            if (P.lev[d].m <= kCoarseSide3) { P.dc = d; break; }
        while (P.dc > 1 && P.dc % 3 != 0) P.dc--;
        // the persistent kernel stages these levels in LDS (at most 1585 points per kind)
        size_t staged = 0;
        for (int d = P.dc; d <= P.D; d++) {
            const Level3& v = P.lev[d];
            staged += v.kind == 0 ? sizeG(v.m) : v.kind == 1 ? sizeR(v.m) : sizeME(v.m) + sizeMO(v.m);
        }
        if (P.dc && staged > 1585) return MG_ERR_SIZE;
    }
    P.total = off;
    return MG_OK;
}

int plan3_setup(Plan3& P, void* ws, size_t ws_bytes, hipStream_t stream)
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
    // zero the whole workspace once: boundary entries of every level stay 0
    return hip_status(hipMemsetAsync(P.ws, 0, P.total, P.stream));
}

int plan3_bind_static(Plan3& P, void* ws, hipStream_t stream)
{
    if (!ws || ((uintptr_t)ws % kAlign) != 0) return MG_ERR_WS;
    P.ws = (char*)ws;
    P.stream = stream;
    P.tm.stream = stream;
    if (hipGetDevice(&P.device) != hipSuccess) return MG_ERR_HIP;
    // every call starts from a zero workspace (boundary entries of every
    // level read 0; the previous call's contents are gone)
    launch_zero(P.ws, P.total, stream);
    return last_launch();
}

void plan3_destroy(Plan3& P)
{
    P.tm.destroy();
    if (P.live) (void)hipStreamSynchronize(P.stream);
    if (P.hctl) (void)hipHostFree(P.hctl);
    if (P.hstate) (void)hipHostFree(P.hstate);
}

int plan3_vcycle(Plan3& P, double* u, const double* f, double* relres)
{
    Ctl* ctl = at<Ctl>(P, P.ctl);
    double* part = at<double>(P, P.partial);
    if (P.rorder == 4) {   // the kernels read the right-hand side combination made from f
        launch_rhs4_3d(P.n, f, at<double>(P, P.g), P.stream);
        f = at<double>(P, P.g);
    }
    launch_ctl_reset(ctl, 0, 0, 0.0, P.stream, P.has_net ? 1 : 0);
    if (relres) {
        launch_sumsq(3, P.n, f, part, P.nparts, ctl, P.stream);
        enqueue_finalize(P, 0, ctl);
    }
    enqueue_residual(P, u, f, ctl);
    if (relres) enqueue_finalize(P, 1, ctl);
    enqueue_cycle_any(P, u, ctl);
    int e = last_launch();
    if (e) return e;
    if (relres && !P.hctl) {   // bound without pinned memory: one double straight into the caller's
        if (hipMemcpyAsync(relres, &ctl->last, sizeof(double), hipMemcpyDeviceToHost, P.stream) != hipSuccess ||
            hipStreamSynchronize(P.stream) != hipSuccess)
            return MG_ERR_HIP;
        return MG_OK;
    }
    if (relres) {
        if (hipMemcpyAsync(P.hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, P.stream) != hipSuccess) return MG_ERR_HIP;
        if (hipStreamSynchronize(P.stream) != hipSuccess) return MG_ERR_HIP;
        *relres = P.hctl->last;
    }
    return MG_OK;
}

int plan3_solve(Plan3& P, double* u, const double* f, double rtol, int max_cycles, int* cycles_out, double* rel_res_out,
                double* history)
{
    Ctl* ctl = at<Ctl>(P, P.ctl);
    double* part = at<double>(P, P.partial);
    hipStream_t s = P.stream;
    if (P.rorder == 4) {
        launch_rhs4_3d(P.n, f, at<double>(P, P.g), s);
        f = at<double>(P, P.g);
    }
    P.hstate->k = 0;   // the pinned evaluation count the loop polls, fresh before any kernel
    P.hstate->done = 0;
    launch_ctl_reset(ctl, 1, max_cycles, rtol, s, P.has_net ? 1 : 0);
    launch_sumsq(3, P.n, f, part, P.nparts, ctl, s);
    enqueue_finalize(P, 0, ctl);
    enqueue_residual(P, u, f, ctl);
    enqueue_finalize(P, 1, ctl, P.hstate);
    // The device decides after every residual evaluation (later launches of
    // a finished solve return at once) and its finalize kernel writes the
    // decision into pinned host memory.  While the host waits for what
    // iteration it decided, iteration it+1 is already queued, so the GPU does
    // not wait for the host between cycles -- unless the residual trend says
    // iteration it is probably the last: then the host waits first, rather
    // than queue a whole gated iteration that would only return.  (The host
    // may see the next evaluation's state: done never reverts, and that
    // evaluation is already queued, so stopping on it is right.)
    auto launch = [&](int it1) -> int {   // iteration it1: cycle, residual evaluation it1
        enqueue_cycle_any(P, u, ctl);
        enqueue_residual(P, u, f, ctl);
        enqueue_finalize(P, 1, ctl, P.hstate);
        (void)it1;
        return last_launch();
    };
    double rr1 = -1, rr2 = -1;   // relative residuals of evaluations it-1, it-2
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
    int cyc = H.done ? H.cycles : max_cycles;
    if (cycles_out) *cycles_out = cyc;
    if (rel_res_out) *rel_res_out = H.last;
    if (history)
        for (int k = 0; k <= cyc; k++) history[k] = H.hist[k];
    return H.done ? H.status : MG_ERR_NOT_CONVERGED;
}

int plan3_level_get(Plan3& P, int depth, int which, double* dst)
{
    if (depth < 0 || depth > P.D || (which != 0 && which != 1) || (which == 1 && depth == 0)) return MG_ERR_ARG;
    const Level3& q = P.lev[depth];
    size_t src = which == 0 ? (depth == 0 ? P.r0 : q.r) : q.v;
    size_t src2 = which == 0 ? q.r2 : q.v2;
    if (P.prec == MG_FP64)
        launch_level_get3<double>(q.kind, q.m, at<double>(P, src), q.kind == 2 ? at<double>(P, src2) : nullptr, dst,
                                  P.stream);
    else
        launch_level_get3<float>(q.kind, q.m, at<float>(P, src), q.kind == 2 ? at<float>(P, src2) : nullptr, dst,
                                 P.stream);
    return last_launch();
}

// ------------------------------------------------ learned coarse correction

int plan3_set_net(Plan3& P, const float* w, int cut_level)
{
    if (cut_level != kNetCut) return MG_ERR_ARG;
    if (w) {
        const int nw = NetGeo<3>::NW;
        std::vector<float> wm(w, w + nw);
        for (int i = 0; i < nw; i++) {   // the padded channels are not parameters
            int layer = (i >> 8) / NetGeo<3>::T, ci = (i >> 4) & 15, co = i & 15;
            if ((layer == 0 && ci) || (layer == kNetLayers - 1 && co)) wm[i] = 0.f;
        }
        std::vector<bf16_t> wf(NetGeo<3>::PACK);
        net_pack_host(3, wm.data(), wf.data(), nullptr);
        if (hipStreamSynchronize(P.stream) != hipSuccess ||
            hipMemcpy(P.ws + P.net, wf.data(), sizeof(bf16_t) * wf.size(), hipMemcpyHostToDevice) != hipSuccess)
            return MG_ERR_HIP;
    }
    P.has_net = w != nullptr;
    return MG_OK;
}

int plan3_net_stats(Plan3& P, int* net_cycles, int* fell_back, double* q_net, double* q_plain)
{
    if (hipMemcpyAsync(P.hctl, at<Ctl>(P, P.ctl), kCtlHead, hipMemcpyDeviceToHost, P.stream) != hipSuccess ||
        hipStreamSynchronize(P.stream) != hipSuccess)
        return MG_ERR_HIP;
    const Ctl& c = *P.hctl;
    if (net_cycles) *net_cycles = c.net_used;
    if (fell_back) *fell_back = c.net_off;
    if (q_net) *q_net = c.q_net;
    if (q_plain) *q_plain = c.theta;
    return MG_OK;
}

// aligned level `level` (0 = the coarsest) of the 3D hierarchy: depth D - level
int plan3_coarse_export(Plan3& P, int level, double* dst)
{
    if (level < 0 || level > P.D || !dst) return MG_ERR_ARG;
    return plan3_level_get(P, P.D - level, 0, dst);
}

}  // namespace dmg

// Host runtime of the 2D solver (Roberts, Section 2): a plan for a batch of
// independent problems (a single problem is a batch of one).
//
// Levels are aligned from the coarsest grid: at aligned level lambda every
// problem's grid has side 2^(1+ceil(lambda/2)) (axis grid for even lambda,
// diagonal grid for odd) and the same Jacobi coefficient, so one launch per
// level serves every problem that has that level.  The launches read their
// arrays from item tables in the workspace; a per-problem done flag makes a
// converged problem's items return at once.
//
// One outer iteration (cycle + next residual + stopping decision) is captured
// once in a hipGraph and replayed; its kernel arguments never change (the u and
// f pointers are read from a table updated before each solve).  The host
// launches iteration k+1 before it reads the number of active problems left
// by iteration k, so the GPU never waits for the host round trip; the one
// iteration launched after the last problem stops runs as gated no-ops.
#include "dmg_b2d.hpp"
#include "dmg_launch.hpp"
#include "dmg_host.hpp"
#include "dmg_net.hpp"
#include "dmg_plan2d.hpp"

#include <algorithm>
#include <chrono>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

namespace dmg {

namespace {

constexpr int kCoarseSide2 = 64;  // aligned levels of side <= this run in the coarse kernel
constexpr int kMaxSide2 = 1 << 15;

int side_of(int lam) { return 1 << (1 + (lam + 1) / 2); }

// does a problem (finest level D, coarse top `top`) run the Jacobi of level
// lam as a launch of its own
bool jac_one(const Plan2& P, int lam, int D, int top)
{
    return D >= 1 && lam >= top + 1 && lam <= D - 1 - (int)fin_fused(D, P.lamc) && !pair_level(lam, D, P.pairs) &&
           !pair_level(lam + 1, D, P.pairs);
}

// ... and the restriction into level lam
bool rs_one(const Plan2& P, int lam, int D, int top)
{
    return D >= 1 && lam >= top && lam <= D - 2 - (int)fin_fused(D, P.lamc) && !pair_level(lam + 1, D, P.pairs) &&
           !pair_level(lam + 2, D, P.pairs);
}

}  // namespace

int plan2_layout(Plan2& P, int nprob, const int* n, int prec, double p, bool allow_oop)
{
    if (nprob < 1 || !n) return MG_ERR_ARG;
    P.rorder = (prec & MG_ORDER4) ? 4 : 2;
    prec &= ~MG_ORDER4;
    if (prec != MG_FP64 && prec != MG_FP32_REFINED) return MG_ERR_ARG;
    if (P.rorder == 4 && nprob != 1) return MG_ERR_ARG;
    P.nprob = nprob;
    P.prec = prec;
    P.p = p;
    P.n.assign(n, n + nprob);
    P.D.resize(nprob);
    P.Dmax = 0;
    for (int i = 0; i < nprob; i++) {
        int K = ilog2(n[i]);
        if (K < 1 || n[i] > kMaxSide2) return MG_ERR_SIZE;
        P.D[i] = 2 * (K - 1);
        P.Dmax = std::max(P.Dmax, P.D[i]);
    }
    P.lamc = 0;
    while (side_of(P.lamc + 1) <= kCoarseSide2) P.lamc++;
    P.oop = allow_oop && nprob == 1 && (prec == MG_FP64 || prec == MG_FP32_REFINED) && P.rorder == 2 && n[0] >= 8 &&
            fin_fused(P.D[0], P.lamc);
    P.r0_stale = false;
    size_t es = prec == MG_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = alignUp(off + bytes);
        return o;
    };
    // size classes (distinct n, ascending); fin-table slots grouped by class
    std::vector<int> ord(nprob);
    for (int i = 0; i < nprob; i++) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return n[a] < n[b]; });
    P.order = ord;
    P.cls_n.clear(); P.cls_first.clear(); P.cls_count.clear(); P.nparts.clear();
    for (int s = 0; s < nprob; s++) {
        int nn = n[ord[s]];
        if (P.cls_n.empty() || P.cls_n.back() != nn) {
            P.cls_n.push_back(nn);
            P.cls_first.push_back(s);
            P.cls_count.push_back(0);
            P.nparts.push_back(b_resid_parts(nn));
        }
        P.cls_count.back()++;
    }
    P.off_ctl = take(sizeof(Ctl) * (size_t)nprob);
    P.off_nactive = take(sizeof(int) * 4);
    P.off_zero = take(sizeof(double) * 64);
    P.off_fin = take(sizeof(Fin2<double>) * (size_t)nprob);
    P.off_coarse = take(sizeof(Coarse2B<double>) * (size_t)nprob);
    P.off_net = take(sizeof(bf16_t) * (size_t)NetGeo<2>::PACK);
    P.off_lg_item = take(2 * sizeof(Item2<double>));
    P.off_rs_items.assign(P.Dmax + 1, 0);
    P.off_jac_items.assign(P.Dmax + 1, 0);
    P.n_rs_items.assign(P.Dmax + 1, 0);
    P.n_jac_items.assign(P.Dmax + 1, 0);
    P.pairs = nprob == 1;
    P.off_pair_items.assign(P.Dmax + 1, 0);
    P.n_pair_items.assign(P.Dmax + 1, 0);
    P.off_rsp_items.assign(P.Dmax + 1, 0);
    P.n_rsp_items.assign(P.Dmax + 1, 0);
    for (int lam = 0; lam <= P.Dmax; lam++) {
        for (int i = 0; i < nprob; i++) {
            int Dp = P.D[i];
            int top = std::min(P.lamc, Dp - 1);
            // restriction into lam (into D-2 it runs in the residual kernel when
            // fused; pair levels restrict two levels at once)
            if (rs_one(P, lam, Dp, top)) P.n_rs_items[lam]++;
            if (pair_level(lam, Dp, P.pairs)) P.n_rsp_items[lam]++;
            // Jacobi at lam (the first diagonal level's runs in the finest kernel
            // when fused; pair levels run together)
            if (jac_one(P, lam, Dp, top)) P.n_jac_items[lam]++;
            if (pair_level(lam, Dp, P.pairs)) P.n_pair_items[lam]++;
        }
        if (P.n_pair_items[lam]) P.off_pair_items[lam] = take(sizeof(JPair2<double>) * (size_t)P.n_pair_items[lam]);
        if (P.n_rsp_items[lam]) P.off_rsp_items[lam] = take(sizeof(RsPair2<double>) * (size_t)P.n_rsp_items[lam]);
        if (P.n_rs_items[lam]) P.off_rs_items[lam] = take(sizeof(Item2<double>) * (size_t)P.n_rs_items[lam]);
        if (P.n_jac_items[lam]) P.off_jac_items[lam] = take(sizeof(Item2<double>) * (size_t)P.n_jac_items[lam]);
    }
    P.n_coarse_items = 0;
    for (int i = 0; i < nprob; i++)
        if (P.D[i] >= 1) P.n_coarse_items++;
    P.off_r0.resize(nprob);
    P.off_part.resize(nprob);
    P.off_partf.resize(nprob);
    P.off_r.assign(nprob, {});
    P.off_v.assign(nprob, {});
    for (int s = 0; s < nprob; s++) {
        int i = ord[s];
        int m = n[i];
        size_t cnt = sizeA(m);
        P.off_r0[i] = take((P.oop ? sizeof(double) : es) * cnt);   // out of place: the second iterate
        int cls = (int)(std::lower_bound(P.cls_n.begin(), P.cls_n.end(), m) - P.cls_n.begin());
        P.off_part[i] = take(sizeof(double) * (size_t)P.nparts[cls]);
        P.off_partf[i] = take(sizeof(double) * (size_t)P.nparts[cls]);
        P.off_r[i].assign(std::max(P.D[i], 1), 0);
        P.off_v[i].assign(std::max(P.D[i], 1), 0);
        for (int lam = P.D[i] - 1; lam >= 0; lam--) {
            int ms = side_of(lam);
            size_t c = (lam & 1) ? sizeD(ms) : sizeA(ms);
            P.off_r[i][lam] = take(es * c);
            P.off_v[i][lam] = take(es * c);
        }
    }
    if (P.rorder == 4) P.off_g = take(sizeof(double) * sizeA(n[0]));
    P.rows_rs.assign(P.Dmax + 1, 0);
    P.rows_jac.assign(P.Dmax + 1, 0);
    for (int lam = 0; lam <= P.Dmax; lam++) {
        // restriction into lam reads level lam+1
        int mf = side_of(lam + 1);
        P.rows_rs[lam] = b_default_rows(((lam + 1) & 1) ? 1 : 0, mf);
        P.rows_jac[lam] = b_default_rows((lam & 1) ? 2 : 3, side_of(lam));
    }
    P.total = off;
    return MG_OK;
}

namespace {

template <typename T>
T* at(Plan2& P, size_t off) { return reinterpret_cast<T*>(P.ws + off); }

double coef(const Plan2& P, int lam)
{
    double sh = 1.0 / side_of(lam);   // sigma * h
    return (lam & 1) ? 2 * P.p * sh * sh : P.p * sh * sh;
}

// host bytes into the workspace at offset off: a synchronous copy, or (plans
// bound without allocation) into a host image of the table region that
// plan2_bind_static then writes with a few stream-ordered kernels
int put(Plan2& P, size_t off, const void* src, size_t bytes)
{
    if (P.stat) {
        if (bytes % 4) return MG_ERR_ARG;
        if (P.stage.size() < off + bytes) P.stage.resize(off + bytes, 0);
        memcpy(P.stage.data() + off, src, bytes);
        P.stage_lo = std::min(P.stage_lo, off);
        return MG_OK;
    }
    return hip_status(hipMemcpy(P.ws + off, src, bytes, hipMemcpyHostToDevice));
}

// the finest item of problem i (u and f are filled per call)
template <typename T>
Fin2<T> fin_item(Plan2& P, int i)
{
    T* zero = at<T>(P, P.off_zero);
    Fin2<T> x;
    memset(&x, 0, sizeof(x));
    x.r0 = at<T>(P, P.off_r0[i]);
    x.r1 = P.D[i] >= 1 ? at<T>(P, P.off_r[i][P.D[i] - 1]) : nullptr;
    x.v1 = P.D[i] >= 1 ? at<T>(P, P.off_v[i][P.D[i] - 1]) : zero;
    x.v2 = P.D[i] >= 2 ? at<T>(P, P.off_v[i][P.D[i] - 2]) : zero;
    x.r2 = fin_fused(P.D[i], P.lamc) ? at<T>(P, P.off_r[i][P.D[i] - 2]) : nullptr;
    x.part = at<double>(P, P.off_part[i]);
    x.partf = at<double>(P, P.off_partf[i]);
    x.ub = P.oop ? at<double>(P, P.off_r0[i]) : nullptr;
    x.prob = i;
    return x;
}

// host images of the item tables (pointers into the workspace)
template <typename T>
int write_tables(Plan2& P)
{
    std::vector<Item2<T>> items;
    T* zero = at<T>(P, P.off_zero);
    for (int lam = 0; lam <= P.Dmax; lam++) {
        items.clear();
        for (int i = 0; i < P.nprob; i++) {
            int Dp = P.D[i];
            int top = std::min(P.lamc, Dp - 1);
            if (rs_one(P, lam, Dp, top))
                items.push_back(Item2<T>{at<T>(P, P.off_r[i][lam]), at<T>(P, P.off_v[i][lam]),
                                         at<T>(P, P.off_r[i][lam + 1]), i, 0});
        }
        if (!items.empty() && put(P, P.off_rs_items[lam], items.data(), items.size() * sizeof(Item2<T>)))
            return MG_ERR_HIP;
        items.clear();
        for (int i = 0; i < P.nprob; i++) {
            int Dp = P.D[i];
            int top = std::min(P.lamc, Dp - 1);
            if (jac_one(P, lam, Dp, top))
                items.push_back(Item2<T>{at<T>(P, P.off_r[i][lam]), at<T>(P, P.off_v[i][lam]),
                                         lam >= 1 ? at<T>(P, P.off_v[i][lam - 1]) : zero, i, 0});
        }
        if (!items.empty() && put(P, P.off_jac_items[lam], items.data(), items.size() * sizeof(Item2<T>)))
            return MG_ERR_HIP;
        std::vector<RsPair2<T>> rsp;
        for (int i = 0; i < P.nprob; i++)
            if (pair_level(lam, P.D[i], P.pairs))
                rsp.push_back(RsPair2<T>{at<T>(P, P.off_r[i][lam]), at<T>(P, P.off_r[i][lam - 2]), i, 0});
        if (!rsp.empty() && put(P, P.off_rsp_items[lam], rsp.data(), rsp.size() * sizeof(RsPair2<T>)))
            return MG_ERR_HIP;
        std::vector<JPair2<T>> pairs;
        for (int i = 0; i < P.nprob; i++)
            if (pair_level(lam, P.D[i], P.pairs))
                pairs.push_back(JPair2<T>{at<T>(P, P.off_r[i][lam]), at<T>(P, P.off_v[i][lam - 2]),
                                          at<T>(P, P.off_v[i][lam]), i, 0});
        if (!pairs.empty() && put(P, P.off_pair_items[lam], pairs.data(), pairs.size() * sizeof(JPair2<T>)))
            return MG_ERR_HIP;
    }
    std::vector<Coarse2B<T>> co;
    for (int i = 0; i < P.nprob; i++) {
        if (P.D[i] < 1) continue;
        Coarse2B<T> c;
        memset(&c, 0, sizeof(c));
        c.top = std::min(P.lamc, P.D[i] - 1);
        c.prob = i;
        for (int lam = 0; lam <= c.top; lam++) {
            c.r[lam] = at<T>(P, P.off_r[i][lam]);
            c.v[lam] = at<T>(P, P.off_v[i][lam]);
        }
        co.push_back(c);
    }
    if (!co.empty() && put(P, P.off_coarse, co.data(), co.size() * sizeof(Coarse2B<T>)))
        return MG_ERR_HIP;
    // finest items (u, f filled per call), in class order; a statically
    // bound plan writes its one item with u and f on every call instead
    if (P.hfin) {
        Fin2<T>* hf = reinterpret_cast<Fin2<T>*>(P.hfin);
        for (int s = 0; s < P.nprob; s++) hf[s] = fin_item<T>(P, P.order[s]);
    }
    return MG_OK;
}

template <typename T>
const Fin2<T>* fin_items(Plan2& P, int cls) { return at<Fin2<T>>(P, P.off_fin) + P.cls_first[cls]; }

// small_only: only the size classes whose residual kernel does not sum f^2
// itself (n < 4; see enq_resid)
template <typename T>
void enq_norm_f(Plan2& P, Ctl* ctls, int* nact, bool small_only = false)
{
    for (size_t c = 0; c < P.cls_n.size(); c++) {
        if (small_only && P.cls_n[c] >= 4) continue;
        launch_b_sumsq<T>(P.cls_n[c], fin_items<T>(P, (int)c), P.cls_count[c], ctls, P.stream);
        launch_b_finalize<T>(0, fin_items<T>(P, (int)c), P.cls_count[c], P.nparts[c], ctls, nact, P.stream);
    }
}

// fused (n >= 8): the restriction onto the axis level below the first
// diagonal level ((n/2 - 1)^2 interior points) is written instead of the
// diagonal level itself (which the finest Jacobi restricts again)
// oop: the finest residual is not stored
double bytes_resid(int n, size_t es, bool fused, bool oop = false)
{
    double inter = (double)(n - 1) * (n - 1), M = n / 2;
    const bool fz = fused && n >= 8;
    return 8 * (double)sizeA(n) + 8 * inter + (oop ? 0 : es * inter) +
           (n >= 4 && !fz ? es * (M * M + (M - 1) * (M - 1)) : 0) + (fz ? es * (M - 1) * (M - 1) : 0);
}
// fused: the correction of the level below the first diagonal level (a
// quarter of the points) replaces the read of the diagonal level's correction
// oop: f (8 bytes) is read instead of the stored residual
double bytes_finest(int n, size_t es, bool fused, bool oop = false)
{
    double inter = (double)(n - 1) * (n - 1), M = n / 2;
    double lev = fused ? (M + 1) * (M + 1) : (double)sizeD(n);
    return (oop ? 8 : es) * inter + es * lev + 16 * inter;
}
double bytes_rs(int diag_in, int m, size_t es)
{
    double M = m / 2;
    if (!diag_in) return es * ((double)sizeA(m) + M * M + (M - 1) * (M - 1));
    return es * ((double)sizeD(m) + (M - 1) * (M - 1));
}
double bytes_jac(int diag, int m, size_t es)
{
    double M = m / 2;
    if (diag) return es * (2 * (M * M + (M - 1) * (M - 1)) + (double)sizeA(m / 2));
    return es * (2.0 * (m - 1) * (m - 1) + (double)sizeD(m));
}

// withf: the first evaluation of a solve: the residual kernel of every size
// class with n >= 4 also sums f^2, so that the norm of f needs no pass of its
// own (the others have theirs from enq_norm_f(small_only))
// oop: the out-of-place solve step (P.oop)
// formed: the finest kernel of the cycle has formed the residual already
// (kb_finest_res); only the stopping decision is left
template <typename T>
void enq_resid(Plan2& P, Ctl* ctls, int* nact, bool withf_all = false, bool oop = false, bool formed = false)
{
    size_t es = sizeof(T);
    for (size_t c = 0; c < P.cls_n.size(); c++) {
        const bool withf = withf_all && P.cls_n[c] >= 4;
        if (!formed) {
            const int n = P.cls_n[c];
            const bool fz = fin_fused(2 * (ilog2(n) - 1), P.lamc);
            Timed t(&P.tm, MG_K_RESIDUAL, bytes_resid(n, es, fz, oop) * P.cls_count[c], true);
            launch_b_resid<T>(n, fz ? 1 : 0, P.rorder, fin_items<T>(P, (int)c), P.cls_count[c], ctls, P.stream,
                              withf ? 1 : 0, oop ? 1 : 0);
        }
        Timed t(&P.tm, MG_K_NORM, 8.0 * P.nparts[c] * P.cls_count[c] * (withf ? 2 : 1));
        launch_b_finalize<T>(withf ? 2 : 1, fin_items<T>(P, (int)c), P.cls_count[c], P.nparts[c], ctls, nact,
                             P.stream, P.nprob == 1 && !P.stat ? P.hctl : nullptr);
    }
}


// A single problem whose aligned levels kMidTop .. kMidLow (sides 256 .. 64)
// all run one thread per point, with the coarse kernel starting at kMidLow:
// the fused mid-level kernels replace those eight launches.
bool use_mid(const Plan2& P)
{
    if (P.nprob != 1 || P.D[0] < kMidTop + 2 || P.lamc != kMidLow) return false;
    for (int lam = kMidLow; lam < kMidTop; lam++)
        if (P.n_rs_items[lam] != 1 || P.rows_rs[lam] != 0) return false;
    for (int lam = kMidLow + 1; lam <= kMidTop; lam++)
        if (P.n_jac_items[lam] != 1 || P.rows_jac[lam] != 0) return false;
    return true;
}

// res (with oop): the finest kernel also forms the next evaluation's residual
// where its grid allows (kb_finest_res); returns whether it did
template <typename T>
bool enq_cycle(Plan2& P, Ctl* ctls, bool oop = false, bool res = false)
{
    size_t es = sizeof(T);
    const bool mid = use_mid(P);
    auto R = [&](int lam) { return at<T>(P, P.off_r[0][lam]); };
    auto V = [&](int lam) { return at<T>(P, P.off_v[0][lam]); };
    for (int lam = P.Dmax - 2; lam >= 0; lam--) {
        if (int kp = lam + 1 <= P.Dmax ? P.n_rsp_items[lam + 1] : 0) {   // into lam and lam-1
            const int m = side_of(lam + 1);
            const double M = m / 2;
            Timed t(&P.tm, MG_K_RESTRICT, es * ((double)sizeA(m) + (M - 1) * (M - 1)) * kp);
            launch_b_rs_pair<T>(m, at<RsPair2<T>>(P, P.off_rsp_items[lam + 1]), kp, ctls, P.stream);
        }
        int k = P.n_rs_items[lam];
        if (!k) continue;
        if (mid && lam >= kMidLow && lam < kMidTop) {
            if (lam == kMidTop - 1) {
                double b = 0;
                for (int l = kMidLow; l < kMidTop; l++) b += bytes_rs((l + 1) & 1, side_of(l + 1), es);
                for (int l = kMidCoarseTop; l < kMidLow; l++) b += bytes_rs((l + 1) & 1, side_of(l + 1), es);
                Timed t(&P.tm, MG_K_RESTRICT, b);
                T* r[6] = {R(8), R(9), R(10), R(11), R(12), R(13)};
                launch_b_mid_down<T>(R(14), r, ctls, P.stream);
            }
            continue;
        }
        int diag_in = (lam + 1) & 1;
        Timed t(&P.tm, MG_K_RESTRICT, bytes_rs(diag_in, side_of(lam + 1), es) * k);
        launch_b_restrict<T>(diag_in, side_of(lam + 1), P.rows_rs[lam], at<Item2<T>>(P, P.off_rs_items[lam]), k, ctls,
                             P.stream);
    }
    if (P.n_coarse_items) {
        LevInfo<T> lev[kCoarseLevels];
        double cb = 0;
        for (int lam = 0; lam < kCoarseLevels; lam++) {
            lev[lam].m = side_of(lam);
            lev[lam].diag = lam & 1;
            lev[lam].c = (T)coef(P, lam);
            const int ctop = mid ? kMidCoarseTop : P.lamc;
            if (lam <= ctop) {
                cb += bytes_jac(lam & 1, side_of(lam), es);
                if (lam < ctop) cb += bytes_rs((lam + 1) & 1, side_of(lam + 1), es);
            }
        }
        Timed t(&P.tm, MG_K_COARSE, cb * P.n_coarse_items);
        const int cap = mid ? kMidCoarseTop : kCoarseLevels;
        if (P.has_net)
            launch_b_coarse_net<T>(lev, at<Coarse2B<T>>(P, P.off_coarse), P.n_coarse_items, at<T>(P, P.off_zero), ctls,
                                   at<bf16_t>(P, P.off_net), P.stream, cap);
        else
            launch_b_coarse<T>(lev, at<Coarse2B<T>>(P, P.off_coarse), P.n_coarse_items, at<T>(P, P.off_zero), ctls,
                               P.stream, cap);
    }
    for (int lam = 0; lam <= P.Dmax; lam++) {
        if (int kp = P.n_pair_items[lam]) {
            const int m = side_of(lam);
            const double M = m / 2;
            // r of the axis level, v of the level below the pair, v written
            const double b = es * (2.0 * (double)sizeA(m) + (M + 1) * (M + 1));
            Timed t(&P.tm, MG_K_JACOBI, b * kp);
            launch_b_jac_pair<T>(m, (T)coef(P, lam), (T)coef(P, lam - 1), at<JPair2<T>>(P, P.off_pair_items[lam]), kp,
                                 ctls, P.stream);
        }
        int k = P.n_jac_items[lam];
        if (!k) continue;
        if (mid && lam > kMidLow && lam <= kMidTop) {
            if (lam == kMidLow + 1) {
                double b = 0;
                for (int l = kMidCoarseTop + 1; l <= kMidTop; l++) b += bytes_jac(l & 1, side_of(l), es);
                Timed t(&P.tm, MG_K_JACOBI, b);
                const T* r[6] = {R(9), R(10), R(11), R(12), R(13), R(14)};
                T* v[6] = {V(9), V(10), V(11), V(12), V(13), V(14)};
                T c[6];
                for (int k = 0; k < 6; k++) c[k] = (T)coef(P, 9 + k);
                launch_b_mid_up<T>(V(8), r, v, c, ctls, P.stream);
            }
            continue;
        }
        Timed t(&P.tm, MG_K_JACOBI, bytes_jac(lam & 1, side_of(lam), es) * k);
        launch_b_jacobi<T>(lam & 1, side_of(lam), P.rows_jac[lam], (T)coef(P, lam), at<Item2<T>>(P, P.off_jac_items[lam]),
                           k, ctls, P.stream);
    }
    bool formed = false;
    for (size_t c = 0; c < P.cls_n.size(); c++) {
        int n = P.cls_n[c];
        const int D = 2 * (ilog2(n) - 1);
        const bool fz = fin_fused(D, P.lamc);
        double sh = 1.0 / n;
        if (res && oop && fz && P.cls_count[c] == 1 && b_finest_res_fits<T>(n, P.nparts[c])) {
            const double M = n / 2;
            Timed t(&P.tm, MG_K_FINEST, bytes_finest(n, es, fz, oop) + es * (M - 1) * (M - 1), true);
            launch_b_finest_res<T>(n, (T)(P.p * sh * sh), (T)coef(P, D - 1), fin_items<T>(P, (int)c), ctls,
                                   P.nparts[c], P.stream);
            formed = true;
            continue;
        }
        Timed t(&P.tm, MG_K_FINEST, bytes_finest(n, es, fz, oop) * P.cls_count[c], true);
        launch_b_finest<T>(n, (T)(P.p * sh * sh), (T)(fz ? coef(P, D - 1) : 0.0), fz ? 1 : 0, fin_items<T>(P, (int)c),
                           P.cls_count[c], ctls, P.stream, oop ? 1 : 0);
    }
    return formed;
}

// one outer iteration of a solve: cycle, the next residual, the stopping decision
void enq_iteration(Plan2& P)
{
    Ctl* ctls = at<Ctl>(P, P.off_ctl);
    int* nact = at<int>(P, P.off_nactive);
    if (P.prec == MG_FP64) {
        const bool formed = enq_cycle<double>(P, ctls, P.oop, P.res);
        enq_resid<double>(P, ctls, nact, false, P.oop, formed);
    } else {
        const bool formed = enq_cycle<float>(P, ctls, P.oop, P.res);
        enq_resid<float>(P, ctls, nact, false, P.oop, formed);
    }
}

int build_graph(Plan2& P)
{
    if (P.gready) return MG_OK;
    if (!P.cap && hipStreamCreateWithFlags(&P.cap, hipStreamNonBlocking) != hipSuccess) return MG_ERR_HIP;
    hipStream_t keep = P.stream;
    P.stream = P.cap;
    if (hipStreamBeginCapture(P.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) { P.stream = keep; return MG_ERR_HIP; }
    enq_iteration(P);
    hipGraph_t g;
    hipError_t e = hipStreamEndCapture(P.cap, &g);
    P.stream = keep;
    if (e != hipSuccess) return MG_ERR_HIP;
    e = hipGraphInstantiate(&P.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return MG_ERR_HIP;
    P.gready = true;
    return MG_OK;
}

int run_iteration(Plan2& P)
{
    // graphs replay the captured launches; with timing on, launch eagerly so
    // the events bracket each kernel
    if (P.use_graph && P.tm.fam < 0) {
        int e = build_graph(P);
        if (e) return e;
        return hip_status(hipGraphLaunch(P.gexec, P.stream));
    }
    enq_iteration(P);
    return last_launch();
}

// Point the finest-item table at this call's u and f.  The pinned host image
// is only rewritten after the previous upload from it has completed, and only
// uploaded when a pointer changed.
int bind_uf(Plan2& P, double* const* u, const double* const* f)
{
    if (P.stat) {   // one problem: its item, with this call's u and f, written in stream order
        const double* f0 = P.rorder == 4 ? at<double>(P, P.off_g) : f[0];
        if (P.prec == MG_FP64) {
            Fin2<double> x = fin_item<double>(P, 0);
            x.u = u[0];
            x.f = f0;
            launch_put_bytes(P.ws + P.off_fin, &x, sizeof(x), P.stream);
        } else {
            Fin2<float> x = fin_item<float>(P, 0);
            x.u = u[0];
            x.f = f0;
            launch_put_bytes(P.ws + P.off_fin, &x, sizeof(x), P.stream);
        }
        return last_launch();
    }
    bool same = P.fin_valid;
    for (int i = 0; same && i < P.nprob; i++) same = P.last_u[i] == u[i] && P.last_f[i] == f[i];
    if (same) return MG_OK;
    if (P.fin_valid && hipEventSynchronize(P.evu) != hipSuccess) return MG_ERR_HIP;
    for (int s = 0; s < P.nprob; s++) {
        int i = P.order[s];
        // order 4: the kernels read the right-hand side combination made from f
        const double* fi = P.rorder == 4 ? at<double>(P, P.off_g) : f[i];
        if (P.prec == MG_FP64) {
            Fin2<double>* hf = reinterpret_cast<Fin2<double>*>(P.hfin);
            hf[s].u = u[i];
            hf[s].f = fi;
        } else {
            Fin2<float>* hf = reinterpret_cast<Fin2<float>*>(P.hfin);
            hf[s].u = u[i];
            hf[s].f = fi;
        }
    }
    size_t bytes = (P.prec == MG_FP64 ? sizeof(Fin2<double>) : sizeof(Fin2<float>)) * (size_t)P.nprob;
    if (hipMemcpyAsync(P.ws + P.off_fin, P.hfin, bytes, hipMemcpyHostToDevice, P.stream) != hipSuccess) return MG_ERR_HIP;
    if (hipEventRecord(P.evu, P.stream) != hipSuccess) return MG_ERR_HIP;
    P.last_u.assign(u, u + P.nprob);
    P.last_f.assign(f, f + P.nprob);
    P.fin_valid = true;
    return MG_OK;
}

}  // namespace

int plan2_setup(Plan2& P, void* ws, size_t ws_bytes, hipStream_t stream)
{
    if (!ws || ((uintptr_t)ws % kAlign) != 0 || ws_bytes < P.total) return MG_ERR_WS;
    P.ws = (char*)ws;
    P.stream = stream;
    P.tm.stream = stream;
    if (hipGetDevice(&P.device) != hipSuccess) return MG_ERR_HIP;
    size_t fb = sizeof(Fin2<double>) * (size_t)P.nprob;
    if (hipHostMalloc(&P.hfin, fb, hipHostMallocDefault) != hipSuccess) return MG_ERR_HIP;
    // coherent: the finalize kernel's writes reach the polling host without a release
    if (hipHostMalloc((void**)&P.hctl, sizeof(Ctl), hipHostMallocCoherent) != hipSuccess) return MG_ERR_HIP;
    if (hipHostMalloc((void**)&P.hact, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) return MG_ERR_HIP;
    if (hipHostMalloc((void**)&P.hres, kCtlHead * (size_t)P.nprob, hipHostMallocDefault) != hipSuccess)
        return MG_ERR_HIP;
    memset(P.hfin, 0, fb);
    if (hipMemsetAsync(P.ws, 0, P.total, stream) != hipSuccess) return MG_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return MG_ERR_HIP;
    int e = P.prec == MG_FP64 ? write_tables<double>(P) : write_tables<float>(P);
    if (e) return e;
    const char* ng = getenv("DMG_NO_GRAPH");
    P.use_graph = !(ng && ng[0] == '1');
    // out-of-place solves form each evaluation's residual in the finest
    // kernel of the cycle before it unless DMG_NO_FUSED_RESIDUAL=1 (then the
    // residual kernel runs after it, as for the first evaluation)
    const char* nr = getenv("DMG_NO_FUSED_RESIDUAL");
    P.res = P.oop && !(nr && nr[0] == '1');
    for (int k = 0; k < 2; k++)
        if (hipEventCreateWithFlags(&P.ev[k], hipEventDisableTiming) != hipSuccess) return MG_ERR_HIP;
    if (hipEventCreateWithFlags(&P.evu, hipEventDisableTiming) != hipSuccess) return MG_ERR_HIP;
    P.evs = true;
    return plan2_tune_load(P);
}

int plan2_bind_static(Plan2& P, void* ws, hipStream_t stream)
{
    if (P.nprob != 1) return MG_ERR_ARG;
    if (!ws || ((uintptr_t)ws % kAlign) != 0) return MG_ERR_WS;
    P.ws = (char*)ws;
    P.stream = stream;
    P.tm.stream = stream;
    P.stat = true;
    P.use_graph = false;
    if (hipGetDevice(&P.device) != hipSuccess) return MG_ERR_HIP;
    // every call starts from a zero workspace: boundary entries of every
    // level read 0, and the previous call's contents are gone
    launch_zero(P.ws, P.total, stream);
    int e = last_launch();
    if (e) return e;
    P.stage.clear();
    P.stage_lo = P.total;
    if ((e = P.prec == MG_FP64 ? write_tables<double>(P) : write_tables<float>(P))) return e;
    if (P.stage.size() > P.stage_lo) {   // the tables sit together at the start of the workspace
        launch_put_bytes(P.ws + P.stage_lo, P.stage.data() + P.stage_lo, P.stage.size() - P.stage_lo, stream);
        e = last_launch();
    }
    return e;
}

void plan2_destroy(Plan2& P)
{
    P.tm.destroy();
    if (P.gready) (void)hipGraphExecDestroy(P.gexec);
    if (P.cap) (void)hipStreamDestroy(P.cap);
    if (P.evs) {
        (void)hipStreamSynchronize(P.stream);
        for (int k = 0; k < 2; k++) (void)hipEventDestroy(P.ev[k]);
        (void)hipEventDestroy(P.evu);
    }
    if (P.hfin) (void)hipHostFree(P.hfin);
    if (P.hctl) (void)hipHostFree(P.hctl);
    if (P.hact) (void)hipHostFree(P.hact);
    if (P.hres) (void)hipHostFree(P.hres);
}

int plan2_vcycle(Plan2& P, double* const* u, const double* const* f, double* relres)
{
    Ctl* ctls = at<Ctl>(P, P.off_ctl);
    int* nact = at<int>(P, P.off_nactive);
    int e = bind_uf(P, u, f);
    if (e) return e;
    P.r0_stale = false;   // the cycle stores the finest residual
    if (P.rorder == 4) launch_b_rhs4(P.n[0], f[0], at<double>(P, P.off_g), P.stream);
    launch_b_ctl_reset(ctls, P.nprob, 0, 0, 0.0, nact, P.has_net ? 1 : 0, P.stream);
    const bool wf = relres != nullptr;
    if (P.prec == MG_FP64) {
        if (wf) enq_norm_f<double>(P, ctls, nact, true);
        enq_resid<double>(P, ctls, nact, wf);
        enq_cycle<double>(P, ctls);
    } else {
        if (wf) enq_norm_f<float>(P, ctls, nact, true);
        enq_resid<float>(P, ctls, nact, wf);
        enq_cycle<float>(P, ctls);
    }
    e = last_launch();
    if (e) return e;
    if (relres && P.stat) {   // no pinned buffer: one double straight into the caller's
        if (hipMemcpyAsync(relres, &ctls[0].last, sizeof(double), hipMemcpyDeviceToHost, P.stream) != hipSuccess ||
            hipStreamSynchronize(P.stream) != hipSuccess)
            return MG_ERR_HIP;
        return MG_OK;
    }
    if (relres) {
        // relative residual of the entry u of every problem
        if (hipMemcpy2DAsync(P.hres, kCtlHead, ctls, sizeof(Ctl), kCtlHead, P.nprob,
                             hipMemcpyDeviceToHost, P.stream) != hipSuccess)
            return MG_ERR_HIP;
        if (hipStreamSynchronize(P.stream) != hipSuccess) return MG_ERR_HIP;
        for (int i = 0; i < P.nprob; i++) relres[i] = reinterpret_cast<const Ctl*>(P.hres + kCtlHead * (size_t)i)->last;
    }
    return MG_OK;
}

int plan2_solve(Plan2& P, double* const* u, const double* const* f, double rtol, int max_cycles, int* cycles,
                double* relres, int* status, double* history0)
{
    Ctl* ctls = at<Ctl>(P, P.off_ctl);
    int* nact = at<int>(P, P.off_nactive);
    int e = bind_uf(P, u, f);
    if (e) return e;
    if (P.nprob == 1) {   // a fresh pinned count before any kernel of this solve can write it
        P.hctl->k = 0;
        P.hctl->done = 0;
    }
    if (P.rorder == 4) launch_b_rhs4(P.n[0], f[0], at<double>(P, P.off_g), P.stream);
    launch_b_ctl_reset(ctls, P.nprob, 1, max_cycles, rtol, nact, P.has_net ? 1 : 0, P.stream);
    if (P.oop) {   // the second iterate buffer takes u's boundary values
        launch_b_copy_ring(P.n[0], u[0], at<double>(P, P.off_r0[0]), P.stream);
        P.r0_stale = true;
    }
    if (P.prec == MG_FP64) {
        enq_norm_f<double>(P, ctls, nact, true);
        enq_resid<double>(P, ctls, nact, true, P.oop);
    } else {
        enq_norm_f<float>(P, ctls, nact, true);
        enq_resid<float>(P, ctls, nact, true, P.oop);
    }
    if ((e = last_launch())) return e;
    // The active-problem count after evaluation it lands in host slot it & 1
    // before event ev[it & 1]: copied, or for a single problem the finalize
    // kernel writes its decision into the pinned control block itself (then
    // the host may read the next evaluation's; it never reverts, and that
    // evaluation is already queued, so stopping on it is right).
    const bool direct = P.nprob == 1;
    auto mark = [&](int it1) -> int {
        if (direct) return MG_OK;   // the host polls the pinned count instead (see wait)
        const int k = it1 & 1;
        if (hipMemcpyAsync(&P.hact[k], nact, sizeof(int), hipMemcpyDeviceToHost, P.stream) != hipSuccess)
            return MG_ERR_HIP;
        return hip_status(hipEventRecord(P.ev[k], P.stream));
    };
    // wait for evaluation it: a single problem's finalize kernel writes the
    // count of evaluations done (and the decision) into the pinned control
    // block, which the host polls -- no event between iterations, whose
    // system-scope release would stall the queue every cycle.  Should the
    // count not show within 50 ms, a stream synchronisation settles it.
    auto wait = [&](int it) -> int {
        if (!direct) return hipEventSynchronize(P.ev[it & 1]) == hipSuccess ? MG_OK : MG_ERR_HIP;
        const volatile Ctl* h = P.hctl;
        const auto t0 = std::chrono::steady_clock::now();
        for (unsigned spin = 0; h->k < it + 1 && !h->done; spin++) {
            if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50))
                return hipStreamSynchronize(P.stream) == hipSuccess ? MG_OK : MG_ERR_HIP;
        }
        return MG_OK;
    };

    if ((e = mark(0))) return e;
    // Iteration it+1 is launched before the host looks at what iteration it
    // left, so the GPU does not wait for the host between cycles -- unless a
    // single problem's residual trend says iteration it is probably the last:
    // then the host waits first, rather than queue a whole gated iteration
    // that would only return.
    double rr1 = -1, rr2 = -1;   // relative residuals of evaluations it-1, it-2 (single problem)
    for (int it = 0;; it++) {
        const bool likely_last = direct && rr1 > 0 && rr2 > 0 && rr1 * (rr1 / rr2) <= 2 * rtol;
        bool ahead = false;
        if (it < max_cycles && !likely_last) {
            if ((e = run_iteration(P)) || (e = mark(it + 1))) return e;
            ahead = true;
        }
        if ((e = wait(it))) return e;
        const int active = direct ? (*(volatile int*)&P.hctl->done ? 0 : 1) : P.hact[it & 1];
        if (active <= 0 || it >= max_cycles) break;
        if (direct) {
            rr2 = rr1;
            rr1 = *(volatile double*)&P.hctl->last;
        }
        if (!ahead && (e = run_iteration(P)) == MG_OK) e = mark(it + 1);
        if (e) return e;
    }
    // out of place: cycle k left its iterate in ub for odd k (the kernel
    // reads the count); the array's boundary then reads 0 again, as the
    // cycles of mg_vcycle expect
    if (P.oop) launch_b_oop_finish(P.n[0], ctls, at<double>(P, P.off_r0[0]), u[0], P.stream);
    // per-problem outcome: the first fields of each control block (a single
    // problem's are in the pinned copy already)
    if (!direct) {
        if (hipMemcpy2DAsync(P.hres, kCtlHead, ctls, sizeof(Ctl), kCtlHead, P.nprob, hipMemcpyDeviceToHost,
                             P.stream) != hipSuccess)
            return MG_ERR_HIP;
        if (history0 && hipMemcpyAsync(P.hctl, ctls, sizeof(Ctl), hipMemcpyDeviceToHost, P.stream) != hipSuccess)
            return MG_ERR_HIP;
    }
    if (hipStreamSynchronize(P.stream) != hipSuccess) return MG_ERR_HIP;
    int worst = MG_OK;
    for (int i = 0; i < P.nprob; i++) {
        const Ctl* c = direct ? P.hctl : reinterpret_cast<const Ctl*>(P.hres + kCtlHead * (size_t)i);
        int st = c->done ? c->status : MG_ERR_NOT_CONVERGED;
        int cy = c->done ? c->cycles : max_cycles;
        if (cycles) cycles[i] = cy;
        if (relres) relres[i] = c->last;
        if (status) status[i] = st;
        if (st != MG_OK && (worst == MG_OK || st < worst)) worst = st;
    }
    if (history0) {
        const Ctl& H = *P.hctl;
        int cy = H.done ? H.cycles : max_cycles;
        for (int k = 0; k <= cy; k++) history0[k] = H.hist[k];
    }
    return worst;
}

template <typename T>
int recompute_diag(Plan2& P, int lam, size_t above, bool jacobi)
{
    // restriction item (r <- Eq. Erest2r of `in`), then the Jacobi item
    Item2<T> it[2] = {{at<T>(P, P.off_r[0][lam]), nullptr, at<T>(P, above), 0, 0},
                      {at<T>(P, P.off_r[0][lam]), at<T>(P, P.off_v[0][lam]), at<T>(P, P.off_v[0][lam - 1]), 0, 0}};
    if (hipStreamSynchronize(P.stream) != hipSuccess ||
        hipMemcpy(P.ws + P.off_lg_item, it, sizeof(it), hipMemcpyHostToDevice) != hipSuccess)
        return MG_ERR_HIP;
    // the zero block serves as a control block that is never done
    Item2<T>* dit = at<Item2<T>>(P, P.off_lg_item);
    launch_b_restrict<T>(0, side_of(lam), 0, dit, 1, at<Ctl>(P, P.off_zero), P.stream);
    if (jacobi)
        launch_b_jacobi<T>(1, side_of(lam), b_default_rows(2, side_of(lam)), (T)coef(P, lam), dit + 1, 1,
                           at<Ctl>(P, P.off_zero), P.stream);
    return last_launch();
}

int plan2_level_get(Plan2& P, int depth, int which, double* dst)
{
    // problem 0; depth counts from its finest level
    int D = P.D[0];
    if (depth < 0 || depth > D || (which != 0 && which != 1) || (which == 1 && depth == 0)) return MG_ERR_ARG;
    int lam = D - depth;
    int m = side_of(lam);
    int diag = lam & 1;
    // after an out-of-place solve the finest residual's array holds an
    // iterate: the finest residual and the first diagonal level (made from it)
    // are not available until the next mg_vcycle
    if (P.r0_stale && depth <= 1) return MG_ERR_ARG;
    size_t off = (which == 0) ? (depth == 0 ? P.off_r0[0] : P.off_r[0][lam]) : P.off_v[0][lam];
    if ((lam & 1) && ((lam == D - 1 && fin_fused(D, P.lamc) && side_of(D) >= 8) || pair_level(lam + 1, D, P.pairs))) {
        // the cycle restricted and relaxed this diagonal level inside the
        // kernels of the axis level above it without storing either: rerun
        // its restriction and its Jacobi (same arithmetic, so the same
        // values) from the axis level's residual and the coarser correction
        // the cycle left
        const size_t above = lam == D - 1 ? P.off_r0[0] : P.off_r[0][lam + 1];
        int e = P.prec == MG_FP64 ? recompute_diag<double>(P, lam, above, which == 1)
                                  : recompute_diag<float>(P, lam, above, which == 1);
        if (e) return e;
    }
    if (P.prec == MG_FP64) launch_b_level_get<double>(diag, m, at<double>(P, off), dst, P.stream);
    else launch_b_level_get<float>(diag, m, at<float>(P, off), dst, P.stream);
    return last_launch();
}

// ------------------------------------------------------------- autotuner
// For every level launch of the cycle, time each candidate strip length
// (0 = one thread per point, else rows per wave) on the plan's own arrays and
// keep the fastest.  The kernels only write level arrays that the next cycle
// overwrites.  Results can be kept in a text cache (DMG_TUNE_CACHE): one line
// "kind side prec rows" per tuned launch shape.

namespace {

struct TuneKey { int kind, m, prec; };

int cache_lookup(const char* path, int kind, int m, int prec, int* rows)
{
    FILE* fp = path ? fopen(path, "r") : nullptr;
    if (!fp) return 0;
    int k, mm, pr, r, found = 0;
    while (fscanf(fp, "%d %d %d %d", &k, &mm, &pr, &r) == 4)
        if (k == kind && mm == m && pr == prec) { *rows = r; found = 1; }
    fclose(fp);
    return found;
}

void cache_store(const char* path, int kind, int m, int prec, int rows)
{
    FILE* fp = path ? fopen(path, "a") : nullptr;
    if (!fp) return;
    fprintf(fp, "%d %d %d %d\n", kind, m, prec, rows);
    fclose(fp);
}

template <typename T>
float time_launch(Plan2& P, int is_rs, int lam, int rows, hipEvent_t e0, hipEvent_t e1)
{
    Ctl* ctls = at<Ctl>(P, P.off_ctl);
    auto go = [&]() {
        if (is_rs)
            launch_b_restrict<T>((lam + 1) & 1, side_of(lam + 1), rows, at<Item2<T>>(P, P.off_rs_items[lam]),
                                 P.n_rs_items[lam], ctls, P.stream);
        else
            launch_b_jacobi<T>(lam & 1, side_of(lam), rows, (T)coef(P, lam), at<Item2<T>>(P, P.off_jac_items[lam]),
                               P.n_jac_items[lam], ctls, P.stream);
    };
    go();
    (void)hipEventRecord(e0, P.stream);
    for (int k = 0; k < 5; k++) go();
    (void)hipEventRecord(e1, P.stream);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms;
}

}  // namespace

int plan2_tune_load(Plan2& P)
{
    const char* path = getenv("DMG_TUNE_CACHE");
    if (!path) return MG_OK;
    for (int lam = 0; lam <= P.Dmax; lam++) {
        int r;
        if (P.n_rs_items[lam] && cache_lookup(path, ((lam + 1) & 1) ? 1 : 0, side_of(lam + 1), P.prec, &r)) P.rows_rs[lam] = r;
        if (P.n_jac_items[lam] && cache_lookup(path, (lam & 1) ? 2 : 3, side_of(lam), P.prec, &r)) P.rows_jac[lam] = r;
    }
    return MG_OK;
}

int plan2_autotune(Plan2& P)
{
    const char* path = getenv("DMG_TUNE_CACHE");
    Ctl* ctls = at<Ctl>(P, P.off_ctl);
    int* nact = at<int>(P, P.off_nactive);
    launch_b_ctl_reset(ctls, P.nprob, 0, 0, 0.0, nact, 0, P.stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MG_ERR_HIP;
    const int cand[] = {0, 4, 8, 16, 32};
    for (int is_rs = 1; is_rs >= 0; is_rs--) {
        for (int lam = 0; lam <= P.Dmax; lam++) {
            int cnt = is_rs ? P.n_rs_items[lam] : P.n_jac_items[lam];
            if (!cnt) continue;
            int m = is_rs ? side_of(lam + 1) : side_of(lam);
            int kind = is_rs ? (((lam + 1) & 1) ? 1 : 0) : ((lam & 1) ? 2 : 3);
            int best = is_rs ? P.rows_rs[lam] : P.rows_jac[lam];
            float bt = 1e30f;
            for (int r : cand) {
                if (r > 0 && m < 16) continue;
                float t = P.prec == MG_FP64 ? time_launch<double>(P, is_rs, lam, r, e0, e1)
                                            : time_launch<float>(P, is_rs, lam, r, e0, e1);
                if (t < bt) { bt = t; best = r; }
            }
            (is_rs ? P.rows_rs : P.rows_jac)[lam] = best;
            cache_store(path, kind, m, P.prec, best);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (P.gready) {  // the captured graph used the old shapes
        (void)hipGraphExecDestroy(P.gexec);
        P.gready = false;
    }
    return last_launch();
}

}  // namespace dmg

namespace dmg {

// ------------------------------------------------ learned coarse correction

int plan2_set_net(Plan2& P, const float* w, int cut_level)
{
    if (cut_level != kNetCut) return MG_ERR_ARG;
    if (w) {
        std::vector<bf16_t> wf(NetGeo<2>::PACK);
        std::vector<float> wm(w, w + NetGeo<2>::NW);
        for (int i = 0; i < NetGeo<2>::NW; i++) {   // the padded channels are not parameters
            int layer = (i >> 8) / NetGeo<2>::T, ci = (i >> 4) & 15, co = i & 15;
            if ((layer == 0 && ci) || (layer == kNetLayers - 1 && co)) wm[i] = 0.f;
        }
        net_pack_host(2, wm.data(), wf.data(), nullptr);
        if (hipStreamSynchronize(P.stream) != hipSuccess ||
            hipMemcpy(P.ws + P.off_net, wf.data(), sizeof(bf16_t) * wf.size(), hipMemcpyHostToDevice) != hipSuccess)
            return MG_ERR_HIP;
    }
    bool on = w != nullptr;
    if (on != P.has_net && P.gready) {   // the captured iteration launches the other coarse kernel
        (void)hipGraphExecDestroy(P.gexec);
        P.gready = false;
    }
    P.has_net = on;
    return MG_OK;
}

int plan2_net_stats(Plan2& P, int* net_cycles, int* fell_back, double* q_net, double* q_plain)
{
    Ctl* ctls = reinterpret_cast<Ctl*>(P.ws + P.off_ctl);
    if (hipMemcpy2DAsync(P.hres, kCtlHead, ctls, sizeof(Ctl), kCtlHead, P.nprob, hipMemcpyDeviceToHost, P.stream) !=
            hipSuccess ||
        hipStreamSynchronize(P.stream) != hipSuccess)
        return MG_ERR_HIP;
    for (int i = 0; i < P.nprob; i++) {
        const Ctl* c = reinterpret_cast<const Ctl*>(P.hres + kCtlHead * (size_t)i);
        if (net_cycles) net_cycles[i] = c->net_used;
        if (fell_back) fell_back[i] = c->net_off;
        if (q_net) q_net[i] = c->q_net;
        if (q_plain) q_plain[i] = c->theta;
    }
    return MG_OK;
}

int plan2_coarse_export(Plan2& P, int level, double* dst)
{
    if (level < 0 || level > P.lamc || !dst) return MG_ERR_ARG;
    int m = side_of(level), diag = level & 1;
    if (!P.n_coarse_items) return MG_OK;
    Coarse2B<double>* items = reinterpret_cast<Coarse2B<double>*>(P.ws + P.off_coarse);
    if (hipMemsetAsync(dst, 0, sizeof(double) * sizeA(m) * (size_t)P.nprob, P.stream) != hipSuccess) return MG_ERR_HIP;
    if (P.prec == MG_FP64)
        launch_b_coarse_export<double>(level, diag, m, items, P.n_coarse_items, dst, P.stream);
    else
        launch_b_coarse_export<float>(level, diag, m, reinterpret_cast<Coarse2B<float>*>(items), P.n_coarse_items, dst,
                                      P.stream);
    return last_launch();
}

}  // namespace dmg

// Exported C ABI of libdmg (include/dmg.h): argument checks and dispatch to
// the 2D plan (a batch of problems; a single problem is a batch of one) or
// the 3D plan.
#include "dmg_net.hpp"
#include "dmg_plan2d.hpp"
#include "dmg_plan3d.hpp"
#include "dmg_gen.hpp"
#include "dmg_usual.hpp"

#include <new>

using namespace dmg;

struct mg_plan {
    int dim = 0;
    Plan2* p2 = nullptr;
    Plan3* p3 = nullptr;
    PlanU* pu = nullptr;   // the conventional comparison cycle (MG_USUAL)
    PlanG* pg = nullptr;   // the diagonal cycle with nu sweeps and gamma coarse visits
    int device = 0;
    Timing* tm() { return p2 ? &p2->tm : p3 ? &p3->tm : pu ? &pu->tm : &pg->tm; }
};

namespace {

int check_size(int dim, int n)
{
    if (dim != 2 && dim != 3) return MG_ERR_ARG;
    int K = ilog2(n);
    if (K < 1) return MG_ERR_SIZE;
    if (dim == 2 && K > 15) return MG_ERR_SIZE;
    if (dim == 3 && K > 11) return MG_ERR_SIZE;
    return MG_OK;
}

int check_p(const double* p, int np)
{
    for (int i = 0; i < np; i++)
        if (!(p[i] > 0 && p[i] < 1e6)) return MG_ERR_ARG;
    return MG_OK;
}

void free_plan(mg_plan* P)
{
    if (!P) return;
    if (P->p2) { plan2_destroy(*P->p2); delete P->p2; }
    if (P->p3) { plan3_destroy(*P->p3); delete P->p3; }
    if (P->pu) { planu_destroy(*P->pu); delete P->pu; }
    if (P->pg) { plang_destroy(*P->pg); delete P->pg; }
    delete P;
}

}  // namespace

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
    case MG_ERR_SCRATCH: return "problem too large for the static scratch buffer";
    default: return "unknown error code";
    }
}

int mg_level_info(int dim, int n, int depth, int* num_levels, int* side)
{
    int e = check_size(dim, n);
    if (e) return e;
    int nl = dim * (ilog2(n) - 1) + 1;
    if (num_levels) *num_levels = nl;
    if (side) {
        if (depth < 0 || depth >= nl) return MG_ERR_ARG;
        *side = n >> (depth / dim);
    }
    return MG_OK;
}

int mg_workspace_bytes(int dim, int n, int precision, size_t* bytes)
{
    if (!bytes) return MG_ERR_ARG;
    int e = check_size(dim, n);
    if (e) return e;
    if (precision & MG_USUAL) {
        PlanU L;
        if ((e = planu_layout(L, dim, n, precision, 1.0))) return e;
        *bytes = L.total;
        return MG_OK;
    }
    if (dim == 2) {
        Plan2 L;
        if ((e = plan2_layout(L, 1, &n, precision, 1.0))) return e;
        *bytes = L.total;
    } else {
        Plan3 L;
        if ((e = plan3_layout(L, n, precision, nullptr))) return e;
        *bytes = L.total;
    }
    return MG_OK;
}

int mg_batch_workspace_bytes(int nprob, const int* n, int precision, size_t* bytes)
{
    if (!bytes || !n || nprob < 1) return MG_ERR_ARG;
    Plan2 L;
    int e = plan2_layout(L, nprob, n, precision, 1.0);
    if (e) return e;
    *bytes = L.total;
    return MG_OK;
}

int mg_setup_batched(mg_plan** out, int nprob, const int* n, int precision, double p, void* workspace,
                     size_t ws_bytes, void* hip_stream)
{
    if (!out || !n || nprob < 1) return MG_ERR_ARG;
    *out = nullptr;
    if (check_p(&p, 1)) return MG_ERR_ARG;
    mg_plan* P = new (std::nothrow) mg_plan;
    if (!P) return MG_ERR_ALLOC;
    P->dim = 2;
    P->p2 = new (std::nothrow) Plan2;
    if (!P->p2) { delete P; return MG_ERR_ALLOC; }
    int e = plan2_layout(*P->p2, nprob, n, precision, p);
    if (!e) e = plan2_setup(*P->p2, workspace, ws_bytes, (hipStream_t)hip_stream);
    if (e) { free_plan(P); return e; }
    P->device = P->p2->device;
    *out = P;
    return MG_OK;
}

int mg_setup(mg_plan** out, int dim, int n, int precision, const double* p, int np, void* workspace,
             size_t ws_bytes, void* hip_stream)
{
    if (!out || !p) return MG_ERR_ARG;
    *out = nullptr;
    const bool usual = (precision & MG_USUAL) != 0;
    if (usual ? np != 1 : ((dim == 2 && np != 1) || (dim == 3 && np != 4))) return MG_ERR_ARG;
    if (check_p(p, np)) return MG_ERR_ARG;
    int e = check_size(dim, n);
    if (e) return e;
    if (usual) {
        mg_plan* P = new (std::nothrow) mg_plan;
        if (!P) return MG_ERR_ALLOC;
        P->dim = dim;
        P->pu = new (std::nothrow) PlanU;
        if (!P->pu) { delete P; return MG_ERR_ALLOC; }
        e = planu_layout(*P->pu, dim, n, precision, p[0]);
        if (!e) e = planu_setup(*P->pu, workspace, ws_bytes, (hipStream_t)hip_stream);
        if (e) { free_plan(P); return e; }
        P->device = P->pu->device;
        *out = P;
        return MG_OK;
    }
    if (dim == 2) return mg_setup_batched(out, 1, &n, precision, p[0], workspace, ws_bytes, hip_stream);
    mg_plan* P = new (std::nothrow) mg_plan;
    if (!P) return MG_ERR_ALLOC;
    P->dim = 3;
    P->p3 = new (std::nothrow) Plan3;
    if (!P->p3) { delete P; return MG_ERR_ALLOC; }
    e = plan3_layout(*P->p3, n, precision, p);
    if (!e) e = plan3_setup(*P->p3, workspace, ws_bytes, (hipStream_t)hip_stream);
    if (e) { free_plan(P); return e; }
    P->device = P->p3->device;
    *out = P;
    return MG_OK;
}

int mg_cycle_workspace_bytes(int dim, int n, int precision, int nu, int gamma, size_t* bytes)
{
    if (!bytes) return MG_ERR_ARG;
    int e = check_size(dim, n);
    if (e) return e;
    PlanG L;
    if ((e = plang_layout(L, dim, n, precision, nullptr, nu, gamma))) return e;
    *bytes = L.total;
    return MG_OK;
}

int mg_setup_cycle(mg_plan** out, int dim, int n, int precision, const double* p, int np, int nu, int gamma,
                   void* workspace, size_t ws_bytes, void* hip_stream)
{
    if (!out || !p) return MG_ERR_ARG;
    *out = nullptr;
    if ((dim == 2 && np != 1) || (dim == 3 && np != 4)) return MG_ERR_ARG;
    if (check_p(p, np)) return MG_ERR_ARG;
    int e = check_size(dim, n);
    if (e) return e;
    mg_plan* P = new (std::nothrow) mg_plan;
    if (!P) return MG_ERR_ALLOC;
    P->dim = dim;
    P->pg = new (std::nothrow) PlanG;
    if (!P->pg) { delete P; return MG_ERR_ALLOC; }
    e = plang_layout(*P->pg, dim, n, precision, p, nu, gamma);
    if (!e) e = plang_setup(*P->pg, workspace, ws_bytes, (hipStream_t)hip_stream);
    if (e) { free_plan(P); return e; }
    P->device = P->pg->device;
    *out = P;
    return MG_OK;
}

int mg_destroy(mg_plan* P)
{
    if (!P) return MG_ERR_ARG;
    DevGuard g(P->device);
    free_plan(P);
    return MG_OK;
}

int mg_vcycle(mg_plan* P, double* u, const double* f, double* rel_res_before)
{
    if (!P || !u || !f) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->pu) return planu_vcycle(*P->pu, u, f, rel_res_before);
    if (P->pg) return plang_vcycle(*P->pg, u, f, rel_res_before);
    if (P->p3) return plan3_vcycle(*P->p3, u, f, rel_res_before);
    if (P->p2->nprob != 1) return MG_ERR_ARG;
    return plan2_vcycle(*P->p2, &u, &f, rel_res_before);
}

int mg_vcycle_batched(mg_plan* P, double* const* u, const double* const* f, double* rel_res_before)
{
    if (!P || !u || !f || !P->p2) return MG_ERR_ARG;
    for (int i = 0; i < P->p2->nprob; i++)
        if (!u[i] || !f[i]) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    return plan2_vcycle(*P->p2, u, f, rel_res_before);
}

int mg_solve(mg_plan* P, double* u, const double* f, double rtol, int max_cycles, int* cycles_out,
             double* rel_res_out, double* history)
{
    if (!P || !u || !f || !(rtol >= 0) || max_cycles < 0 || max_cycles > kMaxCycles) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->pu) return planu_solve(*P->pu, u, f, rtol, max_cycles, cycles_out, rel_res_out, history);
    if (P->pg) return plang_solve(*P->pg, u, f, rtol, max_cycles, cycles_out, rel_res_out, history);
    if (P->p3) return plan3_solve(*P->p3, u, f, rtol, max_cycles, cycles_out, rel_res_out, history);
    if (P->p2->nprob != 1) return MG_ERR_ARG;
    return plan2_solve(*P->p2, &u, &f, rtol, max_cycles, cycles_out, rel_res_out, nullptr, history);
}

int mg_solve_two_stage(mg_plan* first, mg_plan* second, double* u, const double* f, double rtol1, double rtol,
                       int max_cycles, int* cycles1, int* cycles2, double* rel_res_out)
{
    if (!first || !second || first == second || first->pu || second->pu || first->pg || second->pg) return MG_ERR_ARG;
    auto shape = [](const mg_plan* P, int& dim, int& n, int& order, int& nprob) {
        dim = P->dim;
        n = P->p3 ? P->p3->n : P->p2->n[0];
        order = P->p3 ? P->p3->rorder : P->p2->rorder;
        nprob = P->p3 ? 1 : P->p2->nprob;
    };
    int d1, n1, o1, b1, d2, n2, o2, b2;
    shape(first, d1, n1, o1, b1);
    shape(second, d2, n2, o2, b2);
    if (d1 != d2 || n1 != n2 || o1 != 2 || o2 != 4 || b1 != 1 || b2 != 1) return MG_ERR_ARG;
    int c1 = 0, c2 = 0;
    double rr = 0;
    int e = mg_solve(first, u, f, rtol1, max_cycles, &c1, &rr, nullptr);
    if (e == MG_OK || e == MG_ERR_NOT_CONVERGED)   // mg_solve has synchronised the first plan's stream
        e = mg_solve(second, u, f, rtol, max_cycles, &c2, &rr, nullptr);
    if (cycles1) *cycles1 = c1;
    if (cycles2) *cycles2 = c2;
    if (rel_res_out) *rel_res_out = rr;
    return e;
}

int mg_solve_batched(mg_plan* P, double* const* u, const double* const* f, double rtol, int max_cycles, int* cycles,
                     double* rel_res, int* status)
{
    if (!P || !u || !f || !P->p2 || !(rtol >= 0) || max_cycles < 0 || max_cycles > kMaxCycles) return MG_ERR_ARG;
    for (int i = 0; i < P->p2->nprob; i++)
        if (!u[i] || !f[i]) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    return plan2_solve(*P->p2, u, f, rtol, max_cycles, cycles, rel_res, status, nullptr);
}

int mg_autotune(mg_plan* P)
{
    if (!P || !P->p2) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    return plan2_autotune(*P->p2);
}

int mg_timing_enable(mg_plan* P, int family)
{
    if (!P || family < -1 || family >= MG_K_FAMILIES) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    return P->tm()->enable(family);
}

int mg_timing_read(mg_plan* P, double* ms, long long* launches, double* bytes)
{
    if (!P) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    P->tm()->read(ms, launches, bytes);
    return MG_OK;
}

int mg_net_weight_count(int dim) { return net_weight_count(dim); }

int mg_set_coarse_net(mg_plan* P, const float* w, int cut_level)
{
    if (!P) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->p2) return plan2_set_net(*P->p2, w, cut_level);
    if (!P->p3) return MG_ERR_ARG;
    return plan3_set_net(*P->p3, w, cut_level);
}

int mg_net_stats(mg_plan* P, int* net_cycles, int* fell_back, double* q_net, double* q_plain)
{
    if (!P) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->p2) return plan2_net_stats(*P->p2, net_cycles, fell_back, q_net, q_plain);
    if (!P->p3) return MG_ERR_ARG;
    return plan3_net_stats(*P->p3, net_cycles, fell_back, q_net, q_plain);
}

int mg_coarse_export(mg_plan* P, int level, double* dst)
{
    if (!P || !dst) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->p2) return plan2_coarse_export(*P->p2, level, dst);
    if (!P->p3) return MG_ERR_ARG;
    return plan3_coarse_export(*P->p3, level, dst);
}

int mg_level_get(mg_plan* P, int depth, int which, double* dst)
{
    if (!P || !dst) return MG_ERR_ARG;
    DevGuard g(P->device);
    if (!g.ok) return MG_ERR_HIP;
    if (P->pu) return planu_level_get(*P->pu, depth, which, dst);
    if (P->pg) return plang_level_get(*P->pg, depth, which, dst);
    return P->p3 ? plan3_level_get(*P->p3, depth, which, dst) : plan2_level_get(*P->p2, depth, which, dst);
}

}  // extern "C"

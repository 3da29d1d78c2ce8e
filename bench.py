#!/usr/bin/env python3
"""Benchmark of the diagonally oriented multigrid solver (libdmg) on one GPU.

Workload: 2D unit square, 4097 x 4097 grid (h = 1/4096, 16,769,025 unknowns),
zero Dirichlet data, f = 16 seeded sine modes with N(0,1) amplitudes and
wavenumbers U{1..64} plus 1e-3 white noise (seed 2), p = 1.052.

One step = one solve from u = 0 to a relative residual of 1e-10 with the
plain FP64 V-cycle: residual, the whole restriction hierarchy, the coarse
levels, the Jacobi prolongation and the on-device convergence check, every
cycle.  value = unknowns * cycles / second over the timed steps.  The same
workload is also solved with the single-precision cycle plus FP64 refinement
and with the learned coarse correction (network trained first, outside the
timed region, on 10^4 cut-level pairs from 1025^2 plain solves); the time to
1e-10 of each form is reported under "modes".  The fourth-order residual
(Eq. Efos2) is timed on the same f, directly and in two stages, under
"fourth_order4097"; the 19-point one (Eq. Efos4) on the 257^3 cube under
"fourth_order_cube257".  The over-relaxation parameters re-tuned at 4097^2
and 257^3 (Nelder-Mead on the GPU cycle's factor) and the solves with them
are under "retuned4097" / "retuned_cube257".

roofline: the dominant kernel's algorithmic bytes per launch (every element
it must read or write, counted once) over its mean launch time, measured with
HIP events on the solver's stream inside the timed region.
cpu_baseline: the CPU oracle (plain C, one thread) solving the same workload
to the same tolerance.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time to 1e-10 rel. residual & unknowns*cycles/s; plain FP64 vs FP32-refined/learned"
FAMILY_NAMES = {0: "residual", 1: "restriction", 2: "jacobi", 3: "finest jacobi + u update", 4: "coarse levels",
                5: "norm"}
# the kernels of each family, as rocprofv3 names them
FAMILY_KERNELS = {
    "usual": {0: "k_residual", 1: "ku2_fw / ku3_fw (full weighting)", 2: "ku2_up / ku3_up (interpolation + red-black Jacobi)",
              3: "ku2_up / ku3_up, finest (u += v)", 4: "-", 5: "k_finalize"},
    2: {0: "kb_resid (a solve's first evaluation: r0 formed, not stored; Eqs. Erest2r then Erest2b onto r2, "
           "norm partials)",
        1: "kb_rs_pair, kb_mid_down, kb_rs_*",
        2: "kb_jac_pair, kb_mid_up, kb_jac_*",
        3: "kb_finest_res (r0 from u and f, r1 by Eq. Erest2r, Jacobi of the first diagonal and the finest axis "
           "level, u + v into the other iterate buffer; the next evaluation's residual of u + v, its norm partials "
           "and Eqs. Erest2r then Erest2b onto r2)",
        4: "kb_coarse", 5: "kb_finalize"},
    3: {0: "k3_resid_planes (r0 and Eq. Erred onto the red level, norm partials)",
        1: "k3_r2m_planes, k3_rs_m2b, k3_down_group (a level group of side 16..64 per launch), k3_rs_*",
        2: "k3_mag_planes, k3_red_planes, k3_green_planes, k3_up_group (a level group of side 16..64 per launch), k3_jac_mag",
        3: "k3_green_planes<finest> (green-red Jacobi, u += v)",
        4: "k3_coarse", 5: "k_finalize"},
}


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fp:
            for line in fp:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def err_vs(u, ref):
    """Error of a solution against a reference solution (max-norm and 2-norm, relative)."""
    import numpy as np
    if hasattr(u, "cpu"):
        u = u.cpu().numpy()
    d = u - ref
    return {"inf": float(np.abs(d).max() / np.abs(ref).max()), "l2": float(np.linalg.norm(d) / np.linalg.norm(ref))}


def kernel_table(S, f, cycles, torch):
    """Per kernel family: time, launches and algorithmic bytes per cycle of a
    solve (mg_solve, the path the timed solves take), from HIP events around
    every launch of the family on the solver's stream.  Each figure is the
    difference between a solve of 2 + `cycles` cycles and one of 2 cycles
    (rtol 0, so every cycle runs): the cycles' own launches, without the
    first residual evaluation and the set-up of a solve."""
    u = torch.zeros_like(f)
    S.solve(u, f, rtol=0.0, max_cycles=2)
    torch.cuda.synchronize()
    rows = []
    for fam in range(6):
        S.timing(fam)
        tot = []
        for k in (2, 2 + cycles):
            u.zero_()
            torch.cuda.synchronize()
            S.solve(u, f, rtol=0.0, max_cycles=k)
            tot.append(S.timing_read())
        S.timing(-1)
        ms, cnt, byt = (b - a for a, b in zip(*tot))
        if cnt <= 0:
            continue
        gbs = byt / (ms * 1e-3) / 1e9
        key = "usual" if getattr(S, "scheme", "diagonal") == "usual" else f.dim()
        rows.append({"family": FAMILY_NAMES[fam], "kernels": FAMILY_KERNELS[key][fam],
                     "us_per_cycle": round(1e3 * ms / cycles, 2), "launches_per_cycle": cnt / cycles,
                     "bytes_per_cycle": byt / cycles, "achieved_GBs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "family_id": fam})
    return rows


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic per launch of the roofline kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (calibrated on a copy of known size), as recorded in profiles/
# together with a hash of the kernel sources it was taken on; null when the
# sources have changed since.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_square4097.md")
KERNEL_SOURCES = ("dmg_b2d.hip", "dmg_rows.hpp", "dmg_common.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_math_9907190_amd", "csrc", f), "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def measured_traffic(family):
    key = {3: "finest_traffic_bytes_per_launch", 0: "residual_traffic_bytes_per_launch"}.get(family)
    if key is None or not os.path.exists(TRAFFIC_PROFILE):
        return None
    vals = {}
    with open(TRAFFIC_PROFILE) as fp:
        for line in fp:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_source_hash() or key not in vals:
        return None
    return float(vals[key])


def timed_solves(S, f, steps, warmup, rtol, family, torch):
    us = [torch.zeros_like(f) for _ in range(steps + warmup)]
    for k in range(warmup):
        st, cyc, rr, hist = S.solve(us[k], f, rtol=rtol, max_cycles=60)
        assert st == 0, (st, cyc, rr)
    torch.cuda.synchronize()
    if family is not None:
        S.timing(family)
    t0 = time.perf_counter()
    cycles = []
    for k in range(warmup, warmup + steps):
        st, cyc, rr, hist = S.solve(us[k], f, rtol=rtol, max_cycles=60)
        assert st == 0 and rr <= rtol, (st, cyc, rr)
        cycles.append(cyc)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = S.timing_read() if family is not None else None
    if family is not None:
        S.timing(-1)
    return dt, cycles, kern, us[-1], hist


def bench_fourth_order(dmg, f, dev, torch, args, ref=None):
    """Fourth-order solution (Eq. Efos2 / Efos4): fourth-order cycles from
    u = 0 with the parameters tuned for them (Sections 2.4 / 3.4) against the
    two-stage solve (second-order cycles with the tuned second-order
    parameters to 1e-3, then fourth-order cycles), each to a 1e-10
    fourth-order relative residual, FP64 and FP32-refined levels."""
    n = f.shape[0] - 1
    dim = f.dim()
    out = {}
    for pname, prec in (("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)):
        S2 = dmg.Solver(dim, n, precision=prec, device=dev)
        S4 = dmg.Solver(dim, n, precision=prec, device=dev, order=4)
        for mode in ("direct", "two_stage"):
            us = [torch.zeros_like(f) for _ in range(args.steps + args.warmup)]

            def one(u):
                if mode == "direct":
                    st, c2, rr, _ = S4.solve(u, f, rtol=args.rtol, max_cycles=60)
                    c1 = 0
                else:
                    st, c1, c2, rr = dmg.solve_two_stage(S2, S4, u, f, rtol1=1e-3, rtol=args.rtol, max_cycles=60)
                assert st == 0 and rr <= args.rtol, (st, c1, c2, rr)
                return c1, c2

            for k in range(args.warmup):
                one(us[k])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.warmup, args.warmup + args.steps):
                c1, c2 = one(us[k])
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / args.steps
            out["%s_%s" % (pname, mode)] = {"ms_to_rtol": round(ms, 4), "cycles_order2": c1, "cycles_order4": c2}
            if ref is not None:   # against the oracle's fourth-order FP64 solution
                out["%s_%s" % (pname, mode)]["err_vs_oracle"] = err_vs(us[-1], ref)
            log("  fourth order %s %s: %.3f ms per solve, %d + %d cycles" % (pname, mode, ms, c1, c2))
        S2.close()
        S4.close()
        torch.cuda.empty_cache()
    for pname in ("fp64", "fp32_refined"):
        out[pname + "_two_stage"]["speedup_vs_direct"] = round(
            out[pname + "_direct"]["ms_to_rtol"] / out[pname + "_two_stage"]["ms_to_rtol"], 3)
    return out


def bench_retuned(dmg, f, dev, torch, args, ref=None):
    """Over-relaxation parameters re-tuned at this size (Nelder-Mead on the GPU
    cycle's factor, Sections 2.4 / 3.4; the tuning is outside the timed
    region and timed on its own), then FP64 solves to 1e-10 with the paper's
    parameters and with the re-tuned ones."""
    from paper_math_9907190_amd import tune

    dim, n = f.dim(), f.shape[0] - 1
    paper = dmg.P2D_TUNED if dim == 2 else dmg.P3D_TUNED
    t0 = time.perf_counter()
    p, fac, nfev = tune.tune_p(dim, n, p0=paper, device=dev, maxfev=40 if dim == 2 else 120)
    tune_s = time.perf_counter() - t0
    out = {"p": [round(x, 4) for x in p], "factor": round(fac, 5), "evaluations": nfev, "tune_s": round(tune_s, 2),
           "paper_p": list(paper), "paper_factor": round(tune.gpu_factor(dim, n, paper, device=dev), 5)}
    for name, pp in (("paper_p", paper), ("retuned_p", p)):
        S = dmg.Solver(dim, n, precision=dmg.MG_FP64, p=pp, device=dev)
        dt, cycles, _, u_last, hist = timed_solves(S, f, args.steps, args.warmup, args.rtol, None, torch)
        out[name + "_fp64"] = {"ms_to_rtol": round(1e3 * dt / args.steps, 4), "cycles": cycles[-1],
                               "final_rel_res": hist[-1]}
        if ref is not None:
            out[name + "_fp64"]["err_vs_oracle"] = err_vs(u_last, ref)
        S.close()
        torch.cuda.empty_cache()
    out["speedup"] = round(out["paper_p_fp64"]["ms_to_rtol"] / out["retuned_p_fp64"]["ms_to_rtol"], 3)
    log("  retuned p %s (factor %.4f vs %.4f, %d evaluations, %.1f s): %.3f ms (%d cycles) vs %.3f ms (%d cycles)"
        % (out["p"], fac, out["paper_factor"], nfev, tune_s, out["retuned_p_fp64"]["ms_to_rtol"],
           out["retuned_p_fp64"]["cycles"], out["paper_p_fp64"]["ms_to_rtol"], out["paper_p_fp64"]["cycles"]))
    return out


def bench_usual(dmg, f, dev, torch, args, diag, ref=None):
    """The conventional comparison cycle (Sections 2.1-2.3, 3.1-3.3: full
    weighting, linear interpolation plus one red-black Jacobi iteration, the
    parameter the paper tunes for it) on the same workload to the same
    tolerance, FP64 and FP32-refined, against the diagonal cycle's times
    `diag` ({form: ms}) measured on the same GPU: the paper's claim that the
    diagonal grids are about twice as fast (Abstract, Sections 2.3, 3.4)."""
    dim, n = f.dim(), f.shape[0] - 1
    out = {}
    for pname, prec in (("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)):
        S = dmg.Solver(dim, n, precision=prec, scheme="usual", device=dev)
        dt, cycles, _, u_last, hist = timed_solves(S, f, args.steps, args.warmup, args.rtol, None, torch)
        ms = 1e3 * dt / args.steps
        d = {"ms_to_rtol": round(ms, 4), "cycles": cycles[-1], "p": S.p[0], "final_rel_res": hist[-1],
             "unknowns_cycles_per_s": (n - 1) ** dim * sum(cycles) / dt}
        if ref is not None:
            d["err_vs_oracle"] = err_vs(u_last, ref)
        if pname in diag:
            d["diagonal_ms_to_rtol"] = diag[pname]
            d["diagonal_speedup"] = round(ms / diag[pname], 3)
        if pname == "fp64":
            out["kernels"] = kernel_table(S, f, max(args.steps, 5), torch)
        out[pname] = d
        log("  usual %dD %s: %.3f ms, %d cycles (diagonal %s ms)" % (dim, pname, ms, cycles[-1], diag.get(pname)))
        S.close()
        del S
        torch.cuda.empty_cache()
    return out


CYCLE_SHAPES = ((1, 1), (2, 1), (3, 1), (1, 2), (2, 2))


def bench_cycles(dmg, f, dev, torch, args, v_ms, ref=None):
    """More Jacobi sweeps per level (nu) and W-cycles (gamma = 2), the
    directions Section 4 leaves to further research, on the same workload:
    FP64 time to 1e-10, cycles, the cycle's asymptotic factor (power
    iteration, f = 0) and the error against the oracle, for each (nu, gamma)
    through the per-level launches of mg_setup_cycle; (1, 1) there is the
    V-cycle without the fused kernels, so the ratios to it isolate the
    algorithm and the ratio to v_ms (the fused V-cycle) the whole cost.  The
    parameters are the paper's (tuned for nu = gamma = 1); nu = 2 is also run
    with parameters re-tuned for it at this size."""
    from paper_math_9907190_amd import tune

    dim, n = f.dim(), f.shape[0] - 1
    paper = dmg.P2D_TUNED if dim == 2 else dmg.P3D_TUNED
    out = {"fused_v_cycle_ms": v_ms}
    runs = [(nu, g, paper) for nu, g in CYCLE_SHAPES]
    t0 = time.perf_counter()
    p2, fac2, nfev = tune.tune_p(dim, n, p0=paper, device=dev, maxfev=30 if dim == 2 else 80, nu=2, gamma=1)
    out["retuned_nu2"] = {"p": [round(x, 4) for x in p2], "factor": round(fac2, 5), "evaluations": nfev,
                          "tune_s": round(time.perf_counter() - t0, 2)}
    runs.append((2, 1, p2))
    for nu, g, p in runs:
        key = "nu%d_gamma%d%s" % (nu, g, "" if p is paper else "_retuned")
        S = dmg.Solver(dim, n, p=p, device=dev, nu=nu, gamma=g)
        dt, cycles, _, u_last, hist = timed_solves(S, f, args.steps, args.warmup, args.rtol, None, torch)
        S.close()
        d = {"ms_to_rtol": round(1e3 * dt / args.steps, 4), "cycles": cycles[-1], "final_rel_res": hist[-1],
             "factor": round(tune.gpu_factor(dim, n, p, device=dev, nu=nu, gamma=g), 5)}
        if ref is not None:
            d["err_vs_oracle"] = err_vs(u_last, ref)
        out[key] = d
        torch.cuda.empty_cache()
    base = out["nu1_gamma1"]["ms_to_rtol"]
    for k, d in out.items():
        if k.startswith("nu"):
            d["time_vs_nu1_gamma1"] = round(d["ms_to_rtol"] / base, 3)
            d["time_vs_fused_v_cycle"] = round(d["ms_to_rtol"] / v_ms, 3)
            log("  %dD %s: %.3f ms, %d cycles, factor %.4f" % (dim, k, d["ms_to_rtol"], d["cycles"], d["factor"]))
    return out


def bench_batched(dmg, workloads, dev, torch, args, with_oracle=False):
    """512 independent 2D problems, sides drawn from {129, 257, 513, 1025}
    (seed 4), smooth-mode f per problem (seed 4+b); single-precision cycles with
    FP64 refinement to 1e-10; one launch per aligned level for the whole
    batch, iteration replayed from a hipGraph; launch shapes autotuned at
    setup (outside the timed region)."""
    ns = workloads.batch_sizes(512, seed=4)
    log("batched: generating %d problems" % len(ns))
    fs = [torch.from_numpy(workloads.batch_problem(n, b)).to(dev) for b, n in enumerate(ns)]
    B = dmg.BatchSolver(ns, precision=dmg.MG_FP32_REFINED, device=dev)
    B.autotune()
    unknowns = sum((n - 1) ** 2 for n in ns)
    us = [[torch.zeros_like(f) for f in fs] for _ in range(args.steps + args.warmup)]
    for k in range(args.warmup):
        st, cyc, rr, sts = B.solve(us[k], fs, rtol=args.rtol, max_cycles=60)
        assert st == 0, st
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ucs = 0
    for k in range(args.warmup, args.warmup + args.steps):
        st, cyc, rr, sts = B.solve(us[k], fs, rtol=args.rtol, max_cycles=60)
        assert st == 0 and max(rr) <= args.rtol, (st, max(rr))
        ucs += sum((n - 1) ** 2 * c for n, c in zip(ns, cyc))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {"workload": "512 problems, sides from {129,257,513,1025} (seed 4), 4 smooth modes each, "
                       "FP32 cycles + FP64 refinement to %.0e" % args.rtol,
           "unknowns": unknowns, "ms_to_rtol": round(1e3 * dt / args.steps, 3),
           "unknowns_cycles_per_s": ucs / dt, "cycles_max": max(cyc), "cycles_min": min(cyc),
           "max_final_rel_res": max(rr)}
    if with_oracle:
        # the first problem of each size against the oracle's FP64 solution
        from oracle import oracle as O
        errs = {}
        for side in sorted(set(ns)):
            b = ns.index(side)
            fh = fs[b].cpu().numpy()
            uo = O.solve(0 * fh, fh, p=(1.052,), rtol=args.rtol, max_cycles=60)[0]
            errs["problem%d_n%d" % (b, side)] = err_vs(us[-1][b], uo)
        res["err_vs_oracle_sample"] = errs
        res["err_vs_oracle_max_inf"] = max(e["inf"] for e in errs.values())
    log("  batched: %.3f ms per batch solve, cycles %d..%d, %.3e unknowns*cycles/s"
        % (res["ms_to_rtol"], min(cyc), max(cyc), res["unknowns_cycles_per_s"]))
    B.close()
    del us, fs, B
    torch.cuda.empty_cache()
    return res


def train_pair_of_nets(L, torch, r, e, log):
    """Trains one network towards the targets (mean squared error) and one on
    the cut-level objective, the same schedule and seeds; reports the cut
    objective of both over the pairs and returns the second one's weights."""
    epochs = sum(k for k, _ in L.SCHEDULE)
    info = {"epochs": epochs, "batch": 256, "lr_schedule": [list(x) for x in L.SCHEDULE], "loss": "cut"}
    w = None
    for loss in ("mse", "cut"):
        t1 = time.perf_counter()
        net, hist = L.train(r, e, batch=256, seed=7, schedule=L.SCHEDULE, loss=loss)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        w = net.weights().copy()
        net.close()
        obj = L.cut_objective(w, r)
        info[loss] = {"train_seconds": round(t2 - t1, 3), "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
                      "cut_objective": obj, "cut_ratio_rms": round(obj ** 0.5, 4)}
        log("  net (%s loss): %d epochs in %.2f s, loss %.3e -> %.3e, cut-level ratio (rms over pairs) %.4f"
            % (loss, epochs, t2 - t1, hist[0], hist[-1], obj ** 0.5))
    info["train_seconds"] = info["cut"]["train_seconds"]
    return w, info


def train_net(dmg, L, torch, log):
    """10^4 (r_c, e_c) pairs from 1250 plain FP64 solves of 1025^2 problems
    (f seeds 1000..2249, 8 cycles each), then Adam on the GPU."""
    t0 = time.perf_counter()
    r, e = L.make_pairs(n=1024, seeds=range(1000, 2250), cycles=8, log=log)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w, info = train_pair_of_nets(L, torch, r, e, log)
    info.update({"pairs": int(r.shape[0]), "pair_seconds": round(t1 - t0, 2)})
    info["train_us_per_step"] = round(1e6 * info["train_seconds"] / (info["epochs"] * (r.shape[0] // 256)), 1)
    del r, e
    torch.cuda.empty_cache()
    return w, info


def bench_learned(dmg, L, dev, torch, args, w, info, with_oracle=False):
    """Held-out 1025^2 problems (f seeds 5000..5031) solved as one batch to
    1e-10, plain against learned, FP64 and FP32-refined; the network's and
    the plain sub-cycle's first-cycle cut-level residual reductions as the
    coarse kernel measured them, and how often the judge kept the network."""
    ns = [1024] * 32
    fs = [torch.from_numpy(f).to(dev) for f in L.eval_problems(1024, range(5000, 5032))]
    refs = {}
    if with_oracle:   # oracle FP64 solutions of two held-out problems (one of each kind)
        from oracle import oracle as O
        for b in (0, 1):
            fh = fs[b].cpu().numpy()
            refs[b] = O.solve(0 * fh, fh, p=(1.052,), rtol=args.rtol, max_cycles=60)[0]
    res = {"workload": "32 held-out 1025^2 problems (f seeds 5000..5031: smooth modes / U(-1,1) alternating), "
                       "batched solve to %.0e; network trained on %d pairs" % (args.rtol, info["pairs"]),
           "training": info}
    for pname, prec in (("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)):
        out = {}
        for mode in ("plain", "learned"):
            B = dmg.BatchSolver(ns, precision=prec, device=dev)
            if mode == "learned":
                B.set_coarse_net(w)
            us = [torch.zeros_like(f) for f in fs]
            B.solve(us, fs, rtol=args.rtol, max_cycles=60)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                us = [torch.zeros_like(f) for f in fs]
                st, cyc, rr, sts = B.solve(us, fs, rtol=args.rtol, max_cycles=60)
                assert st == 0 and max(rr) <= args.rtol, (st, max(rr))
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            d = {"ms_to_rtol": round(1e3 * dt, 3), "cycles_min": min(cyc), "cycles_max": max(cyc),
                 "cycles_total": sum(cyc)}
            if refs:
                d["err_vs_oracle_sample"] = {"problem%d" % b: err_vs(us[b], r) for b, r in refs.items()}
            if mode == "learned":
                used, off, qn, qp = B.net_stats()
                d.update({"net_cycles": sum(used), "judge_switched_off": sum(off),
                          "first_cycle_cut_ratio_net_median": float(sorted(qn)[len(qn) // 2]),
                          "first_cycle_cut_ratio_plain_median": float(sorted(qp)[len(qp) // 2])})
            out[mode] = d
            B.close()
            del B, us
        out["learned_speedup"] = round(out["plain"]["ms_to_rtol"] / out["learned"]["ms_to_rtol"], 3)
        log("  learned %s: plain %.3f ms (%d cycles), learned %.3f ms (%d cycles), net on %d cycles, judge off %d/32"
            % (pname, out["plain"]["ms_to_rtol"], out["plain"]["cycles_total"], out["learned"]["ms_to_rtol"],
               out["learned"]["cycles_total"], out["learned"]["net_cycles"], out["learned"]["judge_switched_off"]))
        res[pname] = out
    del fs
    torch.cuda.empty_cache()
    return res


def bench_learned3d(dmg, L, dev, torch, args, with_oracle=False):
    """3D learned coarse correction: 10^4 pairs from 1250 plain FP64 solves
    of 129^3 problems (f seeds 1000..2249, 8 cycles each; the cut is the 9^3
    green grid), Adam on the GPU, then 8 held-out 129^3 problems (seeds
    5000..5007) solved to 1e-10 plain against learned."""
    t0 = time.perf_counter()
    r, e = L.make_pairs_3d(n=128, seeds=range(1000, 2250), cycles=8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w, info = train_pair_of_nets(L, torch, r, e, lambda m: log(m.replace("net (", "net 3D (")))
    info.update({"pairs": int(r.shape[0]), "pair_seconds": round(t1 - t0, 2)})
    del r, e
    fs = [torch.from_numpy(f).to(dev) for f in L.eval_problems(128, range(5000, 5008), dim=3)]
    ref = None
    if with_oracle:   # the oracle's FP64 solution of the last held-out problem
        from oracle import oracle as O
        fh = fs[-1].cpu().numpy()
        ref = O.solve(0 * fh, fh, p=dmg.P3D_TUNED, rtol=args.rtol, max_cycles=60)[0]
    res = {"workload": "8 held-out 129^3 problems (f seeds 5000..5007), each solved to %.0e; network trained on "
                       "%d cut-level pairs" % (args.rtol, info["pairs"]), "training": info}
    for pname, prec in (("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)):
        out = {}
        for mode in ("plain", "learned"):
            S = dmg.Solver(3, 128, precision=prec, device=dev)
            if mode == "learned":
                S.set_coarse_net(w)
            u = torch.zeros_like(fs[0])
            S.solve(u, fs[0], rtol=args.rtol, max_cycles=60)
            cyc_tot, used_tot, off_tot, qn, qp = 0, 0, 0, [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for f in fs:
                u = torch.zeros_like(f)
                st, cyc, rr, _ = S.solve(u, f, rtol=args.rtol, max_cycles=60)
                assert st == 0 and rr <= args.rtol, (st, rr)
                cyc_tot += cyc
                if mode == "learned":
                    a, b, c, d = S.net_stats()
                    used_tot, off_tot = used_tot + a, off_tot + b
                    qn.append(c)
                    qp.append(d)
            torch.cuda.synchronize()
            d = {"ms_per_problem": round(1e3 * (time.perf_counter() - t0) / len(fs), 3), "cycles_total": cyc_tot}
            if ref is not None:
                d["err_vs_oracle_last_problem"] = err_vs(u, ref)
            if mode == "learned":
                d.update({"net_cycles": used_tot, "judge_switched_off": off_tot,
                          "first_cycle_cut_ratio_net_median": float(sorted(qn)[len(qn) // 2]),
                          "first_cycle_cut_ratio_plain_median": float(sorted(qp)[len(qp) // 2])})
            out[mode] = d
            S.close()
        out["learned_speedup"] = round(out["plain"]["ms_per_problem"] / out["learned"]["ms_per_problem"], 3)
        log("  learned 3D %s: plain %.3f ms (%d cycles), learned %.3f ms (%d cycles), net on %d cycles, judge off %d/8"
            % (pname, out["plain"]["ms_per_problem"], out["plain"]["cycles_total"], out["learned"]["ms_per_problem"],
               out["learned"]["cycles_total"], out["learned"]["net_cycles"], out["learned"]["judge_switched_off"]))
        res[pname] = out
    del fs
    torch.cuda.empty_cache()
    return res


def bench_cube(dmg, workloads, dev, torch, args, ref=None):
    """3D unit cube 257^3 (h = 1/256), f ~ U(-1,1) (seed 3), tuned 3D
    parameters; FP64 against single-precision cycles, both to 1e-10."""
    n = 256
    f = torch.from_numpy(workloads.cube_uniform(n, seed=3)).to(dev)
    res = {"workload": "3D unit cube 257^3, f ~ U(-1,1) (seed 3), p = (1.11, 1.42, 1.08, 0.99), to %.0e" % args.rtol,
           "unknowns": (n - 1) ** 3}
    for name, prec in (("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)):
        S = dmg.Solver(3, n, precision=prec, device=dev)
        us = [torch.zeros_like(f) for _ in range(args.steps + args.warmup)]
        for k in range(args.warmup):
            S.solve(us[k], f, rtol=args.rtol, max_cycles=60)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            st, cyc, rr, hist = S.solve(us[k], f, rtol=args.rtol, max_cycles=60)
            assert st == 0 and rr <= args.rtol, (st, rr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"ms_to_rtol": round(1e3 * dt / args.steps, 3), "cycles": cyc,
                     "unknowns_cycles_per_s": (n - 1) ** 3 * cyc * args.steps / dt, "final_rel_res": rr}
        if ref is not None:
            res[name]["err_vs_oracle"] = err_vs(us[-1], ref)
        if name == "fp64":
            res["kernels3d"] = kernel_table(S, f, max(args.steps, 5), torch)
        log("  cube257 %s: %.3f ms, %d cycles" % (name, res[name]["ms_to_rtol"], cyc))
        S.close()
        del S, us
        torch.cuda.empty_cache()
    return res


def oracle_solve_timed(O, f_host, p, rtol, runs):
    """The CPU oracle's FP64 solve of one workload from u = 0, `runs` times:
    (solution, cycles, median seconds, all times)."""
    import numpy as np
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        uo, co, ro, ho, so = O.solve(np.zeros_like(f_host), f_host, p=p, rtol=rtol, max_cycles=60)
        times.append(time.perf_counter() - t0)
        assert so == O.OK, so
    return uo, co, ro, float(np.median(times)), [round(t, 3) for t in times]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--family", type=int, default=-1,
                    help="kernel family for the roofline (-1: the single-kernel family that takes the most time)")
    ap.add_argument("--cpu-runs", type=int, default=3, help="oracle runs per CPU-baseline leg (median reported)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (CPU baseline and errors against it)")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the 4097^2 modes (no comparison cycles, batched, fourth-order or 3D workloads)")
    ap.add_argument("--no-learned", action="store_true", help="skip training and the learned modes")
    ap.add_argument("--cube-only", action="store_true", help="only the 3D 257^3 workload (for profiling)")
    ap.add_argument("--fourth-only", action="store_true", help="only the fourth-order solves of the 2D workload")
    ap.add_argument("--retune-only", action="store_true", help="only the re-tuned parameter solves")
    ap.add_argument("--batched-only", action="store_true", help="only the 512-problem batched workload")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path (a single grid is "
              "solved on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_math_9907190_amd import dmg, learned, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        nb = args.copy_probe << 20
        a = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nb, "copy_probe_bytes_written": nb, "launches": 5}), flush=True)
        return
    if args.cube_only:
        print(json.dumps({"cube257": bench_cube(dmg, workloads, dev, torch, args)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched512": bench_batched(dmg, workloads, dev, torch, args)}), flush=True)
        return
    n = args.n
    unknowns = (n - 1) ** 2
    log("generating f (n=%d)" % n)
    f_host = workloads.square_modes_noise(n, seed=2)
    f = torch.from_numpy(f_host).to(dev)
    if args.retune_only:
        f3 = torch.from_numpy(workloads.cube_uniform(256, seed=3)).to(dev)
        print(json.dumps({"retuned%d" % (n + 1): bench_retuned(dmg, f, dev, torch, args),
                          "retuned_cube257": bench_retuned(dmg, f3, dev, torch, args)}), flush=True)
        return
    if args.fourth_only:
        f3 = torch.from_numpy(workloads.cube_uniform(256, seed=3)).to(dev)
        print(json.dumps({"fourth_order%d" % (n + 1): bench_fourth_order(dmg, f, dev, torch, args),
                          "fourth_order_cube257": bench_fourth_order(dmg, f3, dev, torch, args)}), flush=True)
        return

    # The CPU oracle first: its FP64 solutions are the references every GPU
    # result's error is stated against, and its timings the CPU baseline.
    refs = {}
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        O.build(force=False)
        log("cpu oracle: FP64 solve of the %d^2 workload to %.0e, %d runs (single thread)" % (n + 1, args.rtol,
                                                                                          args.cpu_runs))
        uo, co, ro, med, times = oracle_solve_timed(O, f_host, (1.052,), args.rtol, args.cpu_runs)
        refs["square"] = uo
        legs = [{"workload": "2D %d^2 (this line's workload), FP64 solve to %.0e" % (n + 1, args.rtol),
                 "cycles": co, "final_rel_res": ro, "median_s": round(med, 3), "runs_s": times,
                 "unknowns_cycles_per_s": unknowns * co / med}]
        cpu = {"value": unknowns * co / med, "unit": "unknowns*cycles/s", "cores": 1, "kind": "oracle",
               "sample": "full FP64 solves of the %d^2 workload to %.0e (%d cycles), median of %d runs, one thread"
                         % (n + 1, args.rtol, co, args.cpu_runs)}
        if not args.no_extra:
            f3_host = workloads.cube_uniform(256, seed=3)
            log("cpu oracle: FP64 solve of the 257^3 workload, %d runs" % args.cpu_runs)
            uo3, co3, ro3, med3, times3 = oracle_solve_timed(O, f3_host, dmg.P3D_TUNED, args.rtol, args.cpu_runs)
            refs["cube"] = uo3
            legs.append({"workload": "3D 257^3, f ~ U(-1,1) (seed 3), FP64 solve to %.0e" % args.rtol, "cycles": co3,
                         "final_rel_res": ro3, "median_s": round(med3, 3), "runs_s": times3,
                         "unknowns_cycles_per_s": 255 ** 3 * co3 / med3})
            log("cpu oracle: fourth-order reference solutions (2D and 3D, untimed)")
            refs["square_o4"] = O.solve(np.zeros_like(f_host), f_host, p=dmg.P2D_H4, rtol=args.rtol, max_cycles=60,
                                        order=4)[0]
            refs["cube_o4"] = O.solve(np.zeros_like(f3_host), f3_host, p=dmg.P3D_H4, rtol=args.rtol, max_cycles=60,
                                      order=4)[0]
            del f3_host
        cpu.update(cpu_info())
        cpu["legs"] = legs

    w_net = net_info = None
    if not args.no_learned:
        log("learned coarse correction: training pairs and training")
        w_net, net_info = train_net(dmg, learned, torch, log)

    # per-family kernel times of the FP64 cycle; the roofline follows the
    # single-kernel family (residual or finest Jacobi) that takes the most time
    S = dmg.Solver(2, n, precision=dmg.MG_FP64, p=(1.052,), device=dev)
    ktab = kernel_table(S, f, max(args.steps, 5), torch)
    S.close()
    del S
    family = args.family
    if family < 0:
        single = [r for r in ktab if r["family_id"] in (dmg.MG_K_RESIDUAL, dmg.MG_K_FINEST)]
        family = max(single, key=lambda r: r["us_per_cycle"])["family_id"]

    modes = {}
    roof = None
    main_val = None
    ms_per_step = None
    forms = [("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)]
    if w_net is not None:
        forms += [("learned_fp64", dmg.MG_FP64), ("learned_fp32_refined", dmg.MG_FP32_REFINED)]
    for name, prec in forms:
        S = dmg.Solver(2, n, precision=prec, p=(1.052,), device=dev)
        if name.startswith("learned"):
            S.set_coarse_net(w_net)
        fam = family if name == "fp64" else None
        log("mode %s: %d warmup + %d timed solves" % (name, args.warmup, args.steps))
        dt, cycles, kern, u_last, hist = timed_solves(S, f, args.steps, args.warmup, args.rtol, fam, torch)
        ms = 1e3 * dt / args.steps
        ucs = unknowns * sum(cycles) / dt
        modes[name] = {"ms_to_rtol": round(ms, 4), "cycles": cycles[-1], "unknowns_cycles_per_s": ucs,
                       "final_rel_res": hist[-1]}
        if "square" in refs:
            modes[name]["err_vs_oracle"] = err_vs(u_last, refs["square"])
        if name.startswith("learned"):
            used, off, qn, qp = S.net_stats()
            modes[name].update({"net_cycles": used, "judge_switched_off": off, "first_cycle_cut_ratio_net": qn,
                                "first_cycle_cut_ratio_plain": qp})
        log("  %s: %.3f ms per solve, %d cycles, %.3e unknowns*cycles/s%s"
            % (name, ms, cycles[-1], ucs, ", error vs oracle %.2e" % modes[name]["err_vs_oracle"]["inf"]
               if "err_vs_oracle" in modes[name] else ""))
        if name == "fp64":
            main_val, ms_per_step = ucs, ms
            kms, kcount, kbytes = kern
            # a solve also launches one gated no-op iteration after the last
            # cycle; bytes count only launches that ran (their few-us no-op
            # time stays in kms, so the figure errs low)
            work = sum(cycles) + (args.steps if family == dmg.MG_K_RESIDUAL else 0)
            if kcount > 0 and work > 0:
                bpl = kbytes / kcount
                achieved = bpl * work / (kms * 1e-3) / 1e9
                traffic = measured_traffic(family)
                roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "kernel": FAMILY_KERNELS[2][family], "family": FAMILY_NAMES[family],
                        "bytes_per_launch": bpl, "us_per_launch": round(kms / work * 1e3, 2),
                        "launches": work, "launches_enqueued": kcount}
        S.close()
        del S
        torch.cuda.empty_cache()
    for k in [m for m, _ in forms[1:]]:
        modes[k]["speedup_vs_fp64"] = round(modes["fp64"]["ms_to_rtol"] / modes[k]["ms_to_rtol"], 3)

    extra = {}
    if not args.no_extra:
        log("conventional comparison cycle on the same workload")
        extra["usual%d" % (n + 1)] = bench_usual(dmg, f, dev, torch, args,
                                                 {k: modes[k]["ms_to_rtol"] for k in ("fp64", "fp32_refined")},
                                                 refs.get("square"))
        log("more sweeps per level and W-cycles on the same workload")
        extra["cycles%d" % (n + 1)] = bench_cycles(dmg, f, dev, torch, args, modes["fp64"]["ms_to_rtol"],
                                                   refs.get("square"))
        log("fourth-order residual: direct and two-stage solves")
        extra["fourth_order%d" % (n + 1)] = bench_fourth_order(dmg, f, dev, torch, args, refs.get("square_o4"))
        extra["batched512"] = bench_batched(dmg, workloads, dev, torch, args, not args.no_cpu)
        if w_net is not None:
            extra["learned1025"] = bench_learned(dmg, learned, dev, torch, args, w_net, net_info, not args.no_cpu)
            log("learned coarse correction in 3D: pairs, training, held-out solves")
            extra["learned129_3d"] = bench_learned3d(dmg, learned, dev, torch, args, not args.no_cpu)
        extra["cube257"] = bench_cube(dmg, workloads, dev, torch, args, refs.get("cube"))
        f3 = torch.from_numpy(workloads.cube_uniform(256, seed=3)).to(dev)
        log("conventional comparison cycle on the cube")
        extra["usual_cube257"] = bench_usual(dmg, f3, dev, torch, args,
                                             {k: extra["cube257"][k]["ms_to_rtol"] for k in ("fp64", "fp32_refined")},
                                             refs.get("cube"))
        log("more sweeps per level and W-cycles on the cube")
        extra["cycles_cube257"] = bench_cycles(dmg, f3, dev, torch, args, extra["cube257"]["fp64"]["ms_to_rtol"],
                                               refs.get("cube"))
        del f3
        log("fourth-order residual in 3D: direct and two-stage solves")
        f3 = torch.from_numpy(workloads.cube_uniform(256, seed=3)).to(dev)
        extra["fourth_order_cube257"] = bench_fourth_order(dmg, f3, dev, torch, args, refs.get("cube_o4"))
        log("over-relaxation re-tuned per size: 4097^2 and 257^3")
        extra["retuned%d" % (n + 1)] = bench_retuned(dmg, f, dev, torch, args, refs.get("square"))
        extra["retuned_cube257"] = bench_retuned(dmg, f3, dev, torch, args, refs.get("cube"))
        del f3

    out = {"metric": METRIC, "value": main_val, "unit": "unknowns*cycles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2D unit square %dx%d (h=1/%d), f = 16 seeded sine modes + 1e-3 noise, "
                                  "p=1.052, solve from u=0 to %.0e rel. residual" % (n + 1, n + 1, n, args.rtol),
                      "unknowns": unknowns, "grid": n + 1, "rtol": args.rtol},
           "modes": modes, "roofline": roof, "kernels2d": ktab, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

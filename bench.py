#!/usr/bin/env python3
"""Benchmark of the diagonally oriented multigrid solver (libdmg) on one GPU.

Workload: 2D unit square, 4097 x 4097 grid (h = 1/4096, 16,769,025 unknowns),
zero Dirichlet data, f = 16 seeded sine modes with N(0,1) amplitudes and
wavenumbers U{1..64} plus 1e-3 white noise (seed 2), p = 1.052.

One step = one solve from u = 0 to a relative residual of 1e-10 with the
plain FP64 V-cycle: residual, the whole restriction hierarchy, the coarse
levels, the Jacobi prolongation and the on-device convergence check, every
cycle.  value = unknowns * cycles / second over the timed steps.  The same
workload is also solved with the single-precision cycle plus FP64 refinement;
the time to 1e-10 of each form is reported under "modes".

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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_solves(S, f, steps, warmup, rtol, family, torch):
    n1 = f.shape[0]
    us = [torch.zeros((n1, n1), dtype=torch.float64, device=f.device) for _ in range(steps + warmup)]
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


def bench_batched(dmg, workloads, dev, torch, args):
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
    log("  batched: %.3f ms per batch solve, cycles %d..%d, %.3e unknowns*cycles/s"
        % (res["ms_to_rtol"], min(cyc), max(cyc), res["unknowns_cycles_per_s"]))
    B.close()
    del us, fs, B
    torch.cuda.empty_cache()
    return res


def bench_cube(dmg, workloads, dev, torch, args):
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
        log("  cube257 %s: %.3f ms, %d cycles" % (name, res[name]["ms_to_rtol"], cyc))
        S.close()
        del S, us
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--family", type=int, default=3, help="kernel family for the roofline (3: finest Jacobi)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and 3D workloads")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path (a single grid is "
              "solved on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_math_9907190_amd import dmg, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = args.n
    unknowns = (n - 1) ** 2
    log("generating f (n=%d)" % n)
    f_host = workloads.square_modes_noise(n, seed=2)
    f = torch.from_numpy(f_host).to(dev)

    modes = {}
    roof = None
    main_val = None
    ms_per_step = None
    for name, prec in (("fp64", dmg.MG_FP64), ("fp32_refined", dmg.MG_FP32_REFINED)):
        S = dmg.Solver(2, n, precision=prec, p=(1.052,), device=dev)
        fam = args.family if prec == dmg.MG_FP64 else None
        log("mode %s: %d warmup + %d timed solves" % (name, args.warmup, args.steps))
        dt, cycles, kern, u_last, hist = timed_solves(S, f, args.steps, args.warmup, args.rtol, fam, torch)
        ms = 1e3 * dt / args.steps
        ucs = unknowns * sum(cycles) / dt
        modes[name] = {"ms_to_rtol": round(ms, 4), "cycles": cycles[-1], "unknowns_cycles_per_s": ucs,
                       "final_rel_res": hist[-1]}
        log("  %s: %.3f ms per solve, %d cycles, %.3e unknowns*cycles/s" % (name, ms, cycles[-1], ucs))
        if prec == dmg.MG_FP64:
            main_val, ms_per_step = ucs, ms
            kms, kcount, kbytes = kern
            if kcount > 0:
                per_launch_s = kms / kcount * 1e-3
                achieved = kbytes / kcount / per_launch_s / 1e9
                roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": FAMILY_NAMES.get(args.family, str(args.family)),
                        "bytes_per_launch": kbytes / kcount, "us_per_launch": round(kms / kcount * 1e3, 2),
                        "launches": kcount}
        S.close()
        del S
        torch.cuda.empty_cache()
    modes["fp32_refined"]["speedup_vs_fp64"] = round(modes["fp64"]["ms_to_rtol"] / modes["fp32_refined"]["ms_to_rtol"], 3)

    extra = {}
    if not args.no_extra:
        extra["batched512"] = bench_batched(dmg, workloads, dev, torch, args)
        extra["cube257"] = bench_cube(dmg, workloads, dev, torch, args)

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        O.build(force=False)
        log("cpu oracle: one FP64 solve of the same workload to %.0e (single thread)" % args.rtol)
        t0 = time.perf_counter()
        uo, co, ro, ho, so = O.solve(np.zeros_like(f_host), f_host, p=(1.052,), rtol=args.rtol, max_cycles=60)
        dt = time.perf_counter() - t0
        cpu = {"value": unknowns * co / dt, "unit": "unknowns*cycles/s", "cores": 1, "kind": "oracle",
               "sample": "one full FP64 solve of the %d^2 workload to %.0e (%d cycles, %.2f s), one thread"
                         % (n + 1, args.rtol, co, dt)}

    out = {"metric": METRIC, "value": main_val, "unit": "unknowns*cycles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2D unit square %dx%d (h=1/%d), f = 16 seeded sine modes + 1e-3 noise, "
                                  "p=1.052, solve from u=0 to %.0e rel. residual" % (n + 1, n + 1, n, args.rtol),
                      "unknowns": unknowns, "grid": n + 1, "rtol": args.rtol},
           "modes": modes, "roofline": roof, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

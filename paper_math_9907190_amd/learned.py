"""Learned coarse correction: training pairs, training, evaluation helpers.

Orchestration only: every arithmetic step runs in libdmg's kernels.

* Pairs (r_c, e_c) of the cut level (aligned level 6: the 17 x 17 axis grid
  of a 2D problem) come from the plain FP64 V-cycle: a batch of problems is
  cycled from u = 0, and after every cycle the cut level's restricted
  residual r_c is exported.  The target e_c = A_c^{-1} r_c is the solution of
  the 17 x 17 Poisson problem with right-hand side r_c, solved by the same
  library (batched, FP64) to a relative residual of 1e-13.
* Training: Adam on the normalised pairs (libdmg's bf16 forward/backward
  kernels, FP32 master weights), either towards e_c (mean squared error) or
  on the cut-level objective the coarse kernel judges the network by: the
  cut level's residual after its own Jacobi step from the network's output.
"""
import concurrent.futures as cf

import numpy as np
import torch

from . import dmg, workloads

CUT = dmg.MG_NET_CUT


def _rhs_batch(n, seeds, threads=8, dim=2):
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda s: workloads.training_rhs(dim, n, s), seeds))


def make_pairs(n=1024, seeds=range(1000, 2250), cycles=8, chunk=125, device=None, target_rtol=1e-13, log=None):
    """(r, e): float64 device tensors of shape (len(seeds) * cycles, 17, 17)."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    seeds = list(seeds)
    rs = []
    for c0 in range(0, len(seeds), chunk):
        sl = seeds[c0:c0 + chunk]
        if log:
            log("pairs: problems %d..%d of %d (n=%d)" % (c0, c0 + len(sl) - 1, len(seeds), n))
        fs = [torch.from_numpy(f).to(device) for f in _rhs_batch(n, sl)]
        us = [torch.zeros_like(f) for f in fs]
        B = dmg.BatchSolver([n] * len(sl), precision=dmg.MG_FP64, device=device)
        for _ in range(cycles):
            B.vcycle(us, fs)
            rs.append(B.coarse_export(CUT))
        B.close()
        del B, us, fs
    r = torch.cat(rs).contiguous()
    e = solve_cut(r, target_rtol, device)
    return r, e


def solve_cut(r, rtol=1e-13, device=None):
    """e = A_c^{-1} r for each 17 x 17 grid of r (FP64 batched solve)."""
    P = r.shape[0]
    G = r.shape[-1]
    e = torch.zeros_like(r)
    T = dmg.BatchSolver([G - 1] * P, precision=dmg.MG_FP64, device=device or r.device)
    st, cyc, rr, sts = T.solve([e[i] for i in range(P)], [r[i] for i in range(P)], rtol=rtol, max_cycles=60)
    T.close()
    bad = [i for i, s in enumerate(sts) if s != dmg.MG_OK and rr[i] > 1e-12]
    if bad:
        raise RuntimeError("target solves failed for %d pairs (first %d: status %d)" % (len(bad), bad[0], sts[bad[0]]))
    return e


def make_pairs_3d(n=128, seeds=range(1000, 1250), cycles=8, device=None, target_rtol=1e-13, log=None):
    """3D pairs: the cut is the green grid of side 8 (9^3 points); one plain
    FP64 solve per right-hand side, the cut residual exported after every
    cycle, targets from FP64 solves of the 9^3 problems.  Shapes (P, 9, 9, 9)."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    seeds = list(seeds)
    S = dmg.Solver(3, n, precision=dmg.MG_FP64, device=device)
    rs = []
    chunk = 64
    for c0 in range(0, len(seeds), chunk):
        if log:
            log("pairs 3D: problems %d..%d of %d (n=%d)" % (c0, min(c0 + chunk, len(seeds)) - 1, len(seeds), n))
        for fh in _rhs_batch(n, seeds[c0:c0 + chunk], dim=3):
            f = torch.from_numpy(fh).to(device)
            u = torch.zeros_like(f)
            for _ in range(cycles):
                S.vcycle(u, f)
                rs.append(S.coarse_export(CUT).clone())
    S.close()
    r = torch.stack(rs).contiguous()
    e = torch.zeros_like(r)
    T = dmg.Solver(3, r.shape[-1] - 1, precision=dmg.MG_FP64, device=device)
    for i in range(r.shape[0]):
        st, cyc, rr, _ = T.solve(e[i], r[i], rtol=target_rtol, max_cycles=60)
        if st != dmg.MG_OK and rr > 1e-12:
            raise RuntimeError("target solve %d failed: status %d" % (i, st))
    T.close()
    return r, e


# staged Adam learning rates (epochs, lr): measured on the 3D cut, the decay
# takes the network from losing to the plain sub-cycle to beating it
SCHEDULE = ((120, 2e-3), (60, 5e-4), (60, 1.25e-4), (100, 3e-5))


def cut_p(dim, p=None):
    """the cut level's over-relaxation parameter: 2D p, 3D p_g (the green
    level's); the library's defaults unless p is given"""
    p = p if p is not None else (dmg.P2D_TUNED if dim == 2 else dmg.P3D_TUNED)
    return float(p[0] if dim == 2 else p[3])


def train(r, e, epochs=30, batch=256, lr=2e-3, seed=7, init_seed=1, net=None, schedule=None, loss="mse", pj=None):
    """Train (or continue training) a network on the pairs; returns (net,
    epoch losses).  schedule: ((epochs, lr), ...) run in order (Adam state
    carried over), instead of epochs at one lr.  loss "mse": towards the
    targets e; "cut": the cut level's residual after its own Jacobi step from
    the network's output (e is not used; pj defaults to cut_p)."""
    dim = r.dim() - 1
    if net is None:
        net = dmg.Net(dim=dim, max_batch=batch, seed=init_seed, device=r.device)
    if loss == "cut":
        net.set_loss(dmg.MG_NET_LOSS_CUT, cut_p(dim) if pj is None else pj)
        e = None
    elif loss == "mse":
        net.set_loss(dmg.MG_NET_LOSS_MSE)
    else:
        raise ValueError("loss must be 'mse' or 'cut'")
    hist = []
    for k, (ep, rate) in enumerate(schedule or ((epochs, lr),)):
        hist += net.train(r, e, epochs=ep, batch=batch, lr=rate, seed=seed + 7919 * k)
    return net, hist


def cut_objective(w, r, batch=256, pj=None):
    """Mean over the pairs' residuals r of the cut-level objective for the
    weights w (mean rho^2 with r normalised to unit rms: the square of the
    cut level's residual reduction, averaged over samples)."""
    dim = r.dim() - 1
    net = dmg.Net(dim=dim, max_batch=batch, device=r.device)
    net.set_weights(w)
    net.set_loss(dmg.MG_NET_LOSS_CUT, cut_p(dim) if pj is None else pj)
    tot, cnt = 0.0, 0
    for i in range(0, r.shape[0], batch):
        rb = r[i:i + batch]
        tot += net.loss_grad(rb, None, normalize=True)[0] * rb.shape[0]
        cnt += rb.shape[0]
    net.close()
    return tot / cnt


def eval_problems(n=1024, seeds=range(5000, 5032), dim=2):
    """Held-out right-hand sides (host arrays)."""
    return _rhs_batch(n, list(seeds), dim=dim)

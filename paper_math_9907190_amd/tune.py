"""Over-relaxation parameters re-tuned per grid size (Sections 2.4 and 3.4).

The paper minimised the V-cycle's factor of convergence over the
over-relaxation parameters with the Nelder-Mead simplex method, on a 65^2
grid (2D, one parameter p) and a 17^3 grid (3D, p_m, p_r1, p_r2, p_g), and
notes that finer 3D grids were out of its reach.  Here the same search runs on
the GPU cycle at any size the library solves.

Factor of a parameter set: power iteration of the cycle's error map.  With
f = 0 a cycle maps u to (I - M A) u; mg_vcycle reports ||r(u)||_2 = ||A u||_2
before each cycle (its relative residual when f = 0), and the ratio of
successive residual norms tends to the spectral radius of A (I - M A) A^-1,
the same as that of the error map.  The factor is the geometric mean of the
last `tail` ratios of `cycles` cycles from a seeded U(-1, 1) start, so that a
complex pair of dominant eigenvalues does not make it oscillate.  Each
evaluation builds a plan with those parameters (they are part of the plan's
level coefficients).

Host-side driver only: every cycle and residual norm runs in libdmg.
"""
import numpy as np

from . import dmg as D
from . import workloads as W


def nelder_mead(factor, p0, xatol=2e-3, fatol=1e-4, maxfev=200):
    """Minimise factor(p) from p0 with the Nelder-Mead simplex method.
    Returns (p, factor(p), evaluations)."""
    from scipy.optimize import minimize

    res = minimize(lambda p: factor(tuple(float(x) for x in p)), np.asarray(p0, dtype=np.float64),
                   method="Nelder-Mead", options={"xatol": xatol, "fatol": fatol, "maxfev": maxfev})
    return tuple(float(x) for x in res.x), float(res.fun), int(res.nfev)


def tail_factor(norms, tail):
    """Geometric mean of the last `tail` ratios of a residual-norm history."""
    r = np.asarray(norms, dtype=np.float64)
    return float((r[-1] / r[-1 - tail]) ** (1.0 / tail))


def gpu_factor(dim, n, p, precision=D.MG_FP64, cycles=30, tail=10, seed=0, device=None, nu=None, gamma=None,
               scheme="diagonal"):
    """Factor of the cycle with parameters p on the GPU (see the module text);
    nu / gamma: the generalised diagonal cycle; scheme "usual": the
    conventional comparison cycle."""
    import torch

    if not 1 <= tail <= cycles:
        raise ValueError("need 1 <= tail <= cycles")
    S = D.Solver(dim, n, precision=precision, p=p, device=device, nu=nu, gamma=gamma, scheme=scheme)
    try:
        u = torch.from_numpy(W.uniform(dim, n, seed)).to(S.device)
        f = torch.zeros_like(u)
        norms = [S.vcycle(u, f, want_relres=True) for _ in range(cycles + 1)]
    finally:
        S.close()
    return tail_factor(norms, tail)


def tune_p(dim, n, p0=None, precision=D.MG_FP64, cycles=30, tail=10, seed=0, maxfev=200, device=None, nu=None,
           gamma=None):
    """Parameters minimising the GPU cycle's factor at this size, from p0
    (default: the paper's tuned values).  Returns (p, factor, evaluations)."""
    if p0 is None:
        p0 = D.P2D_TUNED if dim == 2 else D.P3D_TUNED

    def factor(p):
        if min(p) <= 0:
            return 1e3   # outside the parameters' domain
        return gpu_factor(dim, n, p, precision, cycles, tail, seed, device, nu, gamma)

    return nelder_mead(factor, p0, maxfev=maxfev)

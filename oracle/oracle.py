"""ctypes wrapper of the CPU oracle (``orc_mg.c``, ``orc_net.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain double-precision CPU
reference of the diagonally oriented multigrid V-cycle (Roberts, Sections 1-3)
that the GPU library is checked against.  Only ``tests/``, the smoke check and
the CPU-baseline leg of the benchmark import this module; the GPU package never
does, and the two share no code.

Arrays are numpy float64 in natural order, shape ``(n+1, n+1)`` or
``(n+1, n+1, n+1)`` indexed ``[y, x]`` / ``[z, y, x]`` (x fastest), zero
Dirichlet boundary.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
_lib = None

OK, ERR_ARG, ERR_SIZE, ERR_ALLOC, ERR_NONFINITE, ERR_DIVERGED, ERR_NOT_CONVERGED = 0, -1, -2, -4, -6, -7, -8

# over-relaxation parameters the paper tunes: 2D p (Section 2.4, Table tbl:2d);
# 3D (p_m, p_r1, p_r2, p_g) (Section 3.4, Table tbl:3dopt)
P2D_TUNED = (1.052,)
P3D_TUNED = (1.11, 1.42, 1.08, 0.99)
# tuned for the fourth-order residuals: 2D p = 1.20 (Section 2.4, Table
# tbl:2d); 3D (Section 3.4, Table tbl:3dopt)
P2D_H4 = (1.20,)
P3D_H4 = (0.91, 0.80, 0.70, 1.77)


def build(force=True):
    """Compile ``liborc.so`` with gcc (plain -O2, no FP contraction)."""
    srcs = [os.path.join(_HERE, f) for f in ("orc_mg.c", "orc_net.c")]
    deps = srcs + [os.path.join(_HERE, "orc_mg_body.h")]
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= max(os.path.getmtime(d) for d in deps):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i, d = ctypes.c_int, ctypes.c_double
        L.orc_residual.argtypes = [i, i, dp, dp, dp]
        L.orc_relres.argtypes = [i, i, dp, dp, dp]
        L.orc_vcycle.argtypes = [i, i, dp, i, dp, dp]
        L.orc_vcycle_trace.argtypes = [i, i, dp, i, dp, dp, dp, dp]
        L.orc_solve.argtypes = [i, i, dp, i, dp, dp, d, i, ip, dp, dp]
        L.orc_residual_ord.argtypes = [i, i, i, dp, dp, dp]
        L.orc_relres_ord.argtypes = [i, i, i, dp, dp, dp]
        L.orc_vcycle_ord_trace.argtypes = [i, i, dp, i, i, dp, dp, dp, dp]
        L.orc_solve_ord.argtypes = [i, i, dp, i, i, dp, dp, d, i, ip, dp, dp]
        L.orc_vcycle_usual.argtypes = [i, i, d, i, i, dp, dp, dp, dp]
        L.orc_solve_usual.argtypes = [i, i, d, i, i, dp, dp, d, i, ip, dp, dp]
        L.orc_cycle_gen.argtypes = [i, i, dp, i, i, i, i, dp, dp, dp, dp]
        L.orc_solve_gen.argtypes = [i, i, dp, i, i, i, i, dp, dp, d, i, ip, dp, dp]
        L.orc_step_restrict.argtypes = [i, i, i, dp, dp]
        L.orc_step_jacobi.argtypes = [i, i, i, dp, dp, dp, dp]
        for fn in ("orc_residual", "orc_relres", "orc_vcycle", "orc_vcycle_trace", "orc_solve",
                   "orc_residual_ord", "orc_relres_ord", "orc_vcycle_ord_trace", "orc_solve_ord",
                   "orc_step_restrict", "orc_step_jacobi", "orc_vcycle_usual", "orc_solve_usual",
                   "orc_cycle_gen", "orc_solve_gen"):
            getattr(L, fn).restype = ctypes.c_int
        L.orc_net_forward.argtypes = [i, i, dp, dp, dp]
        L.orc_net_forward.restype = ctypes.c_int
        L.orc_net_loss_grad.argtypes = [i, i, dp, dp, dp, dp]
        L.orc_net_loss_grad.restype = ctypes.c_double
        L.orc_net_judge_loss_grad.argtypes = [i, i, dp, dp, d, dp]
        L.orc_net_judge_loss_grad.restype = ctypes.c_double
        L.orc_net_adam.argtypes = [i, dp, dp, dp, dp, i, d, d, d, d]
        L.orc_net_adam.restype = None
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dimn(a):
    return a.ndim, a.shape[0] - 1


def _params(dim, p):
    if p is None:
        p = P2D_TUNED if dim == 2 else P3D_TUNED
    p = np.ascontiguousarray(np.atleast_1d(np.asarray(p, dtype=np.float64)))
    assert p.size == (1 if dim == 2 else 4)
    return p


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with code %d" % (what, code))
        self.code = code


def _chk(code, what):
    if code != OK:
        raise OracleError(code, what)


def level_sides(dim, n):
    """Side m of each level's array, in depth order (finest first)."""
    K = int(round(np.log2(n)))
    D = (2 if dim == 2 else 3) * (K - 1)
    return [n >> (d // dim) for d in range(D + 1)]


def residual(u, f, order=2):
    """Finest residual: order 2, f - Lap_h u (Eq. Evpois); order 4, Eq. Efos2 / Efos4."""
    dim, n = _dimn(u)
    r = np.zeros_like(u)
    _chk(lib().orc_residual_ord(dim, n, order, _ptr(u), _ptr(f), _ptr(r)), "orc_residual_ord")
    return r


def relres(u, f, order=2):
    """||r(u)|| / ||r(0)|| over interior nodes for the residual of that order."""
    dim, n = _dimn(u)
    out = ctypes.c_double()
    _chk(lib().orc_relres_ord(dim, n, order, _ptr(u), _ptr(f), ctypes.byref(out)), "orc_relres_ord")
    return out.value


def vcycle(u, f, p=None, prec=0, order=2):
    """One V-cycle; returns the new u (the input is not modified)."""
    dim, n = _dimn(u)
    u = np.array(u, dtype=np.float64, order="C")
    _chk(lib().orc_vcycle_ord_trace(dim, n, _ptr(_params(dim, p)), prec, order, _ptr(u), _ptr(f), None, None),
         "orc_vcycle_ord_trace")
    return u


def vcycle_trace(u, f, p=None, prec=0, order=2):
    """One V-cycle; returns (u_new, [r per level], [v per level])."""
    dim, n = _dimn(u)
    sides = level_sides(dim, n)
    sizes = [(m + 1) ** dim for m in sides]
    rt = np.zeros(sum(sizes))
    vt = np.zeros(sum(sizes))
    u = np.array(u, dtype=np.float64, order="C")
    _chk(lib().orc_vcycle_ord_trace(dim, n, _ptr(_params(dim, p)), prec, order, _ptr(u), _ptr(f), _ptr(rt),
                                    _ptr(vt)), "orc_vcycle_ord_trace")
    rs, vs, off = [], [], 0
    for m, s in zip(sides, sizes):
        rs.append(rt[off:off + s].reshape((m + 1,) * dim))
        vs.append(vt[off:off + s].reshape((m + 1,) * dim))
        off += s
    return u, rs, vs


def solve(u, f, p=None, prec=0, rtol=1e-10, max_cycles=50, check=True, order=2):
    """Returns (u, cycles, relres, history, status); relres of the given order."""
    dim, n = _dimn(u)
    u = np.array(u, dtype=np.float64, order="C")
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int()
    rr = ctypes.c_double()
    st = lib().orc_solve_ord(dim, n, _ptr(_params(dim, p)), prec, order, _ptr(u), _ptr(f), rtol, max_cycles,
                             ctypes.byref(cyc), ctypes.byref(rr), _ptr(hist))
    if check and st not in (OK, ERR_NOT_CONVERGED):
        raise OracleError(st, "orc_solve_ord")
    return u, cyc.value, rr.value, hist[:cyc.value + 1], st


def solve_two_stage(u, f, p2=None, p4=None, prec=0, rtol1=1e-6, rtol=1e-10, max_cycles=50):
    """Fourth-order solution in two stages (Sections 2.3 and 3.3): cycles on
    the second-order residual until its relative residual is <= rtol1, then
    cycles on the fourth-order residual (with the parameters tuned for it)
    until that one's is <= rtol.  Returns (u, cycles1, cycles2, relres4)."""
    dim, _ = _dimn(u)
    if p2 is None:
        p2 = P2D_TUNED if dim == 2 else P3D_TUNED
    if p4 is None:
        p4 = P2D_H4 if dim == 2 else P3D_H4
    u, c1, _, _, _ = solve(u, f, p2, prec, rtol1, max_cycles, order=2)
    u, c2, rr, _, _ = solve(u, f, p4, prec, rtol, max_cycles, order=4)
    return u, c1, c2, rr


# --------------------------- more sweeps per level and W-cycles (Section 4)

def cycle_gen(u, f, p=None, nu=1, gamma=1, prec=0, order=2, trace=False):
    """One cycle with nu red-black sweeps per level and gamma coarse visits
    per group of levels (nu = gamma = 1: the V-cycle).  Returns the new u,
    or (u, [r per level], [v per level]) with trace=True."""
    dim, n = _dimn(u)
    u = np.array(u, dtype=np.float64, order="C")
    if not trace:
        _chk(lib().orc_cycle_gen(dim, n, _ptr(_params(dim, p)), prec, order, nu, gamma, _ptr(u), _ptr(f), None, None),
             "orc_cycle_gen")
        return u
    sides = level_sides(dim, n)
    sizes = [(m + 1) ** dim for m in sides]
    rt = np.zeros(sum(sizes))
    vt = np.zeros(sum(sizes))
    _chk(lib().orc_cycle_gen(dim, n, _ptr(_params(dim, p)), prec, order, nu, gamma, _ptr(u), _ptr(f), _ptr(rt),
                             _ptr(vt)), "orc_cycle_gen")
    rs, vs, off = [], [], 0
    for m, s in zip(sides, sizes):
        rs.append(rt[off:off + s].reshape((m + 1,) * dim))
        vs.append(vt[off:off + s].reshape((m + 1,) * dim))
        off += s
    return u, rs, vs


def solve_gen(u, f, p=None, nu=1, gamma=1, prec=0, rtol=1e-10, max_cycles=50, check=True, order=2):
    """Returns (u, cycles, relres, history, status) of the nu / gamma cycle."""
    dim, n = _dimn(u)
    u = np.array(u, dtype=np.float64, order="C")
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int()
    rr = ctypes.c_double()
    st = lib().orc_solve_gen(dim, n, _ptr(_params(dim, p)), prec, order, nu, gamma, _ptr(u), _ptr(f), rtol,
                             max_cycles, ctypes.byref(cyc), ctypes.byref(rr), _ptr(hist))
    if check and st not in (OK, ERR_NOT_CONVERGED):
        raise OracleError(st, "orc_solve_gen")
    return u, cyc.value, rr.value, hist[:cyc.value + 1], st


# ----------------------------------------------- the conventional cycle
# over-relaxation the paper tunes for it: 2D p (Table tbl:2d), 3D p_g
# (Table tbl:3dopt); fourth-order residual: 1.216 (2D), 1.70 (3D)
P2D_USUAL = 1.121
P3D_USUAL = 1.30
P2D_USUAL_H4 = 1.216
P3D_USUAL_H4 = 1.70


def usual_sides(dim, n):
    K = int(round(np.log2(n)))
    return [n >> d for d in range(K)]


def vcycle_usual_trace(u, f, p, prec=0, order=2):
    """One conventional V-cycle (Sections 2.1-2.3, 3.1-3.3); returns
    (u_new, [r per level], [v per level]), finest first."""
    dim, n = _dimn(u)
    sides = usual_sides(dim, n)
    sizes = [(m + 1) ** dim for m in sides]
    rt = np.zeros(sum(sizes))
    vt = np.zeros(sum(sizes))
    u = np.array(u, dtype=np.float64, order="C")
    _chk(lib().orc_vcycle_usual(dim, n, float(p), prec, order, _ptr(u), _ptr(f), _ptr(rt), _ptr(vt)),
         "orc_vcycle_usual")
    rs, vs, off = [], [], 0
    for m, s in zip(sides, sizes):
        rs.append(rt[off:off + s].reshape((m + 1,) * dim))
        vs.append(vt[off:off + s].reshape((m + 1,) * dim))
        off += s
    return u, rs, vs


def vcycle_usual(u, f, p, prec=0, order=2):
    dim, n = _dimn(u)
    u = np.array(u, dtype=np.float64, order="C")
    _chk(lib().orc_vcycle_usual(dim, n, float(p), prec, order, _ptr(u), _ptr(f), None, None), "orc_vcycle_usual")
    return u


def solve_usual(u, f, p, prec=0, rtol=1e-10, max_cycles=100, check=True, order=2):
    """Returns (u, cycles, relres, history, status) of the conventional cycle."""
    dim, n = _dimn(u)
    u = np.array(u, dtype=np.float64, order="C")
    hist = np.zeros(max_cycles + 1)
    cyc = ctypes.c_int()
    rr = ctypes.c_double()
    st = lib().orc_solve_usual(dim, n, float(p), prec, order, _ptr(u), _ptr(f), rtol, max_cycles, ctypes.byref(cyc),
                               ctypes.byref(rr), _ptr(hist))
    if check and st not in (OK, ERR_NOT_CONVERGED):
        raise OracleError(st, "orc_solve_usual")
    return u, cyc.value, rr.value, hist[:cyc.value + 1], st


def step_restrict(dim, kind, fine):
    m = fine.shape[0] - 1
    mc = m // 2 if (dim == 2 and kind in (1, 2)) or (dim == 3 and kind in (2, 3)) else m
    out = np.zeros((mc + 1,) * dim)
    _chk(lib().orc_step_restrict(dim, kind, m, _ptr(np.ascontiguousarray(fine, dtype=np.float64)), _ptr(out)),
         "orc_step_restrict")
    return out


def step_jacobi(dim, kind, c, r, vc):
    m = r.shape[0] - 1
    c = np.ascontiguousarray(np.atleast_1d(np.asarray(c, dtype=np.float64)))
    if c.size < 2:
        c = np.concatenate([c, [0.0]])
    out = np.zeros_like(r)
    _chk(lib().orc_step_jacobi(dim, kind, m, _ptr(c), _ptr(np.ascontiguousarray(r)),
                               _ptr(np.ascontiguousarray(vc)), _ptr(out)), "orc_step_jacobi")
    return out


# ------------------------------------------------------------ network oracle
# Four 3x3 (2D) / 3x3x3 (3D) convolutions, 16 channels, ReLU between, no bias,
# on [B][17][17] or [B][9][9][9] grids (zero boundary); weights
# [4][taps][16][16] (layer, tap, cin, cout), tap = (dy+1)*3+(dx+1) in 2D and
# ((dz+1)*3+(dy+1))*3+(dx+1) in 3D; layer 0 reads cin 0, layer 3 writes cout 0.
NET_G = {2: 17, 3: 9}
NET_TAPS = {2: 9, 3: 27}


def net_shape(dim):
    return (4, NET_TAPS[dim], 16, 16)


def net_forward(inp, w):
    """inp [B][G]^dim -> network output [B][G]^dim (boundary 0)."""
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    dim = inp.ndim - 1
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(net_shape(dim))
    out = np.zeros_like(inp)
    _chk(lib().orc_net_forward(dim, inp.shape[0], _ptr(inp), _ptr(w), _ptr(out)), "orc_net_forward")
    return out


def net_loss_grad(inp, target, w):
    """(loss, dloss/dw) of the mean squared error over interior points."""
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    dim = inp.ndim - 1
    target = np.ascontiguousarray(target, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(net_shape(dim))
    grad = np.zeros(net_shape(dim))
    loss = lib().orc_net_loss_grad(dim, inp.shape[0], _ptr(inp), _ptr(target), _ptr(w), _ptr(grad))
    if not np.isfinite(loss):
        raise OracleError(-1, "orc_net_loss_grad")
    return loss, grad


def net_judge_loss_grad(inp, w, pj):
    """(loss, dloss/dw) of the cut-level objective: the network output at the
    even points goes through the cut level's own red-black Jacobi step (its
    parameter pj) and the loss is the mean squared residual of that level's
    equation, rho = x - L v (spacing 1, the network's units)."""
    inp = np.ascontiguousarray(inp, dtype=np.float64)
    dim = inp.ndim - 1
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(net_shape(dim))
    grad = np.zeros(net_shape(dim))
    loss = lib().orc_net_judge_loss_grad(dim, inp.shape[0], _ptr(inp), _ptr(w), float(pj), _ptr(grad))
    if not np.isfinite(loss):
        raise OracleError(-1, "orc_net_judge_loss_grad")
    return loss, grad


def net_adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays of one shape (step t >= 1)."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_net_adam(w.size, _ptr(w), _ptr(m), _ptr(v), _ptr(g), t, lr, b1, b2, eps)

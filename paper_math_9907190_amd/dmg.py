"""Python binding of libdmg (include/dmg.h): argument marshalling only.

Every function of the C ABI is exposed under the same name; ``Solver`` adds
the plumbing a PyTorch user needs (workspace from the caching allocator,
torch's current stream).  All arithmetic of the V-cycle runs in the HIP
kernels of libdmg.so; there is no CPU path and no fallback: if the library
is missing this module raises on import.
"""
import ctypes
import os

import torch  # loads the HIP runtime libdmg.so binds to (same soname), so it must come first

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmg.so")

MG_OK, MG_ERR_ARG, MG_ERR_SIZE, MG_ERR_WS, MG_ERR_ALLOC, MG_ERR_HIP = 0, -1, -2, -3, -4, -5
MG_ERR_NONFINITE, MG_ERR_DIVERGED, MG_ERR_NOT_CONVERGED, MG_ERR_SCRATCH = -6, -7, -8, -9
MG_STATIC_SCRATCH_BYTES = 64 << 20
MG_FP64, MG_FP32_REFINED = 0, 1
MG_ORDER4 = 0x100   # OR-ed into the precision: fourth-order finest residual (Eqs. Efos2, Efos4)
MG_USUAL = 0x200    # OR-ed into the precision: the conventional comparison cycle (Sections 2.1-2.3, 3.1-3.3)

if not os.path.exists(LIB_PATH):
    raise ImportError("libdmg.so is not built (%s); run __graft_entry__.build() or "
                      "python paper_math_9907190_amd/build.py" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

_vp, _dp, _ip, _sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_size_t
_lib.mg_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_sz)]
_lib.mg_setup.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                          _vp, _sz, _vp]
_lib.mg_vcycle.argtypes = [_vp, _vp, _vp, _dp]
_lib.mg_solve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _ip, _dp, _dp]
_lib.mg_solve_two_stage.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _ip, _ip, _dp]
_lib.mg_level_get.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp]
_lib.mg_level_info.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip]
_lib.mg_destroy.argtypes = [_vp]
_lib.mg_timing_enable.argtypes = [_vp, ctypes.c_int]
_lib.mg_timing_read.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_longlong), _dp]
_lib.mg_batch_workspace_bytes.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.POINTER(_sz)]
_lib.mg_setup_batched.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _ip, ctypes.c_int, ctypes.c_double, _vp, _sz,
                                  _vp]
_lib.mg_solve_batched.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_double, ctypes.c_int,
                                  _ip, _dp, _ip]
_lib.mg_vcycle_batched.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _dp]
_lib.mg_autotune.argtypes = [_vp]
_fp, _ull = ctypes.POINTER(ctypes.c_float), ctypes.c_ulonglong
_lib.mg_net_weight_count.argtypes = [ctypes.c_int]
_lib.mg_net_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_sz)]
_lib.mg_net_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _sz, _vp]
_lib.mg_net_set_weights.argtypes = [_vp, _fp]
_lib.mg_net_get_weights.argtypes = [_vp, _fp]
_lib.mg_net_init.argtypes = [_vp, _ull]
_lib.mg_net_forward.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int]
_lib.mg_net_loss_grad.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _fp, _dp]
_lib.mg_net_train.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float, _ull, _dp]
_lib.mg_net_destroy.argtypes = [_vp]
_lib.mg_net_set_loss.argtypes = [_vp, ctypes.c_int, ctypes.c_double]
_lib.mg_set_coarse_net.argtypes = [_vp, _fp, ctypes.c_int]
_lib.mg_net_stats.argtypes = [_vp, _ip, _ip, _dp, _dp]
_lib.mg_coarse_export.argtypes = [_vp, ctypes.c_int, _vp]
_lib.mg_cycle_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(_sz)]
_lib.mg_setup_cycle.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, _vp, _sz, _vp]
_lib.mg_vcycle_static.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _vp, _vp, _dp, _vp]
_lib.mg_strerror.argtypes = [ctypes.c_int]
_lib.mg_strerror.restype = ctypes.c_char_p
for _f in ("mg_workspace_bytes", "mg_setup", "mg_vcycle", "mg_solve", "mg_solve_two_stage", "mg_level_get", "mg_level_info",
           "mg_destroy", "mg_timing_enable", "mg_timing_read", "mg_batch_workspace_bytes", "mg_setup_batched",
           "mg_solve_batched", "mg_vcycle_batched", "mg_autotune", "mg_net_weight_count", "mg_net_workspace_bytes",
           "mg_net_create", "mg_net_set_weights", "mg_net_get_weights", "mg_net_init", "mg_net_forward",
           "mg_net_loss_grad", "mg_net_train", "mg_net_destroy", "mg_set_coarse_net", "mg_net_stats",
           "mg_coarse_export", "mg_vcycle_static", "mg_cycle_workspace_bytes", "mg_setup_cycle", "mg_net_set_loss"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTS = ("mg_workspace_bytes", "mg_setup", "mg_vcycle", "mg_solve", "mg_solve_two_stage", "mg_level_get", "mg_level_info",
           "mg_destroy", "mg_strerror", "mg_timing_enable", "mg_timing_read", "mg_batch_workspace_bytes",
           "mg_setup_batched", "mg_solve_batched", "mg_vcycle_batched", "mg_autotune", "mg_net_weight_count",
           "mg_net_workspace_bytes", "mg_net_create", "mg_net_set_weights", "mg_net_get_weights", "mg_net_init",
           "mg_net_forward", "mg_net_loss_grad", "mg_net_train", "mg_net_destroy", "mg_set_coarse_net",
           "mg_net_stats", "mg_coarse_export", "mg_vcycle_static", "mg_cycle_workspace_bytes", "mg_setup_cycle",
           "mg_net_set_loss")

MG_NET_CUT = 6
MG_NET_LOSS_MSE, MG_NET_LOSS_CUT = 0, 1
NET_G = {2: 17, 3: 9}

# kernel families for mg_timing_enable
MG_K_RESIDUAL, MG_K_RESTRICT, MG_K_JACOBI, MG_K_FINEST, MG_K_COARSE, MG_K_NORM = range(6)


class MGError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s: %s (%d)" % (what, mg_strerror(code), code))
        self.code = code


def _check(code, what):
    if code != MG_OK:
        raise MGError(code, what)
    return code


# ---------------------------------------------------------------- raw C ABI

def mg_strerror(code):
    return _lib.mg_strerror(int(code)).decode()


def mg_workspace_bytes(dim, n, precision):
    out = _sz()
    _check(_lib.mg_workspace_bytes(dim, n, precision, ctypes.byref(out)), "mg_workspace_bytes")
    return out.value


def mg_level_info(dim, n, depth=0):
    nl, side = ctypes.c_int(), ctypes.c_int()
    _check(_lib.mg_level_info(dim, n, depth, ctypes.byref(nl), ctypes.byref(side)), "mg_level_info")
    return nl.value, side.value


def mg_setup(dim, n, precision, p, workspace_ptr, ws_bytes, stream_ptr):
    plan = _vp()
    arr = (ctypes.c_double * len(p))(*[float(x) for x in p])
    _check(_lib.mg_setup(ctypes.byref(plan), dim, n, precision, arr, len(p), _vp(workspace_ptr), ws_bytes,
                         _vp(stream_ptr)), "mg_setup")
    return plan


def mg_cycle_workspace_bytes(dim, n, precision, nu, gamma):
    out = _sz()
    _check(_lib.mg_cycle_workspace_bytes(dim, n, precision, nu, gamma, ctypes.byref(out)), "mg_cycle_workspace_bytes")
    return out.value


def mg_setup_cycle(dim, n, precision, p, nu, gamma, workspace_ptr, ws_bytes, stream_ptr):
    plan = _vp()
    arr = (ctypes.c_double * len(p))(*[float(x) for x in p])
    _check(_lib.mg_setup_cycle(ctypes.byref(plan), dim, n, precision, arr, len(p), nu, gamma, _vp(workspace_ptr),
                               ws_bytes, _vp(stream_ptr)), "mg_setup_cycle")
    return plan


def mg_vcycle(plan, u_ptr, f_ptr, want_relres=False):
    rr = ctypes.c_double()
    _check(_lib.mg_vcycle(plan, _vp(u_ptr), _vp(f_ptr), ctypes.byref(rr) if want_relres else None), "mg_vcycle")
    return rr.value if want_relres else None


def mg_solve(plan, u_ptr, f_ptr, rtol, max_cycles):
    """Returns (status, cycles, relres, history list)."""
    cyc, rr = ctypes.c_int(), ctypes.c_double()
    hist = (ctypes.c_double * (max_cycles + 1))()
    st = _lib.mg_solve(plan, _vp(u_ptr), _vp(f_ptr), float(rtol), int(max_cycles), ctypes.byref(cyc),
                       ctypes.byref(rr), hist)
    if st not in (MG_OK, MG_ERR_NOT_CONVERGED, MG_ERR_NONFINITE, MG_ERR_DIVERGED):
        raise MGError(st, "mg_solve")
    return st, cyc.value, rr.value, list(hist[:cyc.value + 1])


def mg_level_get(plan, depth, which, dst_ptr):
    _check(_lib.mg_level_get(plan, depth, which, _vp(dst_ptr)), "mg_level_get")


def mg_vcycle_static(dim, n, precision, p, u_ptr, f_ptr, stream_ptr, want_relres=False):
    """One V-cycle on the library's static scratch array (no allocation)."""
    arr = (ctypes.c_double * len(p))(*[float(x) for x in p])
    rr = ctypes.c_double()
    _check(_lib.mg_vcycle_static(dim, n, precision, arr, len(p), _vp(u_ptr), _vp(f_ptr),
                                 ctypes.byref(rr) if want_relres else None, _vp(stream_ptr)), "mg_vcycle_static")
    return rr.value if want_relres else None


def mg_destroy(plan):
    _check(_lib.mg_destroy(plan), "mg_destroy")


def _int_array(xs):
    return (ctypes.c_int * len(xs))(*[int(x) for x in xs])


def _ptr_array(ptrs):
    return (_vp * len(ptrs))(*[_vp(int(x)) for x in ptrs])


def mg_batch_workspace_bytes(ns, precision):
    out = _sz()
    _check(_lib.mg_batch_workspace_bytes(len(ns), _int_array(ns), precision, ctypes.byref(out)),
           "mg_batch_workspace_bytes")
    return out.value


def mg_setup_batched(ns, precision, p, workspace_ptr, ws_bytes, stream_ptr):
    plan = _vp()
    _check(_lib.mg_setup_batched(ctypes.byref(plan), len(ns), _int_array(ns), precision, float(p), _vp(workspace_ptr),
                                 ws_bytes, _vp(stream_ptr)), "mg_setup_batched")
    return plan


def mg_solve_batched(plan, u_ptrs, f_ptrs, rtol, max_cycles):
    """Returns (overall status, cycles list, relres list, status list)."""
    k = len(u_ptrs)
    cyc = (ctypes.c_int * k)()
    rr = (ctypes.c_double * k)()
    st = (ctypes.c_int * k)()
    ret = _lib.mg_solve_batched(plan, _ptr_array(u_ptrs), _ptr_array(f_ptrs), float(rtol), int(max_cycles), cyc, rr,
                                st)
    if ret not in (MG_OK, MG_ERR_NOT_CONVERGED, MG_ERR_NONFINITE, MG_ERR_DIVERGED):
        raise MGError(ret, "mg_solve_batched")
    return ret, list(cyc), list(rr), list(st)


def mg_vcycle_batched(plan, u_ptrs, f_ptrs, want_relres=False):
    k = len(u_ptrs)
    rr = (ctypes.c_double * k)()
    _check(_lib.mg_vcycle_batched(plan, _ptr_array(u_ptrs), _ptr_array(f_ptrs), rr if want_relres else None),
           "mg_vcycle_batched")
    return list(rr) if want_relres else None


def mg_autotune(plan):
    _check(_lib.mg_autotune(plan), "mg_autotune")


def mg_timing_enable(plan, family):
    _check(_lib.mg_timing_enable(plan, int(family)), "mg_timing_enable")


def mg_timing_read(plan):
    """Returns (summed ms, launches, summed algorithmic bytes) since the last read."""
    ms, cnt, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    _check(_lib.mg_timing_read(plan, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by)), "mg_timing_read")
    return ms.value, cnt.value, by.value


# ------------------------------------------- learned coarse correction (raw)

def mg_net_weight_count(dim):
    return _lib.mg_net_weight_count(dim)


def _f32(w, count):
    import numpy as np
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
    if w.size != count:
        raise ValueError("expected %d weights, got %d" % (count, w.size))
    return w, w.ctypes.data_as(_fp)


def mg_net_workspace_bytes(dim, max_batch):
    out = _sz()
    _check(_lib.mg_net_workspace_bytes(dim, max_batch, ctypes.byref(out)), "mg_net_workspace_bytes")
    return out.value


def mg_net_create(dim, max_batch, workspace_ptr, ws_bytes, stream_ptr):
    net = _vp()
    _check(_lib.mg_net_create(ctypes.byref(net), dim, max_batch, workspace_ptr, ws_bytes, stream_ptr), "mg_net_create")
    return net


def mg_net_set_weights(net, dim, w):
    arr, ptr = _f32(w, mg_net_weight_count(dim))
    _check(_lib.mg_net_set_weights(net, ptr), "mg_net_set_weights")


def mg_net_get_weights(net, dim):
    import numpy as np
    w = np.zeros(mg_net_weight_count(dim), dtype=np.float32)
    _check(_lib.mg_net_get_weights(net, w.ctypes.data_as(_fp)), "mg_net_get_weights")
    return w


def mg_net_init(net, seed):
    _check(_lib.mg_net_init(net, seed), "mg_net_init")


def mg_net_forward(net, in_ptr, out_ptr, batch, normalize):
    _check(_lib.mg_net_forward(net, in_ptr, out_ptr, batch, int(normalize)), "mg_net_forward")


def mg_net_loss_grad(net, dim, in_ptr, target_ptr, batch, normalize):
    import numpy as np
    g = np.zeros(mg_net_weight_count(dim), dtype=np.float32)
    loss = ctypes.c_double()
    _check(_lib.mg_net_loss_grad(net, in_ptr, target_ptr, batch, int(normalize), g.ctypes.data_as(_fp),
                                 ctypes.byref(loss)), "mg_net_loss_grad")
    return loss.value, g


def mg_net_train(net, r_ptr, e_ptr, npairs, epochs, batch, lr, seed):
    h = (ctypes.c_double * max(epochs, 1))()
    _check(_lib.mg_net_train(net, r_ptr, e_ptr, npairs, epochs, batch, lr, seed, h), "mg_net_train")
    return list(h)[:epochs]


def mg_net_set_loss(net, kind, pj=1.0):
    _check(_lib.mg_net_set_loss(net, int(kind), float(pj)), "mg_net_set_loss")


def mg_net_destroy(net):
    _check(_lib.mg_net_destroy(net), "mg_net_destroy")


def mg_set_coarse_net(plan, dim, w, cut_level=MG_NET_CUT):
    if w is None:
        _check(_lib.mg_set_coarse_net(plan, None, cut_level), "mg_set_coarse_net")
        return
    arr, ptr = _f32(w, mg_net_weight_count(dim))
    _check(_lib.mg_set_coarse_net(plan, ptr, cut_level), "mg_set_coarse_net")


def mg_net_stats(plan, nprob):
    """(net cycles, switched off, first-cycle cut ratio with the network, with the plain sub-cycle)"""
    used = (ctypes.c_int * nprob)()
    off = (ctypes.c_int * nprob)()
    qn = (ctypes.c_double * nprob)()
    qp = (ctypes.c_double * nprob)()
    _check(_lib.mg_net_stats(plan, used, off, qn, qp), "mg_net_stats")
    return list(used), list(off), list(qn), list(qp)


def mg_coarse_export(plan, level, dst_ptr):
    _check(_lib.mg_coarse_export(plan, level, dst_ptr), "mg_coarse_export")


# ------------------------------------------------------------ torch plumbing

P2D_TUNED = (1.052,)                    # Section 2.4
P2D_H4 = (1.20,)                        # Section 2.4: tuned for the fourth-order residual
P3D_TUNED = (1.11, 1.42, 1.08, 0.99)    # Section 3.4, Table tbl:3dopt
P3D_H4 = (0.91, 0.80, 0.70, 1.77)       # Section 3.4, Table tbl:3dopt: tuned for the fourth-order residual
# the conventional cycle's one parameter as the paper tunes it (Tables tbl:2d, tbl:3dopt, rows "usual")
P_USUAL = {(2, 2): (1.121,), (2, 4): (1.216,), (3, 2): (1.30,), (3, 4): (1.70,)}


class Solver:
    """A plan plus its workspace on one device / stream.

    u, f: float64 CUDA tensors of shape (n+1,)*dim, contiguous (x fastest).
    """

    def __init__(self, dim, n, precision=MG_FP64, p=None, device=None, stream=None, order=2, scheme="diagonal",
                 nu=None, gamma=None):
        if order not in (2, 4):
            raise ValueError("order must be 2 or 4")
        if scheme not in ("diagonal", "usual"):
            raise ValueError("scheme must be 'diagonal' or 'usual'")
        if p is None:
            if scheme == "usual":
                p = P_USUAL[(dim, order)]
            elif order == 4:
                p = P2D_H4 if dim == 2 else P3D_H4
            else:
                p = P2D_TUNED if dim == 2 else P3D_TUNED
        self.dim, self.n, self.precision, self.p = dim, n, precision, tuple(float(x) for x in p)
        self.order = order
        self.scheme = scheme
        # nu / gamma given: the generalised diagonal cycle (mg_setup_cycle)
        self.general = nu is not None or gamma is not None
        self.nu, self.gamma = int(nu or 1), int(gamma or 1)
        if self.general and scheme != "diagonal":
            raise ValueError("nu / gamma apply to the diagonal scheme")
        precision = precision | (MG_ORDER4 if order == 4 else 0) | (MG_USUAL if scheme == "usual" else 0)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws_bytes = (mg_cycle_workspace_bytes(dim, n, precision, self.nu, self.gamma) if self.general
                         else mg_workspace_bytes(dim, n, precision))
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            if self.general:
                self.plan = mg_setup_cycle(dim, n, precision, self.p, self.nu, self.gamma, self._ws_ptr, self.ws_bytes,
                                           self.stream.cuda_stream)
            else:
                self.plan = mg_setup(dim, n, precision, self.p, self._ws_ptr, self.ws_bytes, self.stream.cuda_stream)
        # the usual hierarchy has the grids of side n, n/2, ..., 2
        self.num_levels = n.bit_length() - 1 if scheme == "usual" else mg_level_info(dim, n)[0]

    def _chk(self, t, name):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and tuple(t.shape) == (self.n + 1,) * self.dim and t.device == self.device):
            raise ValueError("%s must be a contiguous float64 tensor of shape %s on %s"
                             % (name, (self.n + 1,) * self.dim, self.device))

    def vcycle(self, u, f, want_relres=False):
        self._chk(u, "u")
        self._chk(f, "f")
        return mg_vcycle(self.plan, u.data_ptr(), f.data_ptr(), want_relres)

    def solve(self, u, f, rtol=1e-10, max_cycles=50):
        self._chk(u, "u")
        self._chk(f, "f")
        return mg_solve(self.plan, u.data_ptr(), f.data_ptr(), rtol, max_cycles)

    def level(self, depth, which=0):
        side = self.n >> depth if self.scheme == "usual" else mg_level_info(self.dim, self.n, depth)[1]
        out = torch.empty((side + 1,) * self.dim, dtype=torch.float64, device=self.device)
        mg_level_get(self.plan, depth, which, out.data_ptr())
        return out

    def timing(self, family):
        mg_timing_enable(self.plan, family)

    def timing_read(self):
        return mg_timing_read(self.plan)

    def autotune(self):
        mg_autotune(self.plan)

    def set_coarse_net(self, w):
        """Learned coarse correction (2D): weights, or None for the plain cycle."""
        mg_set_coarse_net(self.plan, self.dim, w)

    def net_stats(self):
        """(network cycles, judge switched it off, first-cycle cut ratio with the
        network, with the plain sub-cycle) of the last solve."""
        used, off, qn, qp = mg_net_stats(self.plan, 1)
        return used[0], off[0], qn[0], qp[0]

    def coarse_export(self, level=MG_NET_CUT):
        """Restricted residual of aligned level `level` (0 = the coarsest) after the last cycle."""
        K = self.n.bit_length() - 1
        depth = self.dim * (K - 1) - level
        side = mg_level_info(self.dim, self.n, depth)[1]
        out = torch.empty((side + 1,) * self.dim, dtype=torch.float64, device=self.device)
        mg_coarse_export(self.plan, level, out.data_ptr())
        return out

    def close(self):
        if getattr(self, "plan", None) is not None:
            mg_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_two_stage(first, second, u, f, rtol1=1e-4, rtol=1e-10, max_cycles=50):
    """Fourth-order solution in two stages (Sections 2.3 and 3.3): `first`, a
    second-order Solver, cycles until its relative residual is <= rtol1; then
    `second`, an order-4 Solver of the same dim and n, cycles on the same u
    until the fourth-order relative residual is <= rtol.
    Returns (status, cycles of each stage, fourth-order relative residual)."""
    if first.order != 2 or second.order != 4 or (first.dim, first.n) != (second.dim, second.n):
        raise ValueError("two-stage solve needs an order-2 and an order-4 Solver of one size")
    first._chk(u, "u")
    first._chk(f, "f")
    c1, c2, rr = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    st = _lib.mg_solve_two_stage(first.plan, second.plan, _vp(u.data_ptr()), _vp(f.data_ptr()), float(rtol1),
                                 float(rtol), int(max_cycles), ctypes.byref(c1), ctypes.byref(c2), ctypes.byref(rr))
    if st not in (MG_OK, MG_ERR_NOT_CONVERGED, MG_ERR_NONFINITE, MG_ERR_DIVERGED):
        raise MGError(st, "mg_solve_two_stage")
    return st, c1.value, c2.value, rr.value


class BatchSolver:
    """Independent 2D problems solved together: one kernel launch per level
    for the whole batch.  ns: intervals per side of each problem."""

    def __init__(self, ns, precision=MG_FP32_REFINED, p=P2D_TUNED[0], device=None, stream=None):
        self.ns = [int(x) for x in ns]
        self.precision = precision
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws_bytes = mg_batch_workspace_bytes(self.ns, precision)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.ws.data_ptr() + 255) // 256 * 256
            self.plan = mg_setup_batched(self.ns, precision, p, ptr, self.ws_bytes, self.stream.cuda_stream)

    def _chk(self, ts, name):
        if len(ts) != len(self.ns):
            raise ValueError("%s: expected %d tensors" % (name, len(self.ns)))
        for t, n in zip(ts, self.ns):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == (n + 1, n + 1)
                    and t.device == self.device):
                raise ValueError("%s: each tensor must be contiguous float64 (n+1, n+1) on %s" % (name, self.device))

    def solve(self, us, fs, rtol=1e-10, max_cycles=50):
        self._chk(us, "u")
        self._chk(fs, "f")
        return mg_solve_batched(self.plan, [u.data_ptr() for u in us], [f.data_ptr() for f in fs], rtol, max_cycles)

    def vcycle(self, us, fs, want_relres=False):
        self._chk(us, "u")
        self._chk(fs, "f")
        return mg_vcycle_batched(self.plan, [u.data_ptr() for u in us], [f.data_ptr() for f in fs], want_relres)

    def autotune(self):
        mg_autotune(self.plan)

    def set_coarse_net(self, w):
        """Weights (host array, mg_net_weight_count(2) floats) of the learned
        coarse correction, or None for the plain cycle."""
        mg_set_coarse_net(self.plan, 2, w)

    def net_stats(self):
        """Per problem: cycles that used the network, 1 where the judge switched
        it off, and the first cycle's cut-level residual reduction with the
        network and with the plain sub-cycle."""
        return mg_net_stats(self.plan, len(self.ns))

    def coarse_export(self, level=MG_NET_CUT):
        """Restricted residual of aligned level `level` of every problem after the last cycle."""
        side = 1 << (1 + (level + 1) // 2)
        out = torch.empty((len(self.ns), side + 1, side + 1), dtype=torch.float64, device=self.device)
        mg_coarse_export(self.plan, level, out.data_ptr())
        return out

    def close(self):
        if getattr(self, "plan", None) is not None:
            mg_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """Trainer of the learned coarse correction: master weights, Adam state
    and gradient buffers for up to max_batch samples in a torch workspace."""

    def __init__(self, dim=2, max_batch=256, seed=None, device=None, stream=None):
        self.dim, self.max_batch = dim, max_batch
        self.G = NET_G[dim]
        self.nw = mg_net_weight_count(dim)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws_bytes = mg_net_workspace_bytes(dim, max_batch)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.ws.data_ptr() + 255) // 256 * 256
            self.net = mg_net_create(dim, max_batch, ptr, self.ws_bytes, self.stream.cuda_stream)
        if seed is not None:
            mg_net_init(self.net, seed)

    def _grid(self, t, name):
        shape = (self.G,) * self.dim
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape[1:]) == shape
                and t.device == self.device):
            raise ValueError("%s must be a contiguous float64 tensor of shape (B,) + %s on %s" % (name, shape, self.device))

    def set_weights(self, w):
        mg_net_set_weights(self.net, self.dim, w)

    def weights(self):
        return mg_net_get_weights(self.net, self.dim).reshape(4, 3 ** self.dim, 16, 16)

    def forward(self, x, normalize=True):
        self._grid(x, "x")
        out = torch.empty_like(x)
        mg_net_forward(self.net, x.data_ptr(), out.data_ptr(), x.shape[0], normalize)
        return out

    def set_loss(self, kind, pj=1.0):
        """MG_NET_LOSS_MSE, or MG_NET_LOSS_CUT with the cut level's
        over-relaxation parameter pj (then no target is read)."""
        mg_net_set_loss(self.net, kind, pj)
        self.loss_kind = kind

    def _target(self, t, name):
        if t is None and getattr(self, "loss_kind", MG_NET_LOSS_MSE) == MG_NET_LOSS_CUT:
            return None
        self._grid(t, name)
        return t.data_ptr()

    def loss_grad(self, x, target=None, normalize=False):
        self._grid(x, "x")
        tp = self._target(target, "target")
        loss, g = mg_net_loss_grad(self.net, self.dim, x.data_ptr(), tp, x.shape[0], normalize)
        return loss, g.reshape(4, 3 ** self.dim, 16, 16)

    def train(self, r, e, epochs, batch=256, lr=1e-3, seed=0):
        self._grid(r, "r")
        ep = self._target(e, "e")
        return mg_net_train(self.net, r.data_ptr(), ep, r.shape[0], epochs, batch, lr, seed)

    def close(self):
        if getattr(self, "net", None) is not None:
            mg_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

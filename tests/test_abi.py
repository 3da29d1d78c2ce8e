"""CPU checks of the C ABI: libdmg.so loads, exports every function
include/dmg.h declares, and the host-only parts (sizes, level plan, argument
errors raised before any GPU call) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "dmg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s*(mg_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def D():
    from paper_math_9907190_amd import dmg
    return dmg


def test_every_declared_symbol_is_exported(D):
    names = declared()
    assert len(names) >= 8
    for nm in names:
        assert hasattr(D._lib, nm), nm
    assert sorted(D.EXPORTS) == names


def test_level_info(D):
    assert D.mg_level_info(2, 64) == (11, 64)        # 2(K-1)+1 levels for n = 2^K
    assert D.mg_level_info(2, 4096) == (23, 4096)
    assert D.mg_level_info(3, 256) == (22, 256)      # 3(K-1)+1
    assert D.mg_level_info(2, 64, 10)[1] == 2        # coarsest: 3x3
    assert D.mg_level_info(3, 16, 9)[1] == 2         # coarsest: 3x3x3
    assert D.mg_level_info(2, 2) == (1, 2)


def test_workspace_bytes(D):
    b64 = D.mg_workspace_bytes(2, 4096, D.MG_FP64)
    b32 = D.mg_workspace_bytes(2, 4096, D.MG_FP32_REFINED)
    n2 = 4097 ** 2
    # finest residual plus r and v on every coarser level: about 3 arrays of the finest size
    assert 2.9 * 8 * n2 < b64 < 3.2 * 8 * n2
    # FP32-refined: the levels in single; the finest residual's array is the
    # out-of-place solve's second iterate, so it stays (n+1)^2 doubles
    assert 0.45 < (b32 - 4 * n2) / b64 < 0.55
    b3 = D.mg_workspace_bytes(3, 256, D.MG_FP64)
    assert 2.9 * 8 * 257 ** 3 < b3 < 3.4 * 8 * 257 ** 3


def test_order4_flag(D):
    """The fourth-order flag adds one (n+1)^dim double array (the right-hand
    side combination) to the workspace; batches of several problems reject it."""
    for n in (64, 4096):
        plain = D.mg_workspace_bytes(2, n, D.MG_FP64)
        o4 = D.mg_workspace_bytes(2, n, D.MG_FP64 | D.MG_ORDER4)
        assert 8 * (n + 1) ** 2 <= o4 - plain < 8 * (n + 1) ** 2 + 256
        assert D.mg_workspace_bytes(2, n, D.MG_FP32_REFINED | D.MG_ORDER4) > D.mg_workspace_bytes(2, n, D.MG_FP32_REFINED)
    out = ctypes.c_size_t()
    for n in (16, 256):
        plain = D.mg_workspace_bytes(3, n, D.MG_FP64)
        assert 8 * (n + 1) ** 3 <= D.mg_workspace_bytes(3, n, D.MG_FP64 | D.MG_ORDER4) - plain < 8 * (n + 1) ** 3 + 256
    assert D._lib.mg_workspace_bytes(3, 16, 2 | D.MG_ORDER4, ctypes.byref(out)) == D.MG_ERR_ARG
    assert D._lib.mg_workspace_bytes(2, 16, 2 | D.MG_ORDER4, ctypes.byref(out)) == D.MG_ERR_ARG
    ns = (ctypes.c_int * 2)(64, 128)
    assert D._lib.mg_batch_workspace_bytes(2, ns, D.MG_ORDER4, ctypes.byref(out)) == D.MG_ERR_ARG
    assert D._lib.mg_batch_workspace_bytes(1, ns, D.MG_ORDER4, ctypes.byref(out)) == D.MG_OK


@pytest.mark.parametrize("dim,n,code", [(2, 3, -2), (2, 1, -2), (2, 1 << 16, -2), (3, 1 << 12, -2), (4, 8, -1)])
def test_size_errors(D, dim, n, code):
    out = ctypes.c_size_t()
    assert D._lib.mg_workspace_bytes(dim, n, 0, ctypes.byref(out)) == code


def test_setup_argument_errors_before_any_gpu_call(D):
    plan = ctypes.c_void_p()
    p1 = (ctypes.c_double * 1)(1.052)
    p4 = (ctypes.c_double * 4)(1.11, 1.42, 1.08, 0.99)
    # wrong parameter count, bad parameter, bad precision, bad size, null / small workspace
    assert D._lib.mg_setup(ctypes.byref(plan), 2, 64, 0, p4, 4, None, 0, None) == D.MG_ERR_ARG
    bad = (ctypes.c_double * 1)(-1.0)
    assert D._lib.mg_setup(ctypes.byref(plan), 2, 64, 0, bad, 1, None, 0, None) == D.MG_ERR_ARG
    assert D._lib.mg_setup(ctypes.byref(plan), 2, 64, 7, p1, 1, None, 0, None) == D.MG_ERR_ARG
    assert D._lib.mg_setup(ctypes.byref(plan), 2, 48, 0, p1, 1, None, 0, None) == D.MG_ERR_SIZE
    assert D._lib.mg_setup(ctypes.byref(plan), 3, 16, 0, p4, 4, None, 0, None) == D.MG_ERR_WS
    assert D._lib.mg_setup(ctypes.byref(plan), 2, 64, 0, p1, 1, ctypes.c_void_p(4096), 16, None) == D.MG_ERR_WS
    assert D._lib.mg_setup(ctypes.byref(plan), 2, 64, 0, p1, 1, ctypes.c_void_p(4097), 1 << 30, None) == D.MG_ERR_WS
    assert D.mg_strerror(D.MG_ERR_WS).startswith("workspace")
    # two-stage solve: null or identical plans
    assert D._lib.mg_solve_two_stage(None, None, None, None, 1e-4, 1e-10, 10, None, None, None) == D.MG_ERR_ARG


def test_net_sizes_and_argument_errors(D):
    assert D.mg_net_weight_count(2) == 4 * 9 * 16 * 16
    assert D.mg_net_weight_count(3) == 4 * 27 * 16 * 16
    assert D.mg_net_weight_count(4) == 0
    b2 = D.mg_net_workspace_bytes(2, 256)
    # master weights, two Adam moments, two bf16 copies, per-sample gradients
    assert b2 >= 4 * 9216 * (3 + 256) + 2 * 2 * 9216
    assert D.mg_net_workspace_bytes(3, 1) < D.mg_net_workspace_bytes(3, 2)
    out = ctypes.c_size_t()
    assert D._lib.mg_net_workspace_bytes(4, 8, ctypes.byref(out)) == D.MG_ERR_ARG
    assert D._lib.mg_net_workspace_bytes(2, 0, ctypes.byref(out)) == D.MG_ERR_ARG
    net = ctypes.c_void_p()
    assert D._lib.mg_net_create(ctypes.byref(net), 2, 8, None, 0, None) == D.MG_ERR_WS
    assert D._lib.mg_net_create(ctypes.byref(net), 5, 8, None, 0, None) == D.MG_ERR_ARG
    assert D._lib.mg_net_destroy(None) == D.MG_OK
    assert D._lib.mg_net_set_loss(None, D.MG_NET_LOSS_CUT, 1.0) == D.MG_ERR_ARG
    # a plan is required; checked before any GPU call
    assert D._lib.mg_set_coarse_net(None, None, 6) == D.MG_ERR_ARG
    assert D._lib.mg_net_stats(None, None, None, None, None) == D.MG_ERR_ARG
    assert D._lib.mg_coarse_export(None, 6, None) == D.MG_ERR_ARG


def test_batch_workspace_holds_the_net_weights(D):
    # the packed bf16 forward weights (9216 entries) are part of every 2D plan
    b = D.mg_batch_workspace_bytes([4], D.MG_FP64)
    assert b >= 2 * 9216


def test_vcycle_static_errors_before_any_gpu_call(D):
    """The allocation-free cycle rejects bad arguments and problems larger
    than its 64 MiB scratch array before it touches the GPU."""
    p1 = (ctypes.c_double * 1)(1.052)
    p4 = (ctypes.c_double * 4)(1.11, 1.42, 1.08, 0.99)
    u = ctypes.c_void_p(4096)
    f = ctypes.c_void_p(8192)
    call = D._lib.mg_vcycle_static
    assert call(2, 64, 0, p1, 1, None, f, None, None) == D.MG_ERR_ARG
    assert call(2, 64, 0, p1, 1, u, None, None, None) == D.MG_ERR_ARG
    assert call(2, 64, 0, p4, 4, u, f, None, None) == D.MG_ERR_ARG
    assert call(3, 16, 0, p1, 1, u, f, None, None) == D.MG_ERR_ARG
    assert call(2, 48, 0, p1, 1, u, f, None, None) == D.MG_ERR_SIZE
    assert call(2, 64, 5, p1, 1, u, f, None, None) == D.MG_ERR_ARG
    assert call(4, 8, 0, p1, 1, u, f, None, None) == D.MG_ERR_ARG
    # sizes: the largest that fit, and the first that do not
    cap = D.MG_STATIC_SCRATCH_BYTES
    assert D.mg_workspace_bytes(2, 1024, D.MG_FP64 | D.MG_ORDER4) <= cap
    # (2D single-precision levels: mg_workspace_bytes also counts the second
    # iterate of out-of-place solves, 4 more bytes per point than this cycle's)
    assert D.mg_workspace_bytes(2, 2048, D.MG_FP32_REFINED) - 4 * 2049 ** 2 <= cap
    assert D.mg_workspace_bytes(3, 128, D.MG_FP64) <= cap
    for dim, n, prec, p, np_ in ((2, 2048, D.MG_FP64, p1, 1), (2, 4096, D.MG_FP32_REFINED, p1, 1),
                                 (3, 256, D.MG_FP32_REFINED, p4, 4), (3, 128, D.MG_FP64 | D.MG_ORDER4, p4, 4)):
        assert D.mg_workspace_bytes(dim, n, prec) > cap
        assert call(dim, n, prec, p, np_, u, f, None, None) == D.MG_ERR_SCRATCH
    assert "scratch" in D.mg_strerror(D.MG_ERR_SCRATCH)

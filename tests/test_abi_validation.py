"""Argument validation of the C ABI, exercised without a GPU: every entry
point checks its arguments before the first HIP call, so invalid calls
return their status code and message here."""
import ctypes as C
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1302_1861_amd", "libpsl.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB),
                                reason="libpsl.so not built")

DUMMY = C.c_void_p(0x1000)   # never dereferenced: validation fails first


def _P():
    import paper_1302_1861_amd as P
    return P


def _err(P):
    return P.lib().psl_last_error().decode()


def _grid(P, e=(0.0, 1.0, 2.0), x=(-1.0, 0.0, 1.0), y=(-1.0, 1.0)):
    return P.make_grid(np.array(e), np.array(x), np.array(y), 25.0)


def _phsp(P, n):
    p = P.psl_phsp()
    p.n = n
    for k in P.PHSP_KEYS:
        setattr(p, k, 0x1000)
    return p


def test_build_rejects_non_increasing_edges():
    P = _P()
    g = _grid(P, e=(0.0, 2.0, 1.0))
    st = P.lib().psl_build(C.byref(_phsp(P, 10)), C.byref(g),
                           C.byref(_phsp(P, 10)), DUMMY, DUMMY, None, 0, None)
    assert st == P.PSL_EINVAL and "increasing" in _err(P).lower()


def test_build_rejects_null_and_small_output():
    P = _P()
    g = _grid(P)
    L = P.lib()
    assert L.psl_build(None, C.byref(g), C.byref(_phsp(P, 10)), DUMMY, DUMMY,
                       None, 0, None) == P.PSL_EINVAL
    st = L.psl_build(C.byref(_phsp(P, 10)), C.byref(g), C.byref(_phsp(P, 5)),
                     DUMMY, DUMMY, None, 0, None)
    assert st == P.PSL_EINVAL and "capacity" in _err(P)


def test_build_reports_short_workspace():
    P = _P()
    g = _grid(P)
    L = P.lib()
    need = L.psl_build_workspace_bytes(1000, C.byref(g))
    assert need > 0
    st = L.psl_build(C.byref(_phsp(P, 1000)), C.byref(g),
                     C.byref(_phsp(P, 1000)), DUMMY, DUMMY, DUMMY, need - 1,
                     None)
    assert st == P.PSL_ENOSPC and "workspace" in _err(P)


def test_workspace_queries_grow_with_the_problem():
    P = _P()
    L = P.lib()
    g = _grid(P)
    a = L.psl_sample_workspace_bytes(C.byref(g), 1, 1000)
    b = L.psl_sample_workspace_bytes(C.byref(g), 1, 1_000_000)
    c = L.psl_sample_workspace_bytes(C.byref(g), 7, 1_000_000)
    assert 0 < a < b < c
    assert L.psl_build_workspace_bytes(10, C.byref(g)) < \
        L.psl_build_workspace_bytes(10_000_000, C.byref(g))


def test_tally_rejects_bad_op_and_too_few_batches():
    P = _P()
    L = P.lib()
    ph = P.psl_phantom()
    ph.nx = ph.ny = ph.nz = 4
    ph.dx = ph.dy = ph.dz = 1.0
    ph.density = 0x1000
    st = L.dose_tally(None, DUMMY, DUMMY, 7, 2, C.byref(ph), 1.0, DUMMY,
                      DUMMY, None)
    assert st == P.PSL_EINVAL and "op" in _err(P)
    st = L.dose_tally(None, DUMMY, DUMMY, P.PSL_TALLY_FINALIZE, 1,
                      C.byref(ph), 1.0, DUMMY, DUMMY, None)
    assert st == P.PSL_EINVAL and "2 batches" in _err(P)
    ph.nx = 0
    assert L.dose_tally(None, DUMMY, DUMMY, P.PSL_TALLY_FOLD, 0, C.byref(ph),
                        1.0, None, None, None) == P.PSL_EINVAL


def test_gamma_rejects_bad_criteria():
    P = _P()
    L = P.lib()
    args = [DUMMY, DUMMY, 4, 4, 4, 0.25, 0.25, 0.25]
    assert L.dose_gamma(*args, 0.0, 0.2, 0.04, 0.0, None, DUMMY, None) \
        == P.PSL_EINVAL
    st = L.dose_gamma(*args, 1.0, 0.2, 0.001, 0.0, None, DUMMY, None)
    assert st == P.PSL_EINVAL and "offsets" in _err(P)
    assert L.dose_gamma(*args, 1.0, 0.2, 0.04, 0.0, None, None, None) \
        == P.PSL_EINVAL


def test_transport_rejects_bad_queue_and_density_bounds():
    P = _P()
    L = P.lib()
    q = P.psl_queue()
    q.n_ebuckets = 0
    ph = P.psl_phantom()
    phys = P.make_physics()
    acc = P.psl_dose_acc()
    st = L.transport_batch(C.byref(q), C.byref(ph), C.byref(phys), DUMMY, 1,
                           C.byref(acc), DUMMY, None, None, 0, None)
    assert st == P.PSL_EINVAL


def test_unet_sizes_and_shape_checks():
    from oracle import unet as U
    P = _P()
    L = P.lib()
    n = L.unet_param_count(4, 16)
    # the documented flat layout, counted by the float64 reference
    shapes = U.layer_shapes()
    blob = U.pack({**{k: (np.zeros((co, 27, ci)), np.zeros(co))
                      for k, (ci, co) in shapes.items()},
                   "head": (np.zeros(16), 0.0)})
    assert n == blob.size
    assert L.unet_param_count(3, 16) == 0 and L.unet_param_count(4, 8) == 0
    net = P.psl_unet()
    net.levels, net.base, net.n_params = 4, 16, n
    net.params = net.params_bf16 = 0x1000
    assert L.unet_workspace_bytes(C.byref(net), 1, 16, 16, 16, 0) < \
        L.unet_workspace_bytes(C.byref(net), 1, 16, 16, 16, 1)
    st = L.unet_forward(C.byref(net), DUMMY, DUMMY, 1, 12, 16, 16, DUMMY,
                        DUMMY, 1 << 30, None)
    assert st == P.PSL_EINVAL and "divisible by 8" in _err(P)
    net.n_params = n - 1
    assert L.unet_forward(C.byref(net), DUMMY, DUMMY, 1, 16, 16, 16, DUMMY,
                          DUMMY, 1 << 30, None) == P.PSL_EINVAL


def test_brick_blocks_cap_rejects_negative_and_restores_default():
    P = _P()
    assert P.lib().unet_set_brick_blocks(-1) == P.PSL_EINVAL
    assert "max_blocks" in _err(P)
    assert P.lib().unet_set_brick_blocks(5) == 0
    assert P.lib().unet_set_brick_blocks(0) == 0


def test_plan_set_rejects_null_and_bad_counts():
    P = _P()
    L = P.lib()
    assert L.psl_plan_run_set(None, 1, 0, 1, None) == P.PSL_EINVAL
    assert "plan array" in _err(P)
    arr = (C.c_void_p * 2)(None, None)
    for n in (0, 9, -1):
        assert L.psl_plan_run_set(arr, n, 0, 1, None) == P.PSL_EINVAL
        assert "n_plans" in _err(P)
    assert L.psl_plan_run_set(arr, 1, 0, 1, None) == P.PSL_EINVAL
    assert "NULL plan 0" in _err(P)
    assert L.psl_plan_run_set(arr, 2, -1, 1, None) == P.PSL_EINVAL
    assert "batch range" in _err(P)
    assert L.psl_plan_run_set(arr, 2, 0, -3, None) == P.PSL_EINVAL

"""The C-ABI library loads and exports every entry point include/oic.h declares
(CPU only: no call here touches a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_09663_amd import oic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "oic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oic_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["oic_create", "oic_set_weights", "oic_solve", "oic_destroy", "oic_solve_ex",
                 "oic_last_error"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(oic.LIB_PATH), reason="liboic.so not built")
def test_library_exports_every_declared_symbol():
    L = oic.lib()  # loads the library once per process, after torch's HIP runtime
    for name in declared():
        assert hasattr(L, name), name
    assert sorted(oic.EXPORTED) == declared()


@pytest.mark.skipif(not os.path.exists(oic.LIB_PATH), reason="liboic.so not built")
def test_host_side_validation_needs_no_device():
    L = oic.lib()
    assert L.oic_kernel_class_count() >= 10
    L.oic_destroy(None)  # NULL-safe
    assert L.oic_last_error(None) == b"NULL handle"
    cfg = oic.oic_config()
    h = ctypes.c_void_p()
    # invalid configurations are rejected before any device call
    cfg.n, cfg.m, cfg.l, cfg.n_layers = 2, 16, 1, 1
    cfg.channels[0], cfg.channels[1] = 2, 1
    cfg.max_N, cfg.max_H = 4, 2
    assert L.oic_create(ctypes.byref(cfg), ctypes.byref(h)) == oic.OIC_EINVAL
    cfg.n = 16
    cfg.channels[1] = 3  # last layer must have one channel
    assert L.oic_create(ctypes.byref(cfg), ctypes.byref(h)) == oic.OIC_EINVAL
    cfg.channels[1] = 1
    cfg.activation = 7
    assert L.oic_create(ctypes.byref(cfg), ctypes.byref(h)) == oic.OIC_EINVAL
    assert L.oic_solve(None, None, None, None, None, 2, 1, 0, None, None) == oic.OIC_EINVAL


@pytest.mark.skipif(not os.path.exists(oic.LIB_PATH), reason="liboic.so not built")
def test_group_and_server_argument_checks_need_no_device():
    """Groups: slot counts outside 1..OIC_MAX_GROUP_SLOTS and several slots of a configuration
    without grouped kernels (FP32) are rejected before any device call; the footprint of a
    group is its slab times the slots; NULL handles are safe.  Server: the pack size is
    checked and fixed once requests have started."""
    L = oic.lib()
    cfg = oic.oic_config()
    cfg.n, cfg.m, cfg.l, cfg.n_layers = 32, 32, 8, 3
    for k, c in enumerate((2, 16, 16, 1)):
        cfg.channels[k] = c
    cfg.activation, cfg.max_N, cfg.max_H = oic.OIC_ACT_TANH, 32, 3
    g = ctypes.c_void_p()
    cfg.precision = oic.OIC_PREC_BF16
    assert L.oic_group_create(ctypes.byref(cfg), 0, ctypes.byref(g)) == oic.OIC_EINVAL
    assert L.oic_group_create(ctypes.byref(cfg), 65, ctypes.byref(g)) == oic.OIC_EINVAL
    cfg.precision = oic.OIC_PREC_FP32
    assert L.oic_group_create(ctypes.byref(cfg), 2, ctypes.byref(g)) == oic.OIC_EINVAL
    cfg.precision = oic.OIC_PREC_BF16
    one = L.oic_group_footprint_bytes(ctypes.byref(cfg), 1)
    four = L.oic_group_footprint_bytes(ctypes.byref(cfg), 4)
    assert one > 0 and four - 4096 == 4 * (one - 4096) and (one - 4096) % (2 << 20) == 0
    assert L.oic_footprint_bytes(ctypes.byref(cfg)) == one
    L.oic_group_destroy(None)
    assert L.oic_group_slot(None, 0) is None
    assert L.oic_group_solve(None, 1, None, None, None) == oic.OIC_EINVAL
    assert L.oic_group_last_error(None) == b"NULL group"
    # the binding raises on the same checks
    with pytest.raises(oic.OicError):
        oic.Group(32, 32, 8, (2, 16, 16, 1), oic.OIC_ACT_TANH, 32, 3, 0)
    with pytest.raises(oic.OicError):
        oic.Group(32, 32, 8, (2, 16, 16, 1), oic.OIC_ACT_TANH, 32, 3, 2, precision=oic.OIC_PREC_FP32)
    with pytest.raises(oic.OicError):
        oic.Server(1 << 30, max_inflight=1, group_slots=0)
    with oic.Server(1 << 30, max_inflight=1) as srv:
        assert L.oic_server_set_group_slots(srv._s, 0) == oic.OIC_EINVAL
        assert L.oic_server_set_group_slots(srv._s, 65) == oic.OIC_EINVAL
        assert L.oic_server_set_group_slots(srv._s, 4) == oic.OIC_OK
        st = srv.stats()
        assert st["batches"] == 0 and st["packs"] == 0


@pytest.mark.skipif(not os.path.exists(oic.LIB_PATH), reason="liboic.so not built")
def test_stage_cost_matches_oracle_trace_form():
    """Host-side cost of the library vs the oracle's trace form (no device call)."""
    import numpy as np
    from oracle import cost
    from paper_2410_09663_amd import workloads as wl
    rng = np.random.default_rng(4)
    n, m, l = 6, 5, 3
    X, Xr = rng.standard_normal((2, n, m)).astype(np.float32)
    U, dU = rng.standard_normal((2, l, m)).astype(np.float32)
    Q = wl.random_spd(l, 1)
    R = wl.random_spd(n, 2)
    got = oic.stage_cost(X, Xr, U, dU, Q, R)
    ref = cost.stage_cost_trace(X, Xr, U, np.zeros_like(U), dU, R.astype(np.float64),
                                Q.astype(np.float64), Q.astype(np.float64))
    assert abs(got - ref) <= 1e-10 * abs(ref)
    with pytest.raises(oic.OicError):
        oic.stage_cost(X, Xr, U, dU, -Q, R)


def test_column_transform_matches_oracle():
    """oic_columns_expand / oic_columns_project (host functions) against the oracle's
    U = u T and u = U T^T (T T^T)^{-1}, including the repeat-the-column T = [1 ... 1]."""
    from oracle import transform as tr
    rng = np.random.default_rng(4)
    for (l, q, m) in ((3, 1, 8), (4, 2, 16), (2, 5, 5)):
        T = (np.ones((1, m)) if q == 1 else rng.standard_normal((q, m))).astype(np.float32)
        u = rng.standard_normal((l, q)).astype(np.float32)
        U = oic.columns_expand(u, T)
        assert np.allclose(U, tr.expand(u, T), rtol=1e-6, atol=1e-6)
        U2 = rng.standard_normal((l, m)).astype(np.float32)
        got = oic.columns_project(U2, T)
        want = tr.project(U2, T)
        assert np.linalg.norm(got - want) <= 1e-6 * np.linalg.norm(want)
    # rank-deficient T: T T^T singular
    with pytest.raises(oic.OicError):
        oic.columns_project(np.ones((2, 4), np.float32), np.ones((2, 4), np.float32))

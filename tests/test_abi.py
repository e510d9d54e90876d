"""CPU checks of the C ABI: the library loads, exports every function that
include/laps.h declares, and rejects invalid arguments before it touches a
device (no compute calls are made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2601_16696_amd import build, laps
    if not os.path.exists(laps.LIB_PATH):
        build.build(verbose=False)
    return laps


def _declared():
    src = open(os.path.join(ROOT, "include", "laps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(laps_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "laps_init" in names and "laps_step_adjusted" in names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_row_stride_and_defaults(L):
    assert [L.row_stride(d) for d in (1, 2, 8, 9, 100, 2429)] == [8, 8, 8, 16, 104, 2432]
    c = L.Config()
    L.lib().laps_config_default(ctypes.byref(c), 1024, 100)
    assert (c.C, c.alpha, c.eps0_factor, c.switch_tol, c.window_frac, c.acc_tol) == (0.025, 2.0, 0.01, 0.01, 0.2, 0.03)
    assert (c.L_partial_factor, c.n_steps_traj, c.eevpd_mode) == (1.25, 15, 1)


def _cfg_target(L, kind=0, N=16, d=10, side=0):
    c = L.Config()
    L.lib().laps_config_default(ctypes.byref(c), N, d)
    t = L.TargetS()
    t.kind = kind
    t.d = d
    t.data[0] = 0x1000
    t.data[1] = 0x2000
    t.dims[0] = side if side else 7
    return c, t


def _ws(L, c, t):
    n = ctypes.c_size_t(0)
    st = L.lib().laps_workspace_size(ctypes.byref(c), ctypes.byref(t), ctypes.byref(n))
    return st, n.value


def test_validation_codes(L):
    c, t = _cfg_target(L)
    st, n = _ws(L, c, t)
    assert st == L.OK and n > 0 and n % 256 == 0
    c.d = 1
    t.d = 1
    assert _ws(L, c, t)[0] == L.EINVAL           # d - 1 divides the velocity update
    c, t = _cfg_target(L, N=1)
    assert _ws(L, c, t)[0] == L.EINVAL
    c, t = _cfg_target(L)
    t.d = 11
    assert _ws(L, c, t)[0] == L.EINVAL
    c, t = _cfg_target(L, kind=3, d=10, side=3)   # 3 x 3 != 10
    assert _ws(L, c, t)[0] == L.EINVAL
    c, t = _cfg_target(L, kind=3, d=9, side=3)
    assert _ws(L, c, t)[0] == L.OK
    c, t = _cfg_target(L, kind=9)
    assert _ws(L, c, t)[0] == L.EINVAL
    c, t = _cfg_target(L)
    t.data[0] = None
    assert _ws(L, c, t)[0] == L.EINVAL
    c, t = _cfg_target(L, d=40000)
    assert _ws(L, c, t)[0] == L.EUNSUPPORTED
    c, t = _cfg_target(L)
    c.eevpd_mode = 3
    assert _ws(L, c, t)[0] == L.EINVAL


def test_init_rejects_before_touching_the_device(L):
    lib = L.lib()
    c, t = _cfg_target(L)
    st, n = _ws(L, c, t)
    ctx = ctypes.c_void_p()
    P = ctypes.c_void_p
    # null positions
    assert lib.laps_init(ctypes.byref(c), ctypes.byref(t), None, None, P(0x10000), n, None, ctypes.byref(ctx)) == L.EINVAL
    # misaligned positions / workspace
    assert lib.laps_init(ctypes.byref(c), ctypes.byref(t), P(0x10004), None, P(0x10000), n, None,
                         ctypes.byref(ctx)) == L.EINVAL
    assert lib.laps_init(ctypes.byref(c), ctypes.byref(t), P(0x10000), None, P(0x10040), n, None,
                         ctypes.byref(ctx)) == L.EINVAL
    # short workspace
    assert lib.laps_init(ctypes.byref(c), ctypes.byref(t), P(0x10000), None, P(0x10000), n - 256, None,
                         ctypes.byref(ctx)) == L.EWORKSPACE
    assert lib.laps_step_unadjusted(None, 1) == L.EINVAL
    assert lib.laps_step_adjusted(None, 1) == L.EINVAL
    assert lib.laps_status_string(L.EPHASE).decode() == "wrong phase"


def test_batch_and_restart_entry_points_validate(L):
    lib = L.lib()
    P = ctypes.c_void_p
    ms = ctypes.c_float(0.0)
    g = ctypes.c_void_p()
    assert lib.laps_restart(None, None) == L.EINVAL
    assert lib.laps_time_kernel(None, 1, 5, ctypes.byref(ms)) == L.EINVAL
    assert lib.laps_graph_create(None, 1, 1, None, 10, 0, ctypes.byref(g)) == L.EINVAL
    ctxs = (P * 1)(None)
    assert lib.laps_graph_create(ctxs, 1, 1, None, 10, 0, ctypes.byref(g)) == L.EINVAL
    assert lib.laps_graph_create(ctxs, 0, 1, None, 10, 0, ctypes.byref(g)) == L.EINVAL
    assert lib.laps_graph_launch(None, None) == L.EINVAL
    assert lib.laps_graph_destroy(None) == L.OK


@pytest.mark.parametrize("kind,d,side,lanes,ok", [
    (0, 100, 0, 0, True), (0, 100, 0, 4, True), (0, 100, 0, 3, False), (0, 100, 0, 96, False),
    (0, 100, 0, 128, True), (0, 100, 0, 1024, False), (2, 2429, 0, 64, True), (2, 2429, 0, 16, False),
    (3, 4096, 64, 0, True), (3, 144, 12, 4, False), (3, 144, 12, 32, True)])
def test_team_shape_override(L, kind, d, side, lanes, ok):
    """team_lanes picks the lanes per chain; shapes needing more octs per lane
    than the kernels hold (6 in FP32), or lanes that are neither a power of
    two up to 64 nor a multiple of 64 up to 512, are refused.  A phi^4 side
    that is not a multiple of 8 takes one oct per lane."""
    c, t = _cfg_target(L, kind=kind, d=d, side=side)
    c.prec = L.F32
    c.team_lanes = lanes
    st, _ = _ws(L, c, t)
    assert (st == L.OK) == ok, st
    c.team_lanes = -1
    assert _ws(L, c, t)[0] == L.EINVAL


@pytest.mark.parametrize("kind", [1, 4, 5])
def test_update_kernel_targets_limited_to_narrow_teams(L, kind):
    """Logistic regression, callbacks and the dense Gaussian share the
    per-chain update kernels, whose teams have at most 16 lanes (several octs
    per lane above d = 128, up to d = 512).  Logistic regression stops at
    d = 128 (its gradient kernels hold a chain's theta in registers); both
    integrators are accepted."""
    def cfg(d, integ=0):
        c, t = _cfg_target(L, kind=kind, d=d)
        t.cb = 0x3000
        c.integrator_adj = integ
        return c, t
    assert _ws(L, *cfg(100))[0] == L.OK
    assert _ws(L, *cfg(128))[0] == L.OK
    for d in (129, 138, 200, 204, 300, 512):
        for integ in (0, 1, 2):
            want = L.EUNSUPPORTED if kind == L.LOGREG else L.OK
            assert _ws(L, *cfg(d, integ))[0] == want, (d, integ)
    for integ in (0, 1, 2):
        assert _ws(L, *cfg(513, integ))[0] == L.EUNSUPPORTED
    for d in (37, 100, 128):
        assert _ws(L, *cfg(d, 2))[0] == L.OK, d


def test_callback_target_validation(L):
    """A caller-supplied target needs a callback and runs in FP64 or FP32 state."""
    c, t = _cfg_target(L, kind=L.CALLBACK, d=30)
    assert _ws(L, c, t)[0] == L.EINVAL            # no callback
    t.cb = 0x3000
    assert _ws(L, c, t)[0] == L.OK
    c.prec = L.F32
    assert _ws(L, c, t)[0] == L.OK
    c.prec = L.MIXED_BF16
    assert _ws(L, c, t)[0] == L.EUNSUPPORTED


def test_full_rank_probes_validation(L):
    c, t = _cfg_target(L, kind=0, N=600, d=300)
    st0, n0 = _ws(L, c, t)
    assert st0 == L.OK
    c.full_rank_probes = 100
    st1, n1 = _ws(L, c, t)
    # probe dot products [N][P], per-chunk projections [2 chunks][P][d], block sums
    assert st1 == L.OK and n1 >= n0 + 8 * (600 * 100 + 2 * 100 * 300)
    for bad in (-1, 1025):
        c.full_rank_probes = bad
        assert _ws(L, c, t)[0] == L.EINVAL


def test_dense_gauss_validation(L):
    c, t = _cfg_target(L, kind=L.GAUSS_DENSE, d=100)
    assert _ws(L, c, t)[0] == L.OK
    t.data[0] = 0
    assert _ws(L, c, t)[0] == L.EINVAL
    c, t = _cfg_target(L, kind=L.GAUSS_DENSE, d=120)
    st, n = _ws(L, c, t)
    assert st == L.OK and n >= 120 * 120 * 8      # the precision matrix is copied into the workspace
    c.prec = L.MIXED_BF16
    assert _ws(L, c, t)[0] == L.EUNSUPPORTED


def test_launch_shape_fields_validation(L):
    c, t = _cfg_target(L, kind=0, N=64, d=40)
    for b in (0, 64, 128, 256):
        c.block_threads = b
        assert _ws(L, c, t)[0] == L.OK
    c.block_threads = 96
    assert _ws(L, c, t)[0] == L.EINVAL
    c.block_threads = 0
    c.grad_workgroups = -1
    assert _ws(L, c, t)[0] == L.EINVAL


def test_eps_fixed_validation(L):
    c, t = _cfg_target(L, kind=0, N=64, d=40)
    c.eps_fixed = 0.5
    assert _ws(L, c, t)[0] == L.OK
    for bad in (-0.1, float("nan"), float("inf")):
        c.eps_fixed = bad
        assert _ws(L, c, t)[0] == L.EINVAL


def test_dynamics_validation(L):
    c, t = _cfg_target(L, kind=0, N=64, d=40)
    for v in (0, 1):
        c.dynamics = v
        assert _ws(L, c, t)[0] == L.OK
    c.dynamics = 2
    assert _ws(L, c, t)[0] == L.EINVAL


def test_eval_entry_point_rejects_null(L):
    assert L.lib().laps_eval(None, None, None, None) == L.EINVAL


def test_dimension_limits(L):
    # FP64: 2 octs per lane on 512-lane teams; FP32: 6 octs, within the MAMS kernel's 160 KiB of LDS
    for prec, ok_d, bad_d in ((0, 8192, 8200), (1, 20000, 21000)):
        c, t = _cfg_target(L, kind=0, N=4, d=ok_d)
        c.prec = prec
        assert _ws(L, c, t)[0] == L.OK
        c, t = _cfg_target(L, kind=0, N=4, d=bad_d)
        c.prec = prec
        assert _ws(L, c, t)[0] != L.OK


def test_static_init_refuses_oversized_workspace_before_touching_the_device(L):
    """laps_init_static validates like laps_init and refuses configurations
    whose workspace exceeds its static array (32 MiB) with LAPS_EWORKSPACE,
    before any device call."""
    c, t = _cfg_target(L, kind=2, N=4096, d=2429)
    c.prec = L.F32
    st, n = _ws(L, c, t)
    assert st == L.OK and n > 32 << 20
    x = ctypes.c_void_p(0x100000)
    ctx = ctypes.c_void_p()
    assert L.lib().laps_init_static(ctypes.byref(c), ctypes.byref(t), x, None, None, ctypes.byref(ctx)) == L.EWORKSPACE
    assert b"static workspace" in L.lib().laps_last_error(None)
    c, t = _cfg_target(L, kind=0, N=1, d=10)
    assert L.lib().laps_init_static(ctypes.byref(c), ctypes.byref(t), x, None, None, ctypes.byref(ctx)) == L.EINVAL
    c, t = _cfg_target(L, kind=0, N=16, d=10)
    assert L.lib().laps_init_static(ctypes.byref(c), ctypes.byref(t), ctypes.c_void_p(0x100004), None, None,
                                    ctypes.byref(ctx)) == L.EINVAL

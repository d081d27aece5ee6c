"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/prism_proj.h, rejects bad arguments before touching the
device, and its host-side FP64 factor equals the oracle's (independent code)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import factor as ofactor, problem
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("prism_proj.h", "prism_server.h")]


def _lib():
    from paper_2608_25666_amd import _lib as L
    return L, L.load()


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(prism_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert lib.prism_abi_version() == 4


def test_status_strings_and_defaults():
    L, lib = _lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lib.prism_status_str(s)
    o = L.Options()
    lib.prism_options_default(C.byref(o))
    assert o.precision == 0 and o.alpha == 1.0 and o.tol == 0.0 and o.check_every == 10


@pytest.mark.parametrize("H,rho,w", [(2, 1.0, None), (5, 1.0, None), (20, 1.0, None), (50, 1.0, None),
                                     (100, 1.0, None), (128, 0.5, None), (33, 3.0, None),
                                     (50, 1.0, (1.0, 0.05, 4.0, 20.0)), (17, 2.0, (0.5, 1.0, 2.0, 3.0))])
def test_host_factor_matches_oracle(H, rho, w):
    from oracle import admm
    from paper_2608_25666_amd import factor_host
    K, k = factor_host(H, rho, w)
    lim = problem.joint_limits(W.UR5E_BIMANUAL_BOUNDS(1), 0)
    C_ = problem.velocity_unit_rows(H, 0.02, lim, 0.0, 0.0).C
    R = admm.block_penalty(H, rho, w)
    Ko, ko = ofactor.reduced_inverse(np.eye(H) + C_.T @ (R[:, None] * C_))
    np.testing.assert_allclose(K, Ko, atol=1e-10 * max(1.0, np.abs(Ko).max()))
    np.testing.assert_allclose(k, ko, atol=1e-10)
    assert np.all(K[0] == 0.0) and np.all(K[:, 0] == 0.0)


def test_factor_is_independent_of_dt():
    """After the velocity-unit scaling C = [I; L; D1; D2] is unit-free: K depends on H, rho only."""
    lim = problem.joint_limits(W.UR5E_BIMANUAL_BOUNDS(1), 0)
    a = problem.velocity_unit_rows(30, 0.02, lim, 0.0, 0.0).C
    b = problem.velocity_unit_rows(30, 0.05, lim, 0.0, 0.0).C
    np.testing.assert_allclose(a, b, atol=1e-12)


def _bounds(nj, lo=-1.0, hi=1.0):
    arrs = [(C.c_double * nj)(*([lo if i % 2 == 0 else hi] * nj)) for i in range(8)]
    L, _ = _lib()
    return L.Bounds(*[C.cast(a, C.POINTER(C.c_double)) for a in arrs]), arrs


@pytest.mark.parametrize("H,nj,dt,rho", [(1, 2, 0.1, 1.0), (129, 2, 0.1, 1.0), (10, 0, 0.1, 1.0),
                                         (10, 65, 0.1, 1.0), (10, 2, 0.0, 1.0),
                                         (10, 2, float("nan"), 1.0), (10, 2, 0.1, 0.0),
                                         (10, 2, 0.1, -1.0), (10, 2, 0.1, float("inf"))])
def test_create_rejects_bad_arguments(H, nj, dt, rho):
    L, lib = _lib()
    b, keep = _bounds(max(nj, 1))
    h = C.c_void_p()
    assert lib.prism_proj_create(H, nj, dt, C.byref(b), rho, C.byref(h)) == L.PRISM_EINVAL
    assert not h.value


def test_create_rejects_inverted_or_nonfinite_bounds():
    L, lib = _lib()
    h = C.c_void_p()
    b, keep = _bounds(3, lo=1.0, hi=-1.0)
    assert lib.prism_proj_create(10, 3, 0.1, C.byref(b), 1.0, C.byref(h)) == L.PRISM_EINVAL
    b, keep = _bounds(3, lo=-float("inf"), hi=1.0)
    assert lib.prism_proj_create(10, 3, 0.1, C.byref(b), 1.0, C.byref(h)) == L.PRISM_EINVAL
    assert lib.prism_proj_create(10, 3, 0.1, None, 1.0, C.byref(h)) == L.PRISM_EINVAL


def _jerk_bounds(jerk):
    """Bounds with the given per-joint jerk half-widths (the other limits loose)."""
    nj = len(jerk)
    L, _ = _lib()
    arrs = [(C.c_double * nj)(*v) for v in
            ([-7.0] * nj, [7.0] * nj, [-3.0] * nj, [3.0] * nj, [-8.0] * nj, [8.0] * nj,
             [-j for j in jerk], list(jerk))]
    return L.Bounds(*[C.cast(a, C.POINTER(C.c_double)) for a in arrs]), arrs


def test_default_block_weights_and_weight_validation():
    L, lib = _lib()
    w = (C.c_double * 4)()
    # the tuned point: jerk bound 60 rad/s^3 at dt = 0.02, i.e. 0.024 rad/s per step^2
    b, keep = _jerk_bounds([60.0] * 12)
    assert lib.prism_default_block_weights(50, 12, 0.02, C.byref(b), w) == L.PRISM_OK
    assert tuple(w) == (1.7, 2.125 / 50, 13.6, 17.0)
    # dt = 0.05: the jerk bound in velocity units is 6.25x wider, the weights 6.25x smaller
    assert lib.prism_default_block_weights(20, 12, 0.05, C.byref(b), w) == L.PRISM_OK
    np.testing.assert_allclose(tuple(w), np.array((1.7, 2.125 / 20, 13.6, 17.0)) / 6.25,
                               rtol=1e-14)
    # the smallest jerk half-width over the joints decides; asymmetric bounds by half-width
    b, keep = _jerk_bounds([120.0, 30.0, 60.0])
    assert lib.prism_default_block_weights(50, 3, 0.02, C.byref(b), w) == L.PRISM_OK
    np.testing.assert_allclose(w[0], 1.7 * 2.0, rtol=1e-14)
    # clipped to [2^-4.5, 2^1.5]
    b, keep = _jerk_bounds([6000.0])
    assert lib.prism_default_block_weights(50, 1, 0.02, C.byref(b), w) == L.PRISM_OK
    np.testing.assert_allclose(w[0], 1.7 * 2.0 ** -4.5, rtol=1e-14)
    b, keep = _jerk_bounds([1.0])
    assert lib.prism_default_block_weights(50, 1, 0.02, C.byref(b), w) == L.PRISM_OK
    np.testing.assert_allclose(w[0], 1.7 * 2.0 ** 1.5, rtol=1e-14)
    # bad arguments write nothing
    w[0] = -1.0
    for args in ((1, 1, 0.02), (129, 1, 0.02), (50, 0, 0.02), (50, 65, 0.02), (50, 1, 0.0),
                 (50, 1, float("nan"))):
        assert lib.prism_default_block_weights(*args, C.byref(b), w) == L.PRISM_EINVAL
    assert lib.prism_default_block_weights(50, 1, 0.02, None, w) == L.PRISM_EINVAL
    b0, keep0 = _jerk_bounds([0.0])
    assert lib.prism_default_block_weights(50, 1, 0.02, C.byref(b0), w) == L.PRISM_EINVAL
    assert w[0] == -1.0
    b, keep = _bounds(2)
    h = C.c_void_p()
    bad = (C.c_double * 4)(1.0, 0.0, 1.0, 1.0)
    assert lib.prism_proj_create_ex(10, 2, 0.1, C.byref(b), 1.0, bad, C.byref(h)) == L.PRISM_EINVAL
    bad = (C.c_double * 4)(1.0, float("nan"), 1.0, 1.0)
    assert lib.prism_proj_create_ex(10, 2, 0.1, C.byref(b), 1.0, bad, C.byref(h)) == L.PRISM_EINVAL


def test_null_handle_calls_are_rejected():
    L, lib = _lib()
    o = L.Options()
    lib.prism_options_default(C.byref(o))
    assert lib.prism_proj_set_options(None, C.byref(o)) == L.PRISM_EINVAL
    assert lib.prism_proj_solve(None, None, 0, None, None, 0, None, None, None, None) == L.PRISM_EINVAL
    a = L.SolveArgs()
    assert lib.prism_proj_solve_ex(None, C.byref(a), None) == L.PRISM_EINVAL
    la = L.LiteralArgs()
    assert lib.prism_proj_literal(None, C.byref(la), None) == L.PRISM_EINVAL
    assert lib.prism_proj_horizon(None) == -1
    lib.prism_proj_destroy(None)
    assert lib.prism_factor_host(1, 1.0, None, None, None) == L.PRISM_EINVAL


def test_batch_null_arguments_rejected():
    L, lib = _lib()
    assert lib.prism_batch_create(None) == L.PRISM_EINVAL
    assert lib.prism_proj_solve_batch(None, 0, None, None, None) == L.PRISM_EINVAL
    lib.prism_batch_destroy(None)


def test_server_null_and_bad_arguments_rejected():
    L, lib = _lib()
    cfg = L.ServerConfig()
    lib.prism_server_config_default(C.byref(cfg))
    assert cfg.max_inflight == 2 and cfg.max_batch == 64 and cfg.hbm_budget == 1 << 30
    assert cfg.grid_share == 75
    h = C.c_void_p()
    assert lib.prism_server_create(None, C.byref(h)) == L.PRISM_EINVAL
    for field, bad in (("max_inflight", 0), ("max_inflight", 5), ("max_batch", 0),
                       ("max_queue", 0), ("grid_share", 0), ("grid_share", 101),
                       ("hbm_budget", 0)):
        c2 = L.ServerConfig()
        lib.prism_server_config_default(C.byref(c2))
        setattr(c2, field, bad)
        assert lib.prism_server_create(C.byref(c2), C.byref(h)) == L.PRISM_EINVAL, field
    cid = C.c_int32()
    assert lib.prism_server_add_controller(None, None, 1, C.byref(cid)) == L.PRISM_EINVAL
    t = C.c_int64()
    assert lib.prism_server_submit(None, 0, None, C.byref(t)) == L.PRISM_EINVAL
    info = L.TicketInfo()
    assert lib.prism_server_poll(None, 1, C.byref(info)) == L.PRISM_EINVAL
    assert lib.prism_server_wait(None, 1, 0, C.byref(info)) == L.PRISM_EINVAL
    assert lib.prism_server_release(None, 1) == L.PRISM_EINVAL
    st = L.ServerStats()
    assert lib.prism_server_stats(None, C.byref(st)) == L.PRISM_EINVAL
    lib.prism_server_destroy(None)
    a, b = lib.prism_server_now_ns(), lib.prism_server_now_ns()
    assert 0 < a <= b


def test_plan_workspace_and_null_arguments():
    L, lib = _lib()
    assert lib.prism_plan_workspace_bytes(1, 2, 10) == 0
    assert lib.prism_plan_workspace_bytes(20, 0, 10) == 0
    assert lib.prism_plan_workspace_bytes(20, 2, 0) == 0
    n = lib.prism_plan_workspace_bytes(50, 12, 2048)
    # per-column costs, costs and weights, best index, moment partials (8 blocks)
    assert n >= 2048 * 12 * 4 + 2 * 2048 * 8 + 4 + 8 * 600 * 16 and n % 256 == 0
    a = L.PlanArgs()
    assert lib.prism_plan_step(None, C.byref(a), None) == L.PRISM_EINVAL

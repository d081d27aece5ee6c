"""ctypes declarations of the C ABI in include/prism_proj.h.

Loading fails loudly when libprism_proj.so has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libprism_proj.so")

PRISM_OK = 0
PRISM_EINVAL = -1
PRISM_ENOMEM = -2
PRISM_EDEVICE = -3
PRISM_EINFEASIBLE = -4
PRISM_EBUSY = -5
PRISM_EUNSUPPORTED = -6
PRISM_ETOOLARGE = -7
PLAN_STATIC_WORKSPACE_BYTES = 8 << 20

PREC_FP32, PREC_BF16, PREC_FP16 = 0, 1, 2
MAX_H = 128
MAX_JOINTS = 64


class PrismError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.prism_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")


class Bounds(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in
                ("q_min", "q_max", "v_min", "v_max", "a_min", "a_max", "j_min", "j_max")]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("fp32_tail", C.c_int32), ("alpha", C.c_float),
                ("tol", C.c_float), ("check_every", C.c_int32), ("tile_waves", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class SolveArgs(C.Structure):
    _fields_ = [("v_samples", C.c_void_p), ("N", C.c_int32), ("iters", C.c_int32),
                ("q0", C.POINTER(C.c_double)), ("v0", C.POINTER(C.c_double)),
                ("v_out", C.c_void_p), ("r_primal", C.c_void_p), ("r_dual", C.c_void_p),
                ("iters_out", C.c_void_p), ("x_warm", C.c_void_p), ("state_warm", C.c_void_p),
                ("state_out", C.c_void_p), ("opts", C.POINTER(Options)),
                ("warm_shift", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("proj", C.c_void_p), ("v_samples", C.c_void_p), ("N", C.c_int32),
                ("iters", C.c_int32), ("q0", C.POINTER(C.c_double)), ("v0", C.POINTER(C.c_double)),
                ("v_out", C.c_void_p), ("r_primal", C.c_void_p), ("r_dual", C.c_void_p),
                ("iters_out", C.c_void_p), ("x_warm", C.c_void_p), ("state_warm", C.c_void_p),
                ("state_out", C.c_void_p), ("warm_shift", C.c_int32)]


class PlanArgs(C.Structure):
    _fields_ = [("nu", C.c_void_p), ("sigma", C.c_void_p), ("seed", C.c_uint64),
                ("stream", C.c_uint64), ("N", C.c_int32), ("iters", C.c_int32),
                ("q0", C.POINTER(C.c_double)), ("v0", C.POINTER(C.c_double)),
                ("theta_ref", C.c_void_p), ("w_pos", C.c_float), ("w_vel", C.c_float),
                ("tau", C.c_float), ("eps", C.c_float), ("x_out", C.c_void_p),
                ("samples_out", C.c_void_p), ("cost", C.c_void_p), ("omega", C.c_void_p),
                ("nu_out", C.c_void_p), ("var_out", C.c_void_p), ("best", C.c_void_p),
                ("r_primal", C.c_void_p), ("r_dual", C.c_void_p), ("iters_out", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("opts", C.POINTER(Options))]


class LiteralArgs(C.Structure):
    _fields_ = [("v_samples", C.c_void_p), ("x_init", C.c_void_p), ("v_out", C.c_void_p),
                ("violation", C.c_void_p), ("N", C.c_int32), ("iters", C.c_int32),
                ("delta", C.c_double), ("q0", C.POINTER(C.c_double)),
                ("v0", C.POINTER(C.c_double))]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_inflight", C.c_int32), ("max_batch", C.c_int32),
                ("max_queue", C.c_int32), ("grid_share", C.c_int32), ("opts", Options)]


class ServeRequest(C.Structure):
    _fields_ = [("v_samples", C.c_void_p), ("N", C.c_int32), ("iters", C.c_int32),
                ("q0", C.POINTER(C.c_double)), ("v0", C.POINTER(C.c_double)),
                ("v_out", C.c_void_p), ("r_primal", C.c_void_p), ("r_dual", C.c_void_p),
                ("iters_out", C.c_void_p)]


class TicketInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("error", C.c_int32), ("warm", C.c_int32),
                ("batch_size", C.c_int32), ("t_submit_ns", C.c_int64), ("t_launch_ns", C.c_int64),
                ("t_done_ns", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in
                ("submitted", "completed", "failed", "launches", "evictions", "queued", "running",
                 "max_concurrent_launches", "pool_bytes", "pool_used")]


SERVER_QUEUED, SERVER_RUNNING, SERVER_DONE, SERVER_FAILED = 0, 1, 2, 3

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7) with
    # its own HSA runtime. Whichever loads first is the process's runtime, so let
    # torch's load first: the library then shares it with the tensors it reads.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2608_25666_amd.build or __graft_entry__.build())")
    lib = C.CDLL(path)
    H = C.c_void_p      # opaque handle
    st = C.c_int
    sig = {
        "prism_options_default": (None, [C.POINTER(Options)]),
        "prism_proj_create": (st, [C.c_int, C.c_int, C.c_double, C.POINTER(Bounds), C.c_double,
                                   C.POINTER(H)]),
        "prism_proj_create_ex": (st, [C.c_int, C.c_int, C.c_double, C.POINTER(Bounds),
                                      C.c_double, C.POINTER(C.c_double), C.POINTER(H)]),
        "prism_default_block_weights": (C.c_int, [C.c_int, C.c_int, C.c_double, C.POINTER(Bounds),
                                                 C.POINTER(C.c_double)]),
        "prism_proj_get_weights": (st, [H, C.POINTER(C.c_double)]),
        "prism_proj_set_options": (st, [H, C.POINTER(Options)]),
        "prism_proj_get_options": (st, [H, C.POINTER(Options)]),
        "prism_proj_solve": (st, [H, C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]),
        "prism_proj_solve_ex": (st, [H, C.POINTER(SolveArgs), C.c_void_p]),
        "prism_proj_feasibility": (st, [H, C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
        "prism_proj_destroy": (None, [H]),
        "prism_proj_horizon": (C.c_int, [H]),
        "prism_proj_joints": (C.c_int, [H]),
        "prism_proj_get_factor": (st, [H, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "prism_factor_host": (st, [C.c_int, C.c_double, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "prism_batch_create": (st, [C.POINTER(H)]),
        "prism_batch_destroy": (None, [H]),
        "prism_proj_solve_batch": (st, [H, C.c_int, C.POINTER(Request), C.POINTER(Options),
                                        C.c_void_p]),
        "prism_plan_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int]),
        "prism_plan_step": (st, [H, C.POINTER(PlanArgs), C.c_void_p]),
        "prism_plan_step_static": (st, [H, C.POINTER(PlanArgs), C.c_void_p]),
        "prism_proj_literal": (st, [H, C.POINTER(LiteralArgs), C.c_void_p]),
        "prism_server_config_default": (None, [C.POINTER(ServerConfig)]),
        "prism_server_create": (st, [C.POINTER(ServerConfig), C.POINTER(H)]),
        "prism_server_destroy": (None, [H]),
        "prism_server_add_controller": (st, [H, H, C.c_int32, C.POINTER(C.c_int32)]),
        "prism_server_submit": (st, [H, C.c_int32, C.POINTER(ServeRequest),
                                     C.POINTER(C.c_int64)]),
        "prism_server_poll": (st, [H, C.c_int64, C.POINTER(TicketInfo)]),
        "prism_server_wait": (st, [H, C.c_int64, C.c_int64, C.POINTER(TicketInfo)]),
        "prism_server_release": (st, [H, C.c_int64]),
        "prism_server_stats": (st, [H, C.POINTER(ServerStats)]),
        "prism_server_now_ns": (C.c_int64, []),
        "prism_status_str": (C.c_char_p, [C.c_int]),
        "prism_abi_version": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def lib():
    return load()


def check(status: int, where: str):
    if status != PRISM_OK:
        raise PrismError(status, where)


def dbl_array(values):
    arr = (C.c_double * len(values))(*[float(v) for v in values])
    return arr

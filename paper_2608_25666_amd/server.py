"""Python front end of the projection server (include/prism_server.h): argument
marshalling only. The worker thread, admission and launches are native."""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as L


class Server:
    """Continuous-batching server over one GPU's warm-state pool.

    budget: bytes of device memory for the controllers' warm state.
    Tensors passed to submit() are kept referenced until release().
    """

    def __init__(self, budget: int = 1 << 30, opts: Optional[L.Options] = None,
                 max_inflight: int = 2, max_batch: int = 64, max_queue: int = 65536,
                 grid_share: int = 75):
        cfg = L.ServerConfig()
        L.lib().prism_server_config_default(C.byref(cfg))
        cfg.hbm_budget = int(budget)
        cfg.max_inflight = int(max_inflight)
        cfg.max_batch = int(max_batch)
        cfg.max_queue = int(max_queue)
        cfg.grid_share = int(grid_share)
        if opts is not None:
            cfg.opts = opts
        h = C.c_void_p()
        L.check(L.lib().prism_server_create(C.byref(cfg), C.byref(h)), "prism_server_create")
        self._h = h
        self._keep = {}
        self._ctrl = {}

    def close(self):
        if getattr(self, "_h", None):
            L.lib().prism_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_controller(self, proj, max_N: int) -> int:
        cid = C.c_int32()
        L.check(L.lib().prism_server_add_controller(self._h, proj.handle, int(max_N),
                                                    C.byref(cid)), "prism_server_add_controller")
        self._ctrl[cid.value] = proj
        return cid.value

    def submit(self, ctrl: int, samples, q0, v0, iters: int, out, r_primal=None, r_dual=None,
               iters_out=None) -> int:
        P = self._ctrl.get(ctrl)          # unknown ids are rejected by the library
        nj = P.nj if P is not None else int(np.asarray(q0).size)
        if P is not None:
            import torch
            from .projector import _check
            if samples is None or samples.ndim != 3:
                raise ValueError("samples: expected a [N][H][n_joints] tensor")
            N, dev, f32 = int(samples.shape[0]), samples.device, torch.float32
            _check(samples, "samples", (N, P.H, P.nj), f32, dev, optional=False)
            _check(out, "out", (N, P.H, P.nj), f32, dev, optional=False)
            _check(r_primal, "r_primal", (N, P.nj), f32, dev)
            _check(r_dual, "r_dual", (N, P.nj), f32, dev)
            _check(iters_out, "iters_out", (N, P.nj), torch.int32, dev)
        q0a = L.dbl_array(np.broadcast_to(np.asarray(q0, dtype=np.float64), (nj,)))
        v0a = L.dbl_array(np.broadcast_to(np.asarray(v0, dtype=np.float64), (nj,)))
        r = L.ServeRequest()
        r.v_samples = samples.data_ptr()
        r.N = int(samples.shape[0])
        r.iters = int(iters)
        r.q0 = C.cast(q0a, C.POINTER(C.c_double))
        r.v0 = C.cast(v0a, C.POINTER(C.c_double))
        r.v_out = out.data_ptr()
        r.r_primal = None if r_primal is None else r_primal.data_ptr()
        r.r_dual = None if r_dual is None else r_dual.data_ptr()
        r.iters_out = None if iters_out is None else iters_out.data_ptr()
        t = C.c_int64()
        L.check(L.lib().prism_server_submit(self._h, int(ctrl), C.byref(r), C.byref(t)),
                "prism_server_submit")
        self._keep[t.value] = (samples, out, r_primal, r_dual, iters_out)
        return t.value

    @staticmethod
    def _info(i: L.TicketInfo) -> dict:
        return {"state": i.state, "error": i.error, "warm": bool(i.warm),
                "batch_size": i.batch_size, "t_submit_ns": i.t_submit_ns,
                "t_launch_ns": i.t_launch_ns, "t_done_ns": i.t_done_ns}

    def poll(self, ticket: int) -> dict:
        i = L.TicketInfo()
        L.check(L.lib().prism_server_poll(self._h, int(ticket), C.byref(i)), "prism_server_poll")
        return self._info(i)

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        i = L.TicketInfo()
        L.check(L.lib().prism_server_wait(self._h, int(ticket), int(timeout_ms), C.byref(i)),
                "prism_server_wait")
        return self._info(i)

    def release(self, ticket: int):
        L.check(L.lib().prism_server_release(self._h, int(ticket)), "prism_server_release")
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        s = L.ServerStats()
        L.check(L.lib().prism_server_stats(self._h, C.byref(s)), "prism_server_stats")
        return {n: getattr(s, n) for n, _ in L.ServerStats._fields_}


def now_ns() -> int:
    """CLOCK_MONOTONIC nanoseconds, the clock of the ticket timestamps."""
    return int(L.lib().prism_server_now_ns())

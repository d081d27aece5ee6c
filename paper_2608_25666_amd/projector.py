"""Thin Python front end of the C ABI: argument marshalling only.

PyTorch provides device memory and the current HIP stream; every step of the
projection runs in the library's kernels. Tensors must live on the GPU that
was current when the Projector was created.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as L


def options(precision: int = L.PREC_FP32, fp32_tail: int = 0, alpha: float = 1.0,
            tol: float = 0.0, check_every: int = 10, tile_waves: int = 0) -> L.Options:
    o = L.Options()
    L.lib().prism_options_default(C.byref(o))
    o.precision = precision
    o.fp32_tail = fp32_tail
    o.alpha = alpha
    o.tol = tol
    o.check_every = check_every
    o.tile_waves = tile_waves
    return o


def _bounds_struct(bounds, nj):
    arrs = [L.dbl_array(np.broadcast_to(np.asarray(b, dtype=np.float64), (nj,)))
            for b in (bounds.q_min, bounds.q_max, bounds.v_min, bounds.v_max,
                      bounds.a_min, bounds.a_max, bounds.j_min, bounds.j_max)]
    s = L.Bounds(*[C.cast(a, C.POINTER(C.c_double)) for a in arrs])
    return s, arrs


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _on_device(t, device) -> bool:
    return bool(t.is_cuda) and (device is None or t.device == device)


def _check(t, name, shape, dtype, device, optional=True):
    """Checks a tensor before its pointer goes to the library, which cannot: dtype,
    contiguity, the exact shape, and the device (the GPU of the other tensors).
    Raises ValueError naming the argument."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not _on_device(t, device):
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    return t


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def default_block_weights(H: int, n_joints: int, dt: float, bounds):
    """prism_default_block_weights: recommended (velocity, position, acceleration, jerk)
    weights for horizon H, step dt and the joints' bounds."""
    w = (C.c_double * 4)()
    b, keep = _bounds_struct(bounds, int(n_joints))
    L.check(L.lib().prism_default_block_weights(int(H), int(n_joints), float(dt), C.byref(b), w),
            "prism_default_block_weights")
    return tuple(w)


class Projector:
    """Handle for one (H, joints, dt, bounds, rho, block weights) problem family.

    weights: None for the scalar penalty (prism_proj_create), "default" for
    prism_default_block_weights(H, n_joints, dt, bounds), or four positive numbers.
    """

    def __init__(self, H: int, n_joints: int, dt: float, bounds, rho: float = 1.0,
                 weights=None):
        self.H, self.nj, self.dt, self.rho = int(H), int(n_joints), float(dt), float(rho)
        self.bounds = bounds
        if isinstance(weights, str) and weights == "default":
            weights = default_block_weights(self.H, self.nj, self.dt, bounds)
        self.weights = None if weights is None else tuple(float(v) for v in weights)
        b, keep = _bounds_struct(bounds, self.nj)
        h = C.c_void_p()
        wa = None if self.weights is None else (C.c_double * 4)(*self.weights)
        L.check(L.lib().prism_proj_create_ex(self.H, self.nj, self.dt, C.byref(b), self.rho,
                                             wa, C.byref(h)), "prism_proj_create_ex")
        self._h = h
        del keep

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            L.lib().prism_proj_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, opts: L.Options):
        L.check(L.lib().prism_proj_set_options(self._h, C.byref(opts)), "prism_proj_set_options")

    def factor(self):
        K = np.zeros((self.H, self.H))
        k = np.zeros(self.H)
        L.check(L.lib().prism_proj_get_factor(
            self._h, K.ctypes.data_as(C.POINTER(C.c_double)),
            k.ctypes.data_as(C.POINTER(C.c_double))), "prism_proj_get_factor")
        return K, k

    def solve(self, samples, q0, v0, iters: int, opts: Optional[L.Options] = None,
              out=None, r_primal=None, r_dual=None, iters_out=None, x_warm=None,
              state_warm=None, state_out=None, warm_shift=False, stream=None):
        """Project samples ([N][H][nj] float32 on the GPU). Asynchronous on the stream.

        Returns (v_out, r_primal, r_dual); pass preallocated tensors to avoid
        allocation. iters_out / state_out ([N][nj][4][H] dual state q) are filled
        when given; x_warm / state_warm warm-start the iteration, advanced by one
        MPC step first when warm_shift is set.
        """
        import torch
        if samples is None or samples.ndim != 3:
            raise ValueError("samples: expected a [N][H][n_joints] tensor")
        N = int(samples.shape[0])
        dev = samples.device
        f32, i32 = torch.float32, torch.int32
        traj, col, state = (N, self.H, self.nj), (N, self.nj), (N, self.nj, 4, self.H)
        _check(samples, "samples", traj, f32, dev, optional=False)
        if out is None:
            out = torch.empty_like(samples)
        if r_primal is None:
            r_primal = torch.empty(col, dtype=f32, device=dev)
        if r_dual is None:
            r_dual = torch.empty(col, dtype=f32, device=dev)
        _check(out, "out", traj, f32, dev)
        _check(r_primal, "r_primal", col, f32, dev)
        _check(r_dual, "r_dual", col, f32, dev)
        _check(iters_out, "iters_out", col, i32, dev)
        _check(x_warm, "x_warm", traj, f32, dev)
        _check(state_warm, "state_warm", state, f32, dev)
        _check(state_out, "state_out", state, f32, dev)
        q0a = L.dbl_array(np.broadcast_to(np.asarray(q0, dtype=np.float64), (self.nj,)))
        v0a = L.dbl_array(np.broadcast_to(np.asarray(v0, dtype=np.float64), (self.nj,)))
        a = L.SolveArgs()
        a.v_samples = samples.data_ptr()
        a.N = N
        a.iters = int(iters)
        a.q0 = C.cast(q0a, C.POINTER(C.c_double))
        a.v0 = C.cast(v0a, C.POINTER(C.c_double))
        a.v_out = out.data_ptr()
        a.r_primal = r_primal.data_ptr()
        a.r_dual = r_dual.data_ptr()
        a.iters_out = None if iters_out is None else iters_out.data_ptr()
        a.x_warm = None if x_warm is None else x_warm.data_ptr()
        a.state_warm = None if state_warm is None else state_warm.data_ptr()
        a.state_out = None if state_out is None else state_out.data_ptr()
        a.opts = C.pointer(opts) if opts is not None else C.POINTER(L.Options)()
        a.warm_shift = 1 if warm_shift else 0
        L.check(L.lib().prism_proj_solve_ex(self._h, C.byref(a), _stream(stream)),
                "prism_proj_solve_ex")
        return out, r_primal, r_dual

    def literal(self, samples, q0, v0, iters: int, delta: float = 1.0, x_init=None, out=None,
                violation=None, stream=None):
        """The Bregman iteration as Sec. III-D prints it (prism_proj_literal), FP64:
        `iters` passes from x_init (or the samples), lambda_0 = 0. Not the
        projection: it stops at a feasible point near the sample. Asynchronous on
        the stream. Returns (v_out [N][H][nj] float32, violation [N][nj] float64)."""
        import torch
        if samples is None or samples.ndim != 3:
            raise ValueError("samples: expected a [N][H][n_joints] tensor")
        N = int(samples.shape[0])
        dev = samples.device
        traj = (N, self.H, self.nj)
        _check(samples, "samples", traj, torch.float32, dev, optional=False)
        _check(x_init, "x_init", traj, torch.float32, dev)
        if out is None:
            out = torch.empty_like(samples)
        if violation is None:
            violation = torch.empty((N, self.nj), dtype=torch.float64, device=dev)
        _check(out, "out", traj, torch.float32, dev)
        _check(violation, "violation", (N, self.nj), torch.float64, dev)
        q0a = L.dbl_array(np.broadcast_to(np.asarray(q0, dtype=np.float64), (self.nj,)))
        v0a = L.dbl_array(np.broadcast_to(np.asarray(v0, dtype=np.float64), (self.nj,)))
        a = L.LiteralArgs()
        a.v_samples = samples.data_ptr()
        a.x_init = None if x_init is None else x_init.data_ptr()
        a.v_out = out.data_ptr()
        a.violation = violation.data_ptr()
        a.N = N
        a.iters = int(iters)
        a.delta = float(delta)
        a.q0 = C.cast(q0a, C.POINTER(C.c_double))
        a.v0 = C.cast(v0a, C.POINTER(C.c_double))
        L.check(L.lib().prism_proj_literal(self._h, C.byref(a), _stream(stream)),
                "prism_proj_literal")
        return out, violation

    def plan_step(self, nu, sigma, N: int, seed: int, stream_id: int, q0, v0, theta_ref,
                  w_pos: float, w_vel: float, tau: float, eps: float, iters: int,
                  opts: Optional[L.Options] = None, samples_out=None, r_primal=None,
                  r_dual=None, iters_out=None, workspace=None, stream=None, static=False,
                  outputs=None):
        """One optimizer iteration (prism_plan_step): draw N samples from
        N(nu, diag(sigma^2)) on the device, project, score, weight, update moments.
        nu, sigma, theta_ref: [H][nj] float32 on the GPU. Returns a dict of tensors
        x, cost, omega, nu, var, best (and samples when samples_out is given).

        static=True calls prism_plan_step_static (no workspace: the library's static
        device scratch). outputs: an earlier call's result dict whose x, cost, omega,
        nu, var, best tensors are written again instead of new ones (no allocation)."""
        import torch
        dev = nu.device
        N = int(N)
        f32 = torch.float32
        hj, traj, col = (self.H, self.nj), (N, self.H, self.nj), (N, self.nj)
        _check(nu, "nu", hj, f32, dev, optional=False)
        _check(sigma, "sigma", hj, f32, dev, optional=False)
        _check(theta_ref, "theta_ref", hj, f32, dev, optional=False)
        if outputs is None:
            outputs = {"x": torch.empty(traj, dtype=f32, device=dev),
                       "cost": torch.empty(N, dtype=torch.float64, device=dev),
                       "omega": torch.empty(N, dtype=torch.float64, device=dev),
                       "nu": torch.empty(hj, dtype=f32, device=dev),
                       "var": torch.empty(hj, dtype=f32, device=dev),
                       "best": torch.empty(1, dtype=torch.int32, device=dev)}
        x = _check(outputs["x"], "x", traj, f32, dev, optional=False)
        cost = _check(outputs["cost"], "cost", (N,), torch.float64, dev, optional=False)
        omega = _check(outputs["omega"], "omega", (N,), torch.float64, dev, optional=False)
        nu_out = _check(outputs["nu"], "nu_out", hj, f32, dev, optional=False)
        var_out = _check(outputs["var"], "var_out", hj, f32, dev, optional=False)
        best = _check(outputs["best"], "best", (1,), torch.int32, dev, optional=False)
        _check(samples_out, "samples_out", traj, f32, dev)
        _check(r_primal, "r_primal", col, f32, dev)
        _check(r_dual, "r_dual", col, f32, dev)
        _check(iters_out, "iters_out", col, torch.int32, dev)
        if static:
            workspace = None
        else:
            nbytes = int(L.lib().prism_plan_workspace_bytes(self.H, self.nj, N))
            if workspace is None or workspace.numel() < nbytes:
                workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
            if (workspace.dtype != torch.uint8 or not workspace.is_contiguous()
                    or workspace.device != dev):
                raise ValueError("workspace: expected a contiguous uint8 tensor on the device")
        q0a = L.dbl_array(np.broadcast_to(np.asarray(q0, dtype=np.float64), (self.nj,)))
        v0a = L.dbl_array(np.broadcast_to(np.asarray(v0, dtype=np.float64), (self.nj,)))
        a = L.PlanArgs()
        a.nu, a.sigma, a.theta_ref = nu.data_ptr(), sigma.data_ptr(), theta_ref.data_ptr()
        a.seed, a.stream, a.N, a.iters = int(seed), int(stream_id), int(N), int(iters)
        a.q0 = C.cast(q0a, C.POINTER(C.c_double))
        a.v0 = C.cast(v0a, C.POINTER(C.c_double))
        a.w_pos, a.w_vel, a.tau, a.eps = float(w_pos), float(w_vel), float(tau), float(eps)
        a.x_out, a.cost, a.omega = x.data_ptr(), cost.data_ptr(), omega.data_ptr()
        a.nu_out, a.var_out, a.best = nu_out.data_ptr(), var_out.data_ptr(), best.data_ptr()
        a.samples_out = None if samples_out is None else samples_out.data_ptr()
        a.r_primal = None if r_primal is None else r_primal.data_ptr()
        a.r_dual = None if r_dual is None else r_dual.data_ptr()
        a.iters_out = None if iters_out is None else iters_out.data_ptr()
        if workspace is None:
            a.workspace, a.workspace_bytes = None, 0
        else:
            a.workspace, a.workspace_bytes = workspace.data_ptr(), int(workspace.numel())
        a.opts = C.pointer(opts) if opts is not None else C.POINTER(L.Options)()
        if static:
            L.check(L.lib().prism_plan_step_static(self._h, C.byref(a), _stream(stream)),
                    "prism_plan_step_static")
        else:
            L.check(L.lib().prism_plan_step(self._h, C.byref(a), _stream(stream)),
                    "prism_plan_step")
        out = {"x": x, "cost": cost, "omega": omega, "nu": nu_out, "var": var_out, "best": best,
               "workspace": workspace}
        if samples_out is not None:
            out["samples"] = samples_out
        return out

    def feasibility(self, v, q0, v0, out=None, stream=None):
        """FP64 per-column violations [N][nj][5]: position, velocity, acceleration, jerk, |x1-v0|."""
        import torch
        if v is None or v.ndim != 3:
            raise ValueError("v: expected a [N][H][n_joints] tensor")
        N = int(v.shape[0])
        _check(v, "v", (N, self.H, self.nj), torch.float32, v.device, optional=False)
        if out is None:
            out = torch.empty((N, self.nj, 5), dtype=torch.float64, device=v.device)
        _check(out, "out", (N, self.nj, 5), torch.float64, v.device)
        q0a = L.dbl_array(np.broadcast_to(np.asarray(q0, dtype=np.float64), (self.nj,)))
        v0a = L.dbl_array(np.broadcast_to(np.asarray(v0, dtype=np.float64), (self.nj,)))
        L.check(L.lib().prism_proj_feasibility(self._h, _ptr(v), N, q0a, v0a, _ptr(out),
                                               _stream(stream)), "prism_proj_feasibility")
        return out


def factor_host(H: int, rho: float, weights=None):
    """prism_factor_host: the FP64 reduced inverse (K, k) built on the host."""
    K = np.zeros((H, H))
    k = np.zeros(H)
    wa = None if weights is None else (C.c_double * 4)(*[float(v) for v in weights])
    L.check(L.lib().prism_factor_host(H, rho, wa, K.ctypes.data_as(C.POINTER(C.c_double)),
                                      k.ctypes.data_as(C.POINTER(C.c_double))),
            "prism_factor_host")
    return K, k


class Batch:
    """Staging object for prism_proj_solve_batch: many requests, one persistent launch.

    solve() takes a list of dicts with keys proj (a Projector), samples, q0, v0,
    iters and optionally out, r_primal, r_dual, iters_out, x_warm, state_warm,
    state_out (tensors as for Projector.solve) and warm_shift. Missing out / r_primal / r_dual
    are allocated. Returns the list of (v_out, r_primal, r_dual).
    """

    def __init__(self):
        h = C.c_void_p()
        L.check(L.lib().prism_batch_create(C.byref(h)), "prism_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            L.lib().prism_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, requests, opts: Optional[L.Options] = None, stream=None):
        import torch
        n = len(requests)
        arr = (L.Request * max(n, 1))()
        keep, outs = [], []
        for i, r in enumerate(requests):
            P = r["proj"]
            x = r["samples"]
            if x is None or x.ndim != 3:
                raise ValueError(f"request {i}: samples must be a [N][H][n_joints] tensor")
            N = int(x.shape[0])
            dev = x.device
            f32 = torch.float32
            traj, col, state = (N, P.H, P.nj), (N, P.nj), (N, P.nj, 4, P.H)
            _check(x, f"request {i} samples", traj, f32, dev, optional=False)
            out = r.get("out")
            out = torch.empty_like(x) if out is None else out
            rp = r.get("r_primal")
            rp = torch.empty(col, dtype=f32, device=dev) if rp is None else rp
            rd = r.get("r_dual")
            rd = torch.empty(col, dtype=f32, device=dev) if rd is None else rd
            _check(out, f"request {i} out", traj, f32, dev)
            _check(rp, f"request {i} r_primal", col, f32, dev)
            _check(rd, f"request {i} r_dual", col, f32, dev)
            _check(r.get("iters_out"), f"request {i} iters_out", col, torch.int32, dev)
            _check(r.get("x_warm"), f"request {i} x_warm", traj, f32, dev)
            _check(r.get("state_warm"), f"request {i} state_warm", state, f32, dev)
            _check(r.get("state_out"), f"request {i} state_out", state, f32, dev)
            q0a = L.dbl_array(np.broadcast_to(np.asarray(r["q0"], dtype=np.float64), (P.nj,)))
            v0a = L.dbl_array(np.broadcast_to(np.asarray(r["v0"], dtype=np.float64), (P.nj,)))
            keep += [q0a, v0a]
            a = arr[i]
            a.proj = P.handle.value
            a.v_samples = x.data_ptr()
            a.N = N
            a.iters = int(r["iters"])
            a.q0 = C.cast(q0a, C.POINTER(C.c_double))
            a.v0 = C.cast(v0a, C.POINTER(C.c_double))
            a.v_out = out.data_ptr()
            a.r_primal = rp.data_ptr()
            a.r_dual = rd.data_ptr()
            for f in ("iters_out", "x_warm", "state_warm", "state_out"):
                t = r.get(f)
                setattr(a, f, None if t is None else t.data_ptr())
            a.warm_shift = 1 if r.get("warm_shift") else 0
            outs.append((out, rp, rd))
        po = C.pointer(opts) if opts is not None else C.POINTER(L.Options)()
        L.check(L.lib().prism_proj_solve_batch(self._h, n, arr, po, _stream(stream)),
                "prism_proj_solve_batch")
        return outs

"""Residual-mode parity of the GPU solver against the oracle's per-column definition.

The GPU stops a tile of 16 consecutive samples of one joint at the first check point
where every column of the tile meets the tolerance; the oracle has no tiles (each
column stops on its own). So a residual-driven GPU run is compared as follows:

* x: the oracle is run to each column's reported iteration count and must agree
  within the form's bar (1e-4 for FP32);
* the reported counts are check points (multiples of check_every, or the cap) and
  equal within a tile;
* the stop was not early: the GPU's own residuals meet tol, and (FP32 form) the
  oracle's at the same count meet tol up to the FP32/FP64 residual margin;
* the stop was not late (FP32 form): at the tile's previous check point at least one
  of its columns was above tol, up to the same margin.

The residual margin covers FP32 rounding of the quantities the residuals are
differences of: 1e-5 + sqrt(L) 2^-24 max_k (|C|^T |y|)_k after L iterations (r_d is
a difference of terms as large as (|C|^T |y|)_k, and the FP32 multiplier accumulates
one rounding of them per iteration, a random walk).
"""

from __future__ import annotations

import numpy as np

from oracle import admm, problem

TILE = 16   # samples per GPU tile (the solver's stopping group)


def residual_margin(O, H, dt, bounds, q0, v0, iters):
    C = np.abs(problem.velocity_unit_rows(H, dt, problem.joint_limits(bounds, 0), q0[0],
                                          v0[0]).C)
    big = np.einsum("rk,njr->njk", C, np.abs(O.y)).max()
    return 1e-5 + np.sqrt(max(1, int(np.max(iters)))) * 2.0 ** -24 * big


def check_residual_mode(x, rp, rd, it, rows, samples, H, dt, bounds, q0, v0, *, tol,
                        check_every, cap, alpha, weights, rho=1.0, xbar=1e-4,
                        check_stops=True, label="", joints=None):
    """x, rp, rd, it: the GPU results of the sampled rows `rows` (whole tiles of the
    batch, in order); samples: the whole batch [N][H][nj]. check_stops: compare the
    stop points with the oracle's residuals (FP32 form only: a reduced-precision run
    follows a different path, so the oracle's residual at the same count says nothing
    about its stop). joints: check only these joints (columns are independent per
    joint). Returns a dict of figures."""
    rows = np.asarray(rows)
    if joints is not None:
        joints = np.asarray(joints)
        x, rp, rd, it = x[:, :, joints], rp[:, joints], rd[:, joints], it[:, joints]
        samples = samples[:, :, joints]
        bounds = bounds.subset(joints)
        q0, v0 = np.asarray(q0)[joints], np.asarray(v0)[joints]
    S = samples[rows]
    res = np.maximum(rp, rd)
    assert np.all(res <= tol), f"{label}: a reported residual is above tol"
    assert np.all((it % check_every == 0) | (it == cap)), f"{label}: count not a check point"
    tiles = rows // TILE
    for t in np.unique(tiles):
        m = tiles == t
        for j in range(it.shape[1]):
            assert len(np.unique(it[m, j])) == 1, f"{label}: tile {t} joint {j} split"
    kw = dict(rho=rho, alpha=alpha, weights=weights)
    O = admm.solve_request(S, H, dt, bounds, q0, v0, iters=it, **kw)
    err = float(np.abs(x - O.x).max())
    margin = residual_margin(O, H, dt, bounds, q0, v0, it)
    o_res = np.maximum(O.r_p, O.r_d)
    out = {"max_abs": err, "margin": margin, "oracle_res_at_stop": float(o_res.max()),
           "iters": (int(it.min()), float(it.mean()), int(it.max()))}
    print(f"{label}: x max-abs {err:.2e} (bar {xbar:.0e}); counts {out['iters']}; oracle "
          f"residual at stop {o_res.max():.2e} (tol {tol:g}, margin {margin:.1e})")
    assert err <= xbar, f"{label}: x {err:.3e} > {xbar:.0e}"
    if check_stops:
        assert np.all(o_res <= tol + margin), f"{label}: stopped early"
        prev = np.where(it > 0, ((it - 1) // check_every) * check_every, 0)
        P = admm.solve_request(S, H, dt, bounds, q0, v0, iters=prev, **kw)
        p_res = np.maximum(P.r_p, P.r_d)
        lowest = np.inf
        for t in np.unique(tiles):
            m = tiles == t
            for j in range(it.shape[1]):
                if it[m, j][0] == 0:
                    continue
                worst = p_res[m, j].max()
                lowest = min(lowest, worst)
                assert worst > tol - margin, f"{label}: tile {t} joint {j} stopped late"
        out["lowest_tile_residual_at_previous_check"] = float(lowest)
    return out

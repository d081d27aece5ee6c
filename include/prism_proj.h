/*
 * prism_proj.h -- C ABI of the MI355X (gfx950) trajectory-projection library.
 *
 * The library projects sampled joint-velocity trajectories onto the set that
 * satisfies joint position, velocity, acceleration and jerk bounds and the
 * initial-velocity condition. This is the projection QP of PRISM (arXiv
 * 2608.25666), Sec. III-A eqs. (proj_cost)-(proj_boundary), in the compact form
 * of Sec. III-D eq. (compact_qp):
 *
 *   x* = argmin 1/2 ||x - x~||^2  s.t.  x_1 = v0,  G x <= h,
 *
 * solved independently per (sample, joint) column (Sec. III-D "Joint-wise
 * separability", "Batch parallelism") with an ADMM splitting whose primal
 * system is factored once per (H, rho) (Sec. III-D "Pre-computable
 * factorization") and whose boundary values only change the bounds (Sec. III-D
 * "Boundary value update").
 *
 * Units: rad, rad/s, rad/s^2, rad/s^3; dt in seconds. Residuals are reported
 * in velocity units (rad/s): every constraint row is scaled by a positive
 * factor (1, 1/dt, dt, dt^2 for the velocity, position, acceleration and jerk
 * rows), which leaves the feasible set and the projection unchanged.
 *
 * Layouts: trajectories are float32 [N][H][n_joints] row-major (step-major,
 * joint-minor per sample, as the stacked vector of Sec. III-D eq. (G_h_def)).
 * Per-column outputs are [N][n_joints].
 *
 * Devices and streams: a handle belongs to the HIP device that was current
 * when it was created; solves must be issued with that device current. Every
 * solve is asynchronous on the caller's hipStream_t; the caller owns all
 * sample/output buffers (device memory on the handle's device) and must keep
 * them alive until the stream reaches the solve. Host arrays (bounds, q0, v0,
 * request tables) are read before the call returns.
 *
 * Errors: every argument check runs before any work is enqueued; on an error
 * nothing is written to any output. NaN inputs propagate to NaN outputs and NaN
 * residuals (not checked on the hot path; prism_proj_feasibility reports them).
 */
#ifndef PRISM_PROJ_H
#define PRISM_PROJ_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRISM_PROJ_ABI_VERSION 4
#define PRISM_MAX_H 128          /* horizon limit: the x-update inverse is staged on-chip */
#define PRISM_MAX_JOINTS 64

typedef struct prism_proj_s* prism_proj_t;   /* opaque, owned by the library */

typedef enum {
  PRISM_OK = 0,
  PRISM_EINVAL = -1,        /* bad argument (sizes, bounds, rho, pointers, options) */
  PRISM_ENOMEM = -2,        /* host or device allocation failed */
  PRISM_EDEVICE = -3,       /* a HIP call failed, or wrong device current */
  PRISM_EINFEASIBLE = -4,   /* a necessary boundary condition fails (see solve) */
  PRISM_EBUSY = -5,         /* server admission refused (budget or queue full) */
  PRISM_EUNSUPPORTED = -6,  /* combination not built into this library */
  PRISM_ETOOLARGE = -7      /* request exceeds a fixed capacity (prism_plan_step_static) */
} prism_status_t;

/* Joint-wise limits (Sec. III-D "Velocity bounds": joint-wise limit vectors).
 * Host arrays of length n_joints, copied by prism_proj_create. Each lower
 * bound must be <= its upper bound and finite. */
typedef struct {
  const double *q_min, *q_max;   /* position, rad      */
  const double *v_min, *v_max;   /* velocity, rad/s    */
  const double *a_min, *a_max;   /* acceleration       */
  const double *j_min, *j_max;   /* jerk               */
} prism_bounds_t;

typedef enum {
  PRISM_PREC_FP32 = 0,   /* x-update GEMM on FP32 MFMA                              */
  PRISM_PREC_BF16 = 1,   /* x-update GEMM operands BF16 (RNE), FP32 accumulation    */
  PRISM_PREC_FP16 = 2    /* x-update GEMM operands FP16 (RNE), FP32 accumulation    */
} prism_precision_t;

/* Solver options. Everything except the GEMM operands is FP32 (clamps, duals,
 * stencils, residuals). */
typedef struct {
  int32_t precision;    /* prism_precision_t                                         */
  int32_t fp32_tail;    /* reduced forms: with tol <= 0 the last fp32_tail of the
                           iterations use the FP32 GEMM. With tol > 0 the reduced
                           GEMM runs until a group meets tol; then (if fp32_tail >
                           0) exactly fp32_tail FP32 iterations follow (check points
                           inside them do not stop the group), and the group stops
                           at their end if it meets tol there, else at the first
                           later check point that does, staying in FP32. Near
                           alpha = 2 the rounded x-update can make the iterates
                           diverge or stall above tol (BF16 at alpha 1.9 and
                           1.95 measured; FP16 did not), so a group whose max
                           residual at a check point exceeds 64 times the lowest
                           it had before restarts from its samples with a cold
                           state in the FP32 form (which stops at the first
                           check point meeting tol; the reported count includes
                           the abandoned iterations), and a group whose residual
                           sets no new low for 500 iterations enters the FP32
                           phase above from its state. Fixed-count runs have no
                           such guard: keep alpha <= 1.85 for BF16 there         */
  float alpha;          /* over-relaxation in (0, 2); 1 = plain ADMM                 */
  float tol;            /* <= 0: run exactly `iters` iterations. > 0: each group of
                           16 samples of one joint stops at the first check point
                           (iteration 0, every check_every iterations, and iters)
                           where all its columns have max(r_primal, r_dual) <= tol */
  int32_t check_every;  /* residual check period (>= 1) when tol > 0                 */
  int32_t tile_waves;   /* waves per 16-sample tile: 0 = the library's choice (one
                           wave), 1 = one wave, 2 = a pair of waves of one workgroup
                           (each holds half of the steps and computes half of the
                           x-update, handing sums, boundary terms and its defect to
                           the other through LDS). The pair shortens a lone H = 100
                           FP32 tile's iteration by about a tenth; elsewhere the
                           hand-overs cost more than the split saves. Two waves need
                           H >= 16, a chunk size ceil(H/8) built into the library
                           (3, 7 or 13), and no warm start or dual-state output;
                           single solves only (PRISM_EUNSUPPORTED otherwise). Results
                           are the same iteration with another FP32 summation order */
  int32_t reserved[2];  /* must be zero                                              */
} prism_options_t;

/* Fill *opts with the defaults: FP32, fp32_tail 0, alpha 1, tol 0, check_every 10,
 * tile_waves 0. */
void prism_options_default(prism_options_t* opts);

/* prism_proj_create -- build the reusable factor for horizon H and step dt.
 *
 * Forms, in FP64 on the host, P = I + rho C^T C for the velocity-unit
 * constraint rows C = [I; L; D1; D2] (Sec. III-D eqs. (pos_stack), (acc_stack),
 * (jerk_stack) scaled to rad/s), eliminates the equality x_1 = v0 from the KKT
 * matrix M of eq. (admm_primal), and keeps K = Pi - Pi e1 e1^T Pi / Pi_11
 * (Pi = P^-1). C is unit-free after the row scaling, so K depends only on
 * (H, rho): dt, the bounds, q0 and v0 enter only the row bounds.
 * FP32/BF16/FP16 copies of K, laid out for the MFMA x-update, are uploaded to
 * the current device.
 *
 * H in [2, PRISM_MAX_H]; n_joints in [1, PRISM_MAX_JOINTS]; dt > 0 finite;
 * rho > 0 finite; bounds with lo <= hi, all finite.
 * Returns PRISM_EINVAL on a bad argument, PRISM_ENOMEM / PRISM_EDEVICE on
 * allocation or HIP failures; *out is written only on PRISM_OK. */
prism_status_t prism_proj_create(int H, int n_joints, double dt, const prism_bounds_t* bounds,
                                 double rho, prism_proj_t* out);

/* prism_proj_create_ex -- as prism_proj_create with a diagonal block penalty.
 *
 * The penalty of the augmented term becomes R = rho * diag(w) with one weight
 * per constraint block (block_weights[0..3]: velocity, position, acceleration,
 * jerk rows), so P = I + C^T R C. The paper uses one scalar penalty (Sec. III-D
 * eq. (aug_lag)); a positive diagonal penalty keeps the same three steps and one
 * reusable factor and has the same fixed point (the projection), but can reach
 * a residual target in far fewer iterations. block_weights = NULL gives unit
 * weights (identical to prism_proj_create). Every weight must be > 0 and
 * finite, else PRISM_EINVAL. u = y / (rho w_b) is the scaled dual of each row. */
prism_status_t prism_proj_create_ex(int H, int n_joints, double dt, const prism_bounds_t* bounds,
                                    double rho, const double* block_weights, prism_proj_t* out);

/* Recommended block weights for a problem family, for rho = 1 and alpha = 1.8:
 * s (1.7, 2.125/H, 13.6, 17) with s = 0.024 / (J dt^2) clipped to [2^-4.5, 2^1.5],
 * J the smallest jerk half-width (j_max - j_min) / 2 over the joints. J dt^2 is
 * the jerk bound in the rows' velocity units; the block ratios were tuned where
 * it is 0.024 (|j| <= 60 rad/s^3 at dt = 0.02, s = 1), and the best uniform scale
 * falls in proportion as that bound widens (sweeps over dt 0.02-0.1, jerk bounds
 * 15-960, velocity bounds 1-3.14, acceleration bounds 2-32, H 15-100). The
 * weights change the iteration's path, never its fixed point (the projection).
 * They assume the position rows rarely bind; for requests whose trajectories run
 * into the position limits a position weight w[1] 4x (dt = 0.02) to 16x (dt =
 * 0.05) larger converged 3-12x faster in the same sweeps, at a cost where the
 * positions stay clear (a handle with such weights via prism_proj_create_ex).
 * Writes w[0..3]; PRISM_EINVAL for H outside 2..PRISM_MAX_H, a bad joint count,
 * dt not positive and finite, missing bounds or a jerk width that is not
 * positive and finite (nothing written then). */
prism_status_t prism_default_block_weights(int H, int n_joints, double dt,
                                           const prism_bounds_t* bounds, double* w);

/* Set the handle's default options (used by prism_proj_solve). Not safe to
 * call while another thread issues solves on the same handle. */
prism_status_t prism_proj_set_options(prism_proj_t p, const prism_options_t* opts);
prism_status_t prism_proj_get_options(prism_proj_t p, prism_options_t* opts);

/* prism_proj_solve -- project N sampled trajectories (the hot path).
 *
 * v_samples: device, float32 [N][H][n_joints] (x~, the raw samples).
 * q0, v0:    host, float64 [n_joints] (theta_init, thetadot_init), shared by
 *            all N samples. They set the first-row bounds (Sec. III-D
 *            "Boundary value update") and x_1 = v0 (eq. (A_b_def)).
 * iters:     iteration count (tol <= 0) or cap (tol > 0); >= 0.
 * v_out:     device, float32 [N][H][n_joints]; may alias v_samples.
 * r_primal:  device, float32 [N][n_joints]: max_i |(C x)_i - z_i| (rad/s).
 * r_dual:    device, float32 [N][n_joints]: max over steps k >= 2 of
 *            |x_k - x~_k + (C^T y)_k| (rad/s), the stationarity gap.
 * Either residual pointer may be NULL.
 * Returns PRISM_EINFEASIBLE when v0 is outside [v_min, v_max], q0 + dt*v0
 * is outside [q_min, q_max], or 0 is outside [a_min, a_max] for some joint (the
 * rows of step 1 fixed by x_1 = v0 would be unsatisfiable; jerk rows start at
 * step 2, eq. (jerk_stack), so the jerk bounds need not contain 0). N = 0 is a
 * no-op. Any number of solves may be in flight on one handle, on any streams:
 * a solve that takes over a tile-queue counter set from an earlier one waits on
 * its own stream for that solve to finish (64 sets per handle; under graph
 * capture this ordering is not recorded, so a captured graph must not be
 * launched while an earlier launch of it is still running). */
prism_status_t prism_proj_solve(prism_proj_t p, const float* v_samples, int N,
                                const double* q0, const double* v0, int iters, float* v_out,
                                float* r_primal, float* r_dual, hipStream_t stream);

/* Extended solve: optional per-column iteration counts, warm start and dual
 * state, and per-call options.
 *   opts:        NULL = the handle's options.
 *   iters_out:   device int32 [N][n_joints] or NULL: iterations performed.
 *   x_warm:      device float32 [N][H][n_joints] or NULL: initial iterate
 *                (its first step is replaced by v0). NULL = start from v_samples.
 *   state_warm:  device float32 [N][n_joints][4][H] or NULL: dual state to start
 *                from, q = (1 - alpha) z + u per constraint row (z the slack,
 *                u = y / (rho w_b) the scaled multiplier; with alpha = 1 it is
 *                u). Blocks: velocity, position, acceleration, jerk rows; entry
 *                0 of the jerk block is unused (jerk rows are steps 2..H).
 *                NULL = cold start (previous slack C x0, multiplier 0).
 *   state_out:   device float32 [N][n_joints][4][H] or NULL: final q, same
 *                layout, for warm-starting the next MPC step.
 *   warm_shift:  0 or 1. With 1 the warm start is advanced by one MPC step (time
 *                moves by dt): step k takes the previous step k + 1, the last
 *                step repeating, for the iterate x_warm and, row block by row
 *                block, for the scaled multiplier and the slack's deviation from
 *                C x_warm (both held in state_warm); the slack is then rebuilt
 *                on the shifted iterate: q' = (1 - alpha) C x' +
 *                shift(q - (1 - alpha) C x_warm), where x_warm's first step is
 *                the previous boundary velocity. The acceleration row of step 1
 *                (fixed by x_1 = v0) restarts at zero. Requires x_warm when
 *                state_warm is given (PRISM_EINVAL otherwise). x_warm may alias
 *                v_out and state_warm may alias state_out (each column is read
 *                before it is written).
 * The first pass is a relaxed slack/multiplier step t = alpha C x0 + q0,
 * z0 = clip(t), u0 = t - z0, with q0 = state_warm or (1 - alpha) C x0. */
typedef struct {
  const float* v_samples;
  int32_t N;
  int32_t iters;
  const double* q0;
  const double* v0;
  float* v_out;
  float* r_primal;
  float* r_dual;
  int32_t* iters_out;
  const float* x_warm;
  const float* state_warm;
  float* state_out;
  const prism_options_t* opts;
  int32_t warm_shift;
} prism_solve_args_t;

prism_status_t prism_proj_solve_ex(prism_proj_t p, const prism_solve_args_t* args,
                                   hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched solve: many requests (each with its own handle, hence its own H,
 * joint count, dt, bounds and factor) in one persistent launch (Sec. III-D
 * "Batch parallelism": only the samples and right-hand sides differ between
 * QPs; here the factors may differ too). Requests are ordered longest work
 * first; each workgroup stages one request's factor and its waves claim that
 * request's tiles (16 samples of one joint each) one at a time from per-XCD
 * queues, the workgroup moving on to the first request with tiles left once
 * its request is drained (workgroups start spread over the requests in
 * proportion to their work).
 * A batch whose horizons all fall in {17..20, 49..52, 97..100} (chunk sizes
 * {5, 13, 25}) runs as two launches: horizons 97..100 (one wave per SIMD) on
 * the caller's stream and 17..20 and 49..52 (two waves per SIMD) on an
 * internal stream of the staging object, forked from the caller's stream after
 * the tables are uploaded and joined back to it, so the second launch fills the
 * CUs the first one frees; other mixes run one launch per chunk-size class
 * (chunks 2-8, 9-12, 13-16, 17-24, 25-28, 29-30, 31, 32), in order on the
 * caller's stream.
 * Either way the caller's stream is ordered after the whole batch. (The server's
 * launches, which overlap on streams of their own, keep both on one stream.)
 * ------------------------------------------------------------------------- */
typedef struct prism_batch_s* prism_batch_t;   /* staging buffers for request tables */

typedef struct {
  prism_proj_t proj;        /* the request's handle (all on one device)             */
  const float* v_samples;   /* device [N][H][n_joints]                               */
  int32_t N;                /* samples (0 = nothing to do)                           */
  int32_t iters;            /* iteration count / cap, >= 0                           */
  const double* q0;         /* host [n_joints]                                       */
  const double* v0;         /* host [n_joints]                                       */
  float* v_out;             /* device [N][H][n_joints]; may alias v_samples          */
  float* r_primal;          /* device [N][n_joints] or NULL                          */
  float* r_dual;            /* device [N][n_joints] or NULL                          */
  int32_t* iters_out;       /* device [N][n_joints] or NULL                          */
  const float* x_warm;      /* device [N][H][n_joints] or NULL                       */
  const float* state_warm;  /* device [N][n_joints][4][H] or NULL                    */
  float* state_out;         /* device [N][n_joints][4][H] or NULL                    */
  int32_t warm_shift;       /* 0 or 1, as in prism_solve_args_t                      */
} prism_request_t;

/* Create / destroy the staging object (pinned host and device request tables,
 * grown on demand). One object serves one stream at a time: a call waits until
 * the previous call's tables have been copied to the device. */
prism_status_t prism_batch_create(prism_batch_t* out);
void prism_batch_destroy(prism_batch_t b);

/* Solve every request with the same options (NULL = defaults). All checks of
 * every request run before anything is enqueued; PRISM_EINVAL / PRISM_EINFEASIBLE
 * name no request, and nothing is written on error. Each request's outputs are
 * exactly what prism_proj_solve_ex would produce for it alone. */
prism_status_t prism_proj_solve_batch(prism_batch_t b, int n_req, const prism_request_t* reqs,
                                      const prism_options_t* opts, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * One iteration of the sampling optimizer around the projection (Alg. 1 with a
 * synthetic cost in place of the simulator rollouts):
 *   1. draw x~_n = nu + sigma .* z_n, z standard normal (the Gaussian of Alg. 1;
 *      diagonal covariance sigma^2), in the solve kernel's load: element e of
 *      [N][H][n_joints] (row-major index) takes Philox4x32-10 at counter
 *      (e mod 2^32, e div 2^32, stream mod 2^32, stream div 2^32), key
 *      (seed mod 2^32, seed div 2^32); with its first two words as 23-bit
 *      uniforms u = (w div 2^9 + 1/2) / 2^23, z = sqrt(-2 ln u0) cos(2 pi u1);
 *   2. project every sample (Sec. III; the handle's factor and options);
 *   3. score each projected sample: c_n = sum_k sum_j w_pos (theta_kj - ref_kj)^2
 *      + w_vel x_kj^2 with theta_k = q0 + dt sum_{i<=k} x_i (eq. (pos_stack)),
 *      summed in FP64 over joints;
 *   4. weights omega_n = exp(-c_n / tau) / sum_m exp(-c_m / tau)
 *      (eq. (weight_update)), computed in FP64 with the minimum cost taken out;
 *   5. nu' = sum_n omega_n x_n (eq. (mean_update_new)) and
 *      var' = sum_n omega_n (x_n - nu')^2 + eps (diagonal of eq. (cov_update_new)),
 *      accumulated in FP64, stored FP32; best = argmin_n c_n (lowest index on ties).
 * All device arrays are row-major FP32 unless stated; caller-owned.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* nu;          /* device [H][n_joints]: mean of the sampling Gaussian      */
  const float* sigma;       /* device [H][n_joints]: standard deviations                */
  uint64_t seed;            /* generator key                                            */
  uint64_t stream;          /* generator stream (e.g. the optimizer iteration)          */
  int32_t N;                /* samples, >= 1                                            */
  int32_t iters;            /* iteration count / cap of the projection                  */
  const double* q0;         /* host [n_joints]                                          */
  const double* v0;         /* host [n_joints]                                          */
  const float* theta_ref;   /* device [H][n_joints]: reference positions (rad)          */
  float w_pos, w_vel;       /* cost weights, >= 0                                       */
  float tau;                /* softmax temperature, > 0                                 */
  float eps;                /* covariance floor, >= 0                                   */
  float* x_out;             /* device [N][H][n_joints]: projected samples               */
  float* samples_out;       /* device [N][H][n_joints] or NULL: the drawn samples       */
  double* cost;             /* device [N] or NULL: c_n                                  */
  double* omega;            /* device [N] or NULL: weights                              */
  float* nu_out;            /* device [H][n_joints]: nu'                                */
  float* var_out;           /* device [H][n_joints]: var'                               */
  int32_t* best;            /* device [1] or NULL: index of the lowest-cost sample      */
  float* r_primal;          /* device [N][n_joints] or NULL                             */
  float* r_dual;            /* device [N][n_joints] or NULL                             */
  int32_t* iters_out;       /* device [N][n_joints] or NULL                             */
  void* workspace;          /* device, prism_plan_workspace_bytes(H, n_joints, N) bytes */
  size_t workspace_bytes;
  const prism_options_t* opts;   /* NULL = the handle's options                        */
} prism_plan_args_t;

/* Device workspace one prism_plan_step call needs (0 for invalid sizes). */
size_t prism_plan_workspace_bytes(int H, int n_joints, int N);

/* Enqueues the iteration on `stream`. PRISM_EINVAL (bad pointer, N < 1, tau <= 0,
 * negative weights or eps, small workspace), PRISM_EINFEASIBLE (as
 * prism_proj_solve); nothing is enqueued on error. Calls that share a workspace
 * must be ordered (same stream). */
prism_status_t prism_plan_step(prism_proj_t p, const prism_plan_args_t* a, hipStream_t stream);

/* prism_plan_step_static -- prism_plan_step for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. It makes no allocation of any kind (no hipMalloc/hipFree, no
 * library allocator): the workspace and the solve's tile-queue counters live in a
 * static device array of PRISM_PLAN_STATIC_WORKSPACE_BYTES (+ 256 bytes for the
 * counters) that each GPU the library runs on holds until the process ends.
 * a->workspace and a->workspace_bytes are ignored; every other argument, check and
 * result is that of prism_plan_step (same kernels, bit-identical outputs).
 * Returns PRISM_ETOOLARGE, with nothing enqueued, when
 * prism_plan_workspace_bytes(H, n_joints, N) exceeds PRISM_PLAN_STATIC_WORKSPACE_BYTES
 * (N <= 92 666 samples at 12 joints and H = 50). All calls on one GPU share
 * its array: calls that overlap in time on that GPU (different streams, or other
 * threads) race and give wrong results; calls ordered on one stream are safe. The
 * counters are cleared by a kernel at the start of every call. */
#define PRISM_PLAN_STATIC_WORKSPACE_BYTES ((size_t)8 << 20)
prism_status_t prism_plan_step_static(prism_proj_t p, const prism_plan_args_t* a,
                                      hipStream_t stream);

/* ---------------------------------------------------------------------------
 * prism_proj_literal -- the Bregman iteration exactly as Sec. III-D prints it
 * (eqs. (admm_zeta), (admm_primal)/(admm_KKT), (admm_dual)), a fixed number of
 * passes in FP64. NOT the projection: the multiplier lambda is kept in the
 * primal space and the slack step does not see it, so every feasible x with
 * lambda = x - x~ is a fixed point; the passes stop at a feasible trajectory
 * near the sample, not at the nearest one. This is the fast mode behind the
 * paper's remark that ten to twenty iterations suffice (Sec. III-D
 * "Convergence"); prism_proj_solve is the projection.
 *
 * Per (sample, joint) column, with G = [C; -C] and h in the paper's physical
 * row scaling (eq. (G_h_def)), penalty delta, lambda_0 = 0 and
 * x_0 = x_init (or the sample) with its first step set to v0:
 *   zeta'   = max(0, h - G x)
 *   x'      = argmin of eq. (aug_lag) in x subject to x_1 = v0, i.e.
 *             (I + delta G^T G) x' + A^T mu = x~ + lambda + delta G^T (h - zeta')
 *   lambda' = lambda - (delta/2) G^T (G x' - h + zeta').
 * The handle supplies H, dt, the bounds and the device; its options and block
 * weights are not used. The factor of I + delta G^T G is built on the host on
 * the first call with a given delta (one device allocation and a blocking copy,
 * on the calling thread) and kept until prism_proj_destroy; at most 64
 * distinct deltas per handle (PRISM_ENOMEM beyond).
 * Arithmetic is FP64 throughout (samples are widened on load, x is rounded to
 * FP32 on store). v_out may equal v_samples or x_init.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* v_samples;   /* device [N][H][n_joints]: x~                                */
  const float* x_init;      /* device [N][H][n_joints] or NULL: first iterate (x~ if NULL) */
  float* v_out;             /* device [N][H][n_joints]: the iterate after `iters` passes   */
  double* violation;        /* device [N][n_joints] or NULL: largest bound violation of
                               that iterate over all rows of G x <= h, in each row's own
                               physical unit (rad, rad/s, rad/s^2, rad/s^3), >= 0          */
  int32_t N;                /* samples, >= 0 (0: nothing enqueued)                         */
  int32_t iters;            /* passes, >= 0                                                */
  double delta;             /* penalty of eq. (aug_lag), > 0 and finite                    */
  const double* q0;         /* host [n_joints]                                             */
  const double* v0;         /* host [n_joints]                                             */
} prism_literal_args_t;

/* Enqueues the passes on `stream`. PRISM_EINVAL (null pointer, N < 0, iters < 0,
 * delta not positive), PRISM_EINFEASIBLE (as prism_proj_solve), PRISM_EDEVICE
 * (wrong device current, launch failure), PRISM_ENOMEM (factor allocation);
 * nothing is enqueued on error. */
prism_status_t prism_proj_literal(prism_proj_t p, const prism_literal_args_t* a,
                                  hipStream_t stream);

/* prism_proj_feasibility -- FP64 final check of trajectories (device kernel).
 * For each column writes to viol (device, float64 [N][n_joints][5]) the largest
 * violation of the position (rad), velocity (rad/s), acceleration (rad/s^2)
 * and jerk (rad/s^3) bounds, and |x_1 - v0|, recomputing positions by forward
 * Euler and derivatives by backward differences in FP64 (Sec. III-D
 * "From Joint-Velocity Sequences to Derivative Bounds"). NaN input gives NaN. */
prism_status_t prism_proj_feasibility(prism_proj_t p, const float* v, int N, const double* q0,
                                      const double* v0, double* viol, hipStream_t stream);

/* Release the handle and its device memory. The caller must ensure no solve
 * that uses it is still pending on any stream. NULL is ignored. */
void prism_proj_destroy(prism_proj_t p);

/* Introspection for tests and tools. */
int prism_proj_horizon(prism_proj_t p);
int prism_proj_joints(prism_proj_t p);

/* Copy the FP64 reduced inverse K (H*H, row-major) and k (H) built by create
 * into host arrays. Host-only; usable without a GPU via prism_factor_host. */
prism_status_t prism_proj_get_factor(prism_proj_t p, double* K, double* k);
prism_status_t prism_proj_get_weights(prism_proj_t p, double* w);

/* Host-only factor build (no device work), same arithmetic as create:
 * K (H*H row-major) and k (H); w = block weights or NULL for ones.
 * Returns PRISM_EINVAL on bad arguments. */
prism_status_t prism_factor_host(int H, double rho, const double* w, double* K, double* k);

const char* prism_status_str(prism_status_t s);
int prism_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PRISM_PROJ_H */

/* prism_server.h -- continuous-batching server for the projection QP.
 *
 * Many MPC controllers (each with its own handle: horizon, joints, dt, bounds,
 * factor) submit projection requests as they arrive. A worker thread admits
 * them into batched persistent launches (prism_proj_solve_batch's kernels)
 * while earlier launches are still on the GPU: up to `max_inflight` launches
 * run at once on their own streams, so work that arrives during a launch starts
 * on the compute units the launch is releasing instead of waiting for it
 * (Sec. III-D: every sample and joint is an independent QP; the paper runs them
 * in parallel on the GPU for one controller, the server shares the GPU among
 * many). A launch's persistent grid is capped at `grid_share` percent of the
 * GPU's workgroup slots, so a request that arrives while a large launch runs
 * starts on the remaining slots at once instead of after it.
 *
 * Device-resident state: each controller's factor (its handle) and its warm
 * state, the last projected trajectories [max_N][H][n_joints] and the dual
 * state [max_N][n_joints][4][H] (FP32), live on the GPU. The warm state sits in
 * one device pool of `hbm_budget` bytes allocated at creation. A request is
 * admitted when its controller has no request in flight and its warm state is
 * resident or can be made so, evicting the state of idle controllers least
 * recently used first (that controller's next request starts cold). Admission
 * is first come, first served.
 *
 * Warm start: a controller's request with the same sample count as its
 * previous one starts from that solve's result advanced by one step
 * (prism_solve_args_t.warm_shift); otherwise it starts cold.
 *
 * Threading: every call may come from any host thread. Caller-owned buffers
 * (samples, outputs) must stay valid until the request is done. The device
 * that is current at prism_server_create serves every request; all handles
 * must belong to it.
 */
#ifndef PRISM_SERVER_H
#define PRISM_SERVER_H

#include <stddef.h>
#include <stdint.h>

#include "prism_proj.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prism_server_s* prism_server_t;

typedef struct {
  size_t hbm_budget;        /* bytes of device memory for controllers' warm state    */
  int32_t max_inflight;     /* launches on the GPU at once, 1..4                     */
  int32_t max_batch;        /* requests per launch, >= 1                             */
  int32_t max_queue;        /* queued requests before submit returns PRISM_EBUSY     */
  int32_t grid_share;       /* percent (1..100) of the GPU's workgroup slots one
                               launch's persistent grid may take; the rest stays
                               free for requests that arrive while it runs          */
  prism_options_t opts;     /* solver options for every request                      */
} prism_server_config_t;

/* Defaults: 1 GiB budget, 2 in flight, 64 per launch, 65536 queued, grid share
 * 75, options as prism_options_default. */
void prism_server_config_default(prism_server_config_t* cfg);

/* Allocates the pool, the streams and the worker thread on the current device.
 * PRISM_EINVAL for a bad configuration, PRISM_ENOMEM / PRISM_EDEVICE on HIP
 * failures. */
prism_status_t prism_server_create(const prism_server_config_t* cfg, prism_server_t* out);

/* Stops the worker after the launches in flight complete; queued requests are
 * dropped (their tickets report PRISM_SERVER_FAILED). Frees everything. */
void prism_server_destroy(prism_server_t s);

/* Registers a controller using handle `proj` (which must outlive the server)
 * with up to max_N samples per request. Its warm state takes
 * 5 * max_N * H * n_joints * 4 bytes of the pool while resident.
 * PRISM_ENOMEM if that exceeds the whole budget. */
prism_status_t prism_server_add_controller(prism_server_t s, prism_proj_t proj, int32_t max_N,
                                           int32_t* ctrl_id);

typedef struct {
  const float* v_samples;   /* device [N][H][n_joints]                              */
  int32_t N;                /* 0 <= N <= max_N (N = 0 completes at once)            */
  int32_t iters;            /* iteration count (tol <= 0) or cap (tol > 0)          */
  const double* q0;         /* host [n_joints], copied at submit                    */
  const double* v0;         /* host [n_joints], copied at submit                    */
  float* v_out;             /* device [N][H][n_joints]                              */
  float* r_primal;          /* device [N][n_joints] or NULL                         */
  float* r_dual;            /* device [N][n_joints] or NULL                         */
  int32_t* iters_out;       /* device [N][n_joints] or NULL                         */
} prism_serve_request_t;

/* Queues a request; returns at once with its ticket. Checks as
 * prism_proj_solve (PRISM_EINVAL, PRISM_EINFEASIBLE) before queueing;
 * PRISM_EBUSY when max_queue requests are waiting. */
prism_status_t prism_server_submit(prism_server_t s, int32_t ctrl_id,
                                   const prism_serve_request_t* req, int64_t* ticket);

typedef enum {
  PRISM_SERVER_QUEUED = 0,
  PRISM_SERVER_RUNNING = 1,
  PRISM_SERVER_DONE = 2,
  PRISM_SERVER_FAILED = 3
} prism_server_state_t;

typedef struct {
  int32_t state;            /* prism_server_state_t                                 */
  int32_t error;            /* prism_status_t of a failed request                   */
  int32_t warm;             /* 1 if it started from the controller's previous solve */
  int32_t batch_size;       /* requests in its launch                               */
  int64_t t_submit_ns;      /* CLOCK_MONOTONIC nanoseconds (prism_server_now_ns)    */
  int64_t t_launch_ns;      /* its launch was enqueued                              */
  int64_t t_done_ns;        /* the worker saw its launch complete                   */
} prism_ticket_info_t;

/* Current state of a ticket without blocking. PRISM_EINVAL for an unknown or
 * released ticket. */
prism_status_t prism_server_poll(prism_server_t s, int64_t ticket, prism_ticket_info_t* info);

/* Blocks until the ticket is done or failed, or timeout_ms passes (< 0: no
 * limit); PRISM_EBUSY on timeout. */
prism_status_t prism_server_wait(prism_server_t s, int64_t ticket, int64_t timeout_ms,
                                 prism_ticket_info_t* info);

/* Forgets a finished ticket (its record is kept until released). PRISM_EBUSY
 * if it is still queued or running. */
prism_status_t prism_server_release(prism_server_t s, int64_t ticket);

typedef struct {
  int64_t submitted, completed, failed, launches, evictions;
  int64_t queued, running;          /* now                                         */
  int64_t max_concurrent_launches;  /* most launches seen in flight at once        */
  int64_t pool_bytes, pool_used;    /* warm-state pool                             */
} prism_server_stats_t;

prism_status_t prism_server_stats(prism_server_t s, prism_server_stats_t* out);

/* CLOCK_MONOTONIC in nanoseconds: the clock of prism_ticket_info_t. */
int64_t prism_server_now_ns(void);

#ifdef __cplusplus
}
#endif

#endif /* PRISM_SERVER_H */

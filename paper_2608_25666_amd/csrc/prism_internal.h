// Library-internal declarations shared by the ABI front ends (single solve,
// batched solve, server).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <utility>
#include <vector>

#include "admm_kernels.h"
#include "counter_ring.h"
#include "kernel_args.h"
#include "prism_proj.h"

// Tile-queue counter sets per handle (kXcdQueues counters each). Solves take them
// in turn; a set is reused only after the launch that last used it has finished
// (its completion event is waited for on the new solve's stream), so any number
// of solves may be in flight on any streams.
constexpr int kCounterRing = 64;

struct prism_proj_s {
  int H = 0, nj = 0, HQ = 0, device = 0;
  double dt = 0.0, rho = 0.0;
  double w[4] = {1.0, 1.0, 1.0, 1.0};   // block penalty weights (velocity, position, acceleration, jerk)
  std::vector<double> bnd;          // [8][nj]: q_min q_max v_min v_max a_min a_max j_min j_max
  std::vector<double> K, k;         // FP64 master factor
  prism_options_t opts{};
  void* frag_bf16 = nullptr;        // device: FP32 fragments then BF16 fragments
  void* frag_f16 = nullptr;         // device: FP32 fragments then FP16 fragments
  double* d_bounds = nullptr;       // device copy of bnd
  int* d_counters = nullptr;        // ring of tile-queue counter sets
  std::mutex ring_mu;               // guards ring and ring_ev
  prism::CounterRing<kCounterRing> ring;
  hipEvent_t ring_ev[kCounterRing] = {};   // completion of each set's last launch
  int f32_bytes = 0, b16_bytes = 0;
  // two-wave tiles (H >= kPairMinH): eight chunks of HP rows, pair-layout fragments
  int HP = 0;
  void* pair_frag_bf16 = nullptr;   // device: FP32 pair fragments then BF16 pair fragments
  void* pair_frag_f16 = nullptr;    // device: FP32 pair fragments then FP16 pair fragments
  int pair_f32_bytes = 0, pair_b16_bytes = 0;
  std::mutex lit_mu;                              // guards lit
  std::vector<std::pair<double, double*>> lit;    // device factors of the printed iteration, per delta
};

namespace prism {

constexpr int kPairMinH = 16;   // shortest horizon with two-wave tiles (chunks of >= 2 rows)

// The two-wave tile kernel for a solve, or null when the solve cannot use it (horizon,
// chunk size not built, warm start, dual state or sample drawing requested).
PairKernelFn pick_pair_kernel(const prism_proj_s* p, int precision);
int pair_lds_bytes(const prism_proj_s* p, int precision);
// As launch_solve, for the two-wave tile kernel.
prism_status_t launch_pair(prism_proj_s* p, SolveKernelArgs& K, const prism_options_t* o,
                           PairKernelFn fn, hipStream_t stream);

// Frees the printed iteration's device factors of a handle.
void release_literal_factors(prism_proj_s* p);

// Row bounds of every joint for boundary values (q0, v0); PRISM_EINFEASIBLE if
// the first rows (fixed by x_1 = v0) cannot hold.
prism_status_t fill_joint_params(const prism_proj_s* p, const double* q0, const double* v0,
                                 JointRowParams* jp);
SolveKernelFn pick_kernel(int HQ, bool exact, int precision);
int solve_lds_bytes(const prism_proj_s* p, int precision, int waves);
int solve_frag_bytes(const prism_proj_s* p, int precision);
prism_status_t validate_options(const prism_options_t* o);
int kernel_blocks_per_cu(const void* fn, int lds_bytes);
// Fills the solver fields of K (the caller sets samples, outputs, N, iters, jp and
// the optional sampling / cost parts), clears the tile queues and launches fn.
// counters: kXcdQueues device ints owned by the caller, or null to take a set from
// the handle's ring. waves: the kernel's waves per workgroup (its launch bound / 64).
prism_status_t launch_solve(prism_proj_s* p, SolveKernelArgs& K, const prism_options_t* o,
                            SolveKernelFn fn, hipStream_t stream, int* counters = nullptr,
                            int waves = kWaves);
prism_status_t check_device(const prism_proj_s* p);   // occupancy, cached per (kernel, LDS)
int device_cus();

// One request of a batched launch (host-side description).
struct BatchDesc {
  const prism_proj_s* p;
  const float* xin;
  float* xout;
  float* xsave;      // second copy of x or null
  float* rp;
  float* rd;
  int* itout;
  const float* xw;
  const float* uw;
  float* uout;
  int N, iters, shift;
  const double* q0;  // host [nj]
  const double* v0;  // host [nj]
};

// Validates every request, then enqueues the request tables and the batched
// launch(es) on `stream` using the staging object b (see prism_proj_solve_batch).
// grid_pct caps each persistent grid at that percent of the workgroup slots.
prism_status_t enqueue_batch(prism_batch_s* b, const BatchDesc* reqs, int n_req,
                             const prism_options_t& opts, hipStream_t stream, int grid_pct = 100);
hipError_t launch_feasibility(const FeasKernelArgs& a, hipStream_t stream);

}  // namespace prism

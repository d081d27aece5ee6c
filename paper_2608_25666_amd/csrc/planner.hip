// One iteration of the sampling optimizer around the projection (declared in
// include/prism_proj.h as prism_plan_step): a solve launch that draws its samples
// in the load and scores each projected column in the epilogue, then the softmax
// weights over the samples and the weighted mean / diagonal covariance update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>

#include "admm_kernels.h"
#include "prism_internal.h"
#include "prism_proj.h"

using namespace prism;

namespace {

constexpr int kWeightThreads = 1024;
constexpr int kMomentThreads = 256;
constexpr int kMaxMomentBlocks = 256;

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int moment_blocks(int N) {
  const int per = 256;
  return std::max(1, std::min(kMaxMomentBlocks, (N + per - 1) / per));
}

// Sample costs (sum over joints, FP64), the lowest-cost sample, and the weights
// exp(-(c - c_min) / tau) / sum (eq. (weight_update) with the minimum taken out).
__global__ __launch_bounds__(kWeightThreads) void plan_weights_kernel(
    const float* __restrict__ cost_col, int N, int nj, double tau, double* __restrict__ cost,
    double* __restrict__ omega, int* __restrict__ best) {
  __shared__ double sv[kWeightThreads];
  __shared__ int si[kWeightThreads];
  const int tid = threadIdx.x;
  double mn = INFINITY;
  int mi = INT_MAX;
  for (int n = tid; n < N; n += kWeightThreads) {
    double c = 0.0;
    for (int j = 0; j < nj; ++j) c += (double)cost_col[(size_t)n * nj + j];
    cost[n] = c;
    if (c < mn) {
      mn = c;
      mi = n;
    }
  }
  sv[tid] = mn;
  si[tid] = mi;
  __syncthreads();
  for (int s = kWeightThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double o = sv[tid + s];
      const int oi = si[tid + s];
      if (o < sv[tid] || (o == sv[tid] && oi < si[tid])) {
        sv[tid] = o;
        si[tid] = oi;
      }
    }
    __syncthreads();
  }
  const double cmin = sv[0];
  const int bi = si[0];
  __syncthreads();
  double z = 0.0;
  for (int n = tid; n < N; n += kWeightThreads) z += exp(-(cost[n] - cmin) / tau);
  sv[tid] = z;
  __syncthreads();
  for (int s = kWeightThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sv[tid] += sv[tid + s];
    __syncthreads();
  }
  const double Z = sv[0];
  for (int n = tid; n < N; n += kWeightThreads) omega[n] = exp(-(cost[n] - cmin) / tau) / Z;
  if (tid == 0) *best = bi;
}

// Per-block partial sums over a slab of samples: sum w x and sum w x^2 for every
// (step, joint) entry; consecutive threads read consecutive entries of a sample.
__global__ __launch_bounds__(kMomentThreads) void plan_moments_partial_kernel(
    const float* __restrict__ x, const double* __restrict__ omega, int N, int E, int per_block,
    double* __restrict__ part) {
  const int n0 = blockIdx.x * per_block;
  const int n1 = min(N, n0 + per_block);
  for (int e = threadIdx.x; e < E; e += kMomentThreads) {
    double a1 = 0.0, a2 = 0.0;
    for (int n = n0; n < n1; ++n) {
      const double w = omega[n];
      const double v = (double)x[(size_t)n * E + e];
      a1 += w * v;
      a2 += w * v * v;
    }
    part[((size_t)blockIdx.x * E + e) * 2 + 0] = a1;
    part[((size_t)blockIdx.x * E + e) * 2 + 1] = a2;
  }
}

// nu' = sum_n w_n x_n; var' = sum_n w_n x_n^2 - nu'^2 + eps (the weights sum to
// one, so this is eq. (cov_update_new)'s weighted spread about nu').
__global__ __launch_bounds__(kMomentThreads) void plan_moments_final_kernel(
    const double* __restrict__ part, int G, int E, double eps, float* __restrict__ nu,
    float* __restrict__ var) {
  const int e = blockIdx.x * kMomentThreads + threadIdx.x;
  if (e >= E) return;
  double a1 = 0.0, a2 = 0.0;
  for (int b = 0; b < G; ++b) {
    a1 += part[((size_t)b * E + e) * 2 + 0];
    a2 += part[((size_t)b * E + e) * 2 + 1];
  }
  nu[e] = (float)a1;
  var[e] = (float)(fmax(a2 - a1 * a1, 0.0) + eps);
}

SolveKernelFn pick_plan_kernel(int HQ, int precision) {
  switch (precision) {
    case PRISM_PREC_FP32: return plan_kernel_f32(HQ);
    case PRISM_PREC_BF16: return plan_kernel_bf16(HQ);
    case PRISM_PREC_FP16: return plan_kernel_f16(HQ);
    default: return nullptr;
  }
}

bool fin(double v) { return std::isfinite(v); }

// Scratch of prism_plan_step_static, one copy per GPU for the life of the process:
// the solve's tile-queue counters (cleared by a kernel before every launch), then
// the workspace of prism_plan_step (every byte of it written before it is read).
constexpr size_t kStaticCounterBytes = 256;
constexpr size_t kStaticWorkspaceBytes = PRISM_PLAN_STATIC_WORKSPACE_BYTES;
static_assert(kXcdQueues * sizeof(int) <= kStaticCounterBytes, "counters fit");
static __device__ __align__(256) unsigned char scratch[kStaticCounterBytes + kStaticWorkspaceBytes];

// Device address of `scratch` per device, looked up once per device with that device
// current (host code must not use the array's name: it is a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

prism_status_t static_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return PRISM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PRISM_EDEVICE;
    g_scratch[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch[dev];
  return PRISM_OK;
}

}  // namespace

extern "C" size_t prism_plan_workspace_bytes(int H, int n_joints, int N);

namespace {

// One optimizer iteration with the given workspace and, if not null, the given
// tile-queue counters (else a set of the handle's ring).
prism_status_t plan_step_impl(prism_proj_t p, const prism_plan_args_t* a, hipStream_t stream,
                              void* workspace, size_t workspace_bytes, int* counters) {
  const prism_options_t* o = a->opts ? a->opts : &p->opts;
  prism_status_t st = validate_options(o);
  if (st != PRISM_OK) return st;
  if (o->tile_waves == 2) return PRISM_EUNSUPPORTED;   // the optimizer step uses one-wave tiles
  if (a->N < 1 || a->iters < 0 || !a->q0 || !a->v0 || !a->nu || !a->sigma || !a->theta_ref ||
      !a->x_out || !a->nu_out || !a->var_out)
    return PRISM_EINVAL;
  if (!fin(a->tau) || a->tau <= 0.0f || !fin(a->eps) || a->eps < 0.0f || !fin(a->w_pos) ||
      a->w_pos < 0.0f || !fin(a->w_vel) || a->w_vel < 0.0f)
    return PRISM_EINVAL;
  if ((long long)a->N * p->H * p->nj > (1ll << 40)) return PRISM_EINVAL;
  const size_t need = prism_plan_workspace_bytes(p->H, p->nj, a->N);
  if (need == 0 || workspace_bytes < need) return PRISM_EINVAL;
  SolveKernelArgs K{};
  st = fill_joint_params(p, a->q0, a->v0, K.jp);
  if (st != PRISM_OK) return st;
  st = check_device(p);
  if (st != PRISM_OK) return st;
  SolveKernelFn fn = pick_plan_kernel(p->HQ, o->precision);
  if (!fn) return PRISM_EUNSUPPORTED;

  // carve the workspace
  char* w = static_cast<char*>(workspace);
  float* cost_col = reinterpret_cast<float*>(w);
  w += align256((size_t)a->N * p->nj * sizeof(float));
  double* cost = a->cost ? a->cost : reinterpret_cast<double*>(w);
  w += align256((size_t)a->N * sizeof(double));
  double* omega = a->omega ? a->omega : reinterpret_cast<double*>(w);
  w += align256((size_t)a->N * sizeof(double));
  int* best = a->best ? a->best : reinterpret_cast<int*>(w);
  w += align256(sizeof(int));
  double* part = reinterpret_cast<double*>(w);

  K.xin = nullptr;   // samples are drawn in the load
  K.xout = a->x_out;
  K.rp = a->r_primal;
  K.rd = a->r_dual;
  K.itout = a->iters_out;
  K.N = a->N;
  K.iters = a->iters;
  K.gen_on = 1;
  K.gen.nu = a->nu;
  K.gen.sigma = a->sigma;
  K.gen.xs_out = a->samples_out;
  K.gen.seed_lo = (unsigned)(a->seed & 0xffffffffu);
  K.gen.seed_hi = (unsigned)(a->seed >> 32);
  K.gen.stream_lo = (unsigned)(a->stream & 0xffffffffu);
  K.gen.stream_hi = (unsigned)(a->stream >> 32);
  K.cost_on = 1;
  K.cost.ref = a->theta_ref;
  K.cost.cost = cost_col;
  K.cost.w_pos = a->w_pos;
  K.cost.w_vel = a->w_vel;
  K.cost.dt = (float)p->dt;
  st = launch_solve(p, K, o, fn, stream, counters);
  if (st != PRISM_OK) return st;

  hipLaunchKernelGGL(plan_weights_kernel, dim3(1), dim3(kWeightThreads), 0, stream, cost_col, a->N,
                     p->nj, (double)a->tau, cost, omega, best);
  if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  const int E = p->H * p->nj;
  const int G = moment_blocks(a->N);
  const int per = (a->N + G - 1) / G;
  hipLaunchKernelGGL(plan_moments_partial_kernel, dim3(G), dim3(kMomentThreads), 0, stream,
                     a->x_out, omega, a->N, E, per, part);
  if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  hipLaunchKernelGGL(plan_moments_final_kernel, dim3((E + kMomentThreads - 1) / kMomentThreads),
                     dim3(kMomentThreads), 0, stream, part, G, E, (double)a->eps, a->nu_out,
                     a->var_out);
  if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  return PRISM_OK;
}

}  // namespace

extern "C" {

size_t prism_plan_workspace_bytes(int H, int n_joints, int N) {
  if (H < 2 || H > PRISM_MAX_H || n_joints < 1 || n_joints > PRISM_MAX_JOINTS || N < 1) return 0;
  const size_t E = (size_t)H * n_joints;
  return align256((size_t)N * n_joints * sizeof(float)) + 2 * align256((size_t)N * sizeof(double)) +
         align256(sizeof(int)) + align256((size_t)moment_blocks(N) * E * 2 * sizeof(double));
}

prism_status_t prism_plan_step(prism_proj_t p, const prism_plan_args_t* a, hipStream_t stream) {
  if (!p || !a) return PRISM_EINVAL;
  if (!a->workspace) return PRISM_EINVAL;
  return plan_step_impl(p, a, stream, a->workspace, a->workspace_bytes, nullptr);
}

prism_status_t prism_plan_step_static(prism_proj_t p, const prism_plan_args_t* a,
                                      hipStream_t stream) {
  if (!p || !a) return PRISM_EINVAL;
  if (a->N >= 1) {
    const size_t need = prism_plan_workspace_bytes(p->H, p->nj, a->N);
    if (need > kStaticWorkspaceBytes) return PRISM_ETOOLARGE;
  }
  prism_status_t st = check_device(p);
  if (st != PRISM_OK) return st;
  char* base = nullptr;
  st = static_scratch(p->device, &base);
  if (st != PRISM_OK) return st;
  // the tile-queue counters first, then the workspace carve of prism_plan_step
  return plan_step_impl(p, a, stream, base + kStaticCounterBytes, kStaticWorkspaceBytes,
                        reinterpret_cast<int*>(base));
}

}  // extern "C"

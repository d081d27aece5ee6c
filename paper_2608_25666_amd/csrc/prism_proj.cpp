// C ABI of the projection library: argument checks, the reusable factor, and
// launches of the fused ADMM kernel. See include/prism_proj.h.
#include "prism_proj.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "admm_kernels.h"
#include "factor.h"
#include "kernel_args.h"
#include "prism_internal.h"

using namespace prism;

namespace prism {

prism_status_t check_device(const prism_proj_s* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PRISM_EDEVICE;
  return dev == p->device ? PRISM_OK : PRISM_EDEVICE;
}

}  // namespace prism

namespace {

bool is_fin(double v) { return std::isfinite(v); }

struct LaunchInfo {
  int blocks_per_cu = 0;
};

std::mutex g_occ_mu;
std::unordered_map<const void*, std::unordered_map<int, LaunchInfo>> g_occ;
int g_num_cu = 0;

int num_cus() {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  if (g_num_cu == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    g_num_cu = n;
  }
  return g_num_cu;
}

int blocks_per_cu(const void* fn, int lds, int threads = kWaves * 64) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto& m = g_occ[fn];   // a kernel is always launched with the same thread count
  auto it = m.find(lds);
  if (it != m.end()) return it->second.blocks_per_cu;
  if (lds > 64 * 1024) hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds) != hipSuccess || nb <= 0) nb = 1;
  m[lds].blocks_per_cu = nb;
  return nb;
}

__global__ void zero_counter_kernel(int* c) {
  if ((int)threadIdx.x < kXcdQueues) c[threadIdx.x] = 0;
}

}  // namespace

namespace prism {

prism_status_t validate_options(const prism_options_t* o) {
  if (!o) return PRISM_EINVAL;
  if (o->precision < PRISM_PREC_FP32 || o->precision > PRISM_PREC_FP16) return PRISM_EINVAL;
  if (o->fp32_tail < 0) return PRISM_EINVAL;
  if (!(o->alpha > 0.0f && o->alpha < 2.0f)) return PRISM_EINVAL;
  if (!std::isfinite(o->tol)) return PRISM_EINVAL;
  if (o->check_every < 1) return PRISM_EINVAL;
  if (o->tile_waves < 0 || o->tile_waves > 2) return PRISM_EINVAL;
  for (int r : o->reserved)
    if (r != 0) return PRISM_EINVAL;
  return PRISM_OK;
}

int kernel_blocks_per_cu(const void* fn, int lds_bytes) { return blocks_per_cu(fn, lds_bytes); }
int device_cus() { return num_cus(); }

}  // namespace prism

// ---------------------------------------------------------------------------
// Internal helpers shared with the batch and server front ends
// ---------------------------------------------------------------------------
namespace prism {

prism_status_t fill_joint_params(const prism_proj_s* p, const double* q0, const double* v0,
                                 JointRowParams* jp) {
  const int nj = p->nj;
  const double dt = p->dt;
  for (int j = 0; j < nj; ++j) {
    if (!is_fin(q0[j]) || !is_fin(v0[j])) return PRISM_EINVAL;
    const double qmin = p->bnd[0 * nj + j], qmax = p->bnd[1 * nj + j];
    const double vmin = p->bnd[2 * nj + j], vmax = p->bnd[3 * nj + j];
    const double amin = p->bnd[4 * nj + j], amax = p->bnd[5 * nj + j];
    const double jmin = p->bnd[6 * nj + j], jmax = p->bnd[7 * nj + j];
    const double q1 = q0[j] + dt * v0[j];
    // rows fixed by x_1 = v0 (velocity, position and acceleration of step 1) must
    // already hold; jerk rows start at step 2 (eq. (jerk_stack)), so the jerk bounds
    // need not contain 0
    if (v0[j] < vmin || v0[j] > vmax || q1 < qmin || q1 > qmax || amin > 0.0 || amax < 0.0)
      return PRISM_EINFEASIBLE;
    JointRowParams& r = jp[j];
    r.lb[0] = (float)vmin;
    r.ub[0] = (float)vmax;
    r.lb[1] = (float)((qmin - q0[j]) / dt);
    r.ub[1] = (float)((qmax - q0[j]) / dt);
    r.lb[2] = (float)(amin * dt);
    r.ub[2] = (float)(amax * dt);
    r.lb[3] = (float)(jmin * dt * dt);
    r.ub[3] = (float)(jmax * dt * dt);
    r.v0 = (float)v0[j];
    r.q0 = (float)q0[j];
    r.pad[0] = r.pad[1] = 0.0f;
  }
  return PRISM_OK;
}

SolveKernelFn pick_kernel(int HQ, bool exact, int precision) {
  switch (precision) {
    case PRISM_PREC_FP32: return solve_kernel_f32(HQ, exact);
    case PRISM_PREC_BF16: return solve_kernel_bf16(HQ, exact);
    case PRISM_PREC_FP16: return solve_kernel_f16(HQ, exact);
    default: return nullptr;
  }
}

int solve_frag_bytes(const prism_proj_s* p, int precision) {
  return p->f32_bytes + (precision == PRISM_PREC_FP32 ? 0 : p->b16_bytes);
}

int solve_lds_bytes(const prism_proj_s* p, int precision, int waves) {
  return solve_frag_bytes(p, precision) + waves * p->HQ * 64 * (int)sizeof(float);
}

prism_status_t launch_solve(prism_proj_s* p, SolveKernelArgs& K, const prism_options_t* o,
                            SolveKernelFn fn, hipStream_t stream, int* counters, int waves) {
  const int tiles_per_joint = (K.N + kTileCols - 1) / kTileCols;
  const long long ntiles = (long long)tiles_per_joint * p->nj;
  if (ntiles > 0x7fffffff) return PRISM_EINVAL;
  K.frag = (o->precision == PRISM_PREC_FP16) ? p->frag_f16 : p->frag_bf16;
  K.H = p->H;
  K.nj = p->nj;
  K.ntiles = (int)ntiles;
  K.check_every = o->check_every;
  K.tolmode = (o->tol > 0.0f) ? 1 : 0;
  K.tail = (o->precision == PRISM_PREC_FP32) ? 0 : std::min(o->fp32_tail, K.tolmode ? o->fp32_tail : K.iters);
  K.rho = (float)(p->rho * p->w[2]);
  K.cV = (float)(p->w[0] / p->w[2]);
  K.cQ = (float)(p->w[1] / p->w[2]);
  K.cJ = (float)(p->w[3] / p->w[2]);
  K.alpha = o->alpha;
  K.tol = o->tol;
  K.frag_f32_bytes = p->f32_bytes;
  K.frag_16_bytes = p->b16_bytes;
  const int lds = solve_lds_bytes(p, o->precision, waves);
  const int bpc = blocks_per_cu((const void*)fn, lds, waves * 64);
  const long long want = (ntiles + waves - 1) / waves;
  const long long cap = (long long)bpc * num_cus();
  const int grid = (int)std::max(1ll, std::min(want, cap));

  auto enqueue = [&]() -> prism_status_t {
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, stream, K.counter);
    if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
    void* params[] = {&K};
    if (hipLaunchKernel((const void*)fn, dim3(grid), dim3(waves * 64), params, lds, stream) !=
        hipSuccess)
      return PRISM_EDEVICE;
    if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
    return PRISM_OK;
  };
  if (counters) {
    K.counter = counters;
    return enqueue();
  }
  // A counter set of the handle's ring: wait (on this stream) for the last launch that
  // used it, launch, record this launch's completion. Under graph capture the event
  // calls are skipped: a captured graph keeps its set and must not run concurrently
  // with itself.
  hipStreamCaptureStatus cap_st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap_st) != hipSuccess) return PRISM_EDEVICE;
  const bool capturing = cap_st != hipStreamCaptureStatusNone;
  std::lock_guard<std::mutex> lk(p->ring_mu);
  const auto t = p->ring.take();
  K.counter = p->d_counters + (size_t)t.slot * kXcdQueues;
  if (!capturing && t.wait && hipStreamWaitEvent(stream, p->ring_ev[t.slot], 0) != hipSuccess)
    return PRISM_EDEVICE;
  const prism_status_t st = enqueue();
  if (st != PRISM_OK) return st;
  if (!capturing) {
    if (hipEventRecord(p->ring_ev[t.slot], stream) != hipSuccess) return PRISM_EDEVICE;
    p->ring.recorded(t.slot);
  }
  return PRISM_OK;
}

PairKernelFn pick_pair_kernel(const prism_proj_s* p, int precision) {
  if (p->HP == 0 || !p->pair_frag_bf16) return nullptr;
  switch (precision) {
    case PRISM_PREC_FP32: return pair_kernel_f32(p->HP);
    case PRISM_PREC_BF16: return pair_kernel_bf16(p->HP);
    case PRISM_PREC_FP16: return pair_kernel_f16(p->HP);
    default: return nullptr;
  }
}

int pair_lds_bytes(const prism_proj_s* p, int precision) {
  const int frag = p->pair_f32_bytes + (precision == PRISM_PREC_FP32 ? 0 : p->pair_b16_bytes);
  return frag + (kPairWaves / 2) * pair_lds_words(p->HP) * (int)sizeof(float);
}

prism_status_t launch_pair(prism_proj_s* p, SolveKernelArgs& K, const prism_options_t* o,
                           PairKernelFn fn, hipStream_t stream) {
  const int tiles_per_joint = (K.N + kTileCols - 1) / kTileCols;
  const long long ntiles = (long long)tiles_per_joint * p->nj;
  if (ntiles > 0x7fffffff) return PRISM_EINVAL;
  K.frag = (o->precision == PRISM_PREC_FP16) ? p->pair_frag_f16 : p->pair_frag_bf16;
  K.H = p->H;
  K.nj = p->nj;
  K.ntiles = (int)ntiles;
  K.check_every = o->check_every;
  K.tolmode = (o->tol > 0.0f) ? 1 : 0;
  K.tail = (o->precision == PRISM_PREC_FP32) ? 0 : std::min(o->fp32_tail, K.tolmode ? o->fp32_tail : K.iters);
  K.rho = (float)(p->rho * p->w[2]);
  K.cV = (float)(p->w[0] / p->w[2]);
  K.cQ = (float)(p->w[1] / p->w[2]);
  K.cJ = (float)(p->w[3] / p->w[2]);
  K.alpha = o->alpha;
  K.tol = o->tol;
  K.frag_f32_bytes = p->pair_f32_bytes;
  K.frag_16_bytes = p->pair_b16_bytes;
  const int lds = pair_lds_bytes(p, o->precision);
  if (lds > 160 * 1024) return PRISM_EUNSUPPORTED;
  const int threads = kPairWaves * 64;
  int bpc = 0;
  {
    if (lds > 64 * 1024) hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, (const void*)fn, threads, lds) != hipSuccess ||
        bpc <= 0)
      bpc = 1;
  }
  const long long want = (ntiles + kPairWaves / 2 - 1) / (kPairWaves / 2);
  const long long cap = (long long)bpc * num_cus();
  const int grid = (int)std::max(1ll, std::min(want, cap));

  hipStreamCaptureStatus cap_st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap_st) != hipSuccess) return PRISM_EDEVICE;
  const bool capturing = cap_st != hipStreamCaptureStatusNone;
  std::lock_guard<std::mutex> lk(p->ring_mu);
  const auto t = p->ring.take();
  K.counter = p->d_counters + (size_t)t.slot * kXcdQueues;
  if (!capturing && t.wait && hipStreamWaitEvent(stream, p->ring_ev[t.slot], 0) != hipSuccess)
    return PRISM_EDEVICE;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, stream, K.counter);
  if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  void* params[] = {&K};
  if (hipLaunchKernel((const void*)fn, dim3(grid), dim3(threads), params, lds, stream) != hipSuccess)
    return PRISM_EDEVICE;
  if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  if (!capturing) {
    if (hipEventRecord(p->ring_ev[t.slot], stream) != hipSuccess) return PRISM_EDEVICE;
    p->ring.recorded(t.slot);
  }
  return PRISM_OK;
}

}  // namespace prism

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

void prism_options_default(prism_options_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = PRISM_PREC_FP32;
  o->fp32_tail = 0;
  o->alpha = 1.0f;
  o->tol = 0.0f;
  o->check_every = 10;
}

const char* prism_status_str(prism_status_t s) {
  switch (s) {
    case PRISM_OK: return "ok";
    case PRISM_EINVAL: return "invalid argument";
    case PRISM_ENOMEM: return "out of memory";
    case PRISM_EDEVICE: return "device error";
    case PRISM_EINFEASIBLE: return "infeasible boundary condition";
    case PRISM_EBUSY: return "busy (admission refused)";
    case PRISM_EUNSUPPORTED: return "unsupported configuration";
    case PRISM_ETOOLARGE: return "request exceeds a fixed capacity";
  }
  return "unknown status";
}

int prism_abi_version(void) { return PRISM_PROJ_ABI_VERSION; }

namespace {
bool valid_weights(const double* w) {
  if (!w) return true;
  for (int b = 0; b < 4; ++b)
    if (!(w[b] > 0.0) || !is_fin(w[b])) return false;
  return true;
}
}  // namespace

prism_status_t prism_default_block_weights(int H, int n_joints, double dt,
                                           const prism_bounds_t* bounds, double* w) {
  if (!w || !bounds || !bounds->j_min || !bounds->j_max || H < 2 || H > PRISM_MAX_H ||
      n_joints < 1 || n_joints > PRISM_MAX_JOINTS || !(dt > 0.0) || !is_fin(dt))
    return PRISM_EINVAL;
  double jw = 0.0;   // the smallest jerk half-width over the joints
  for (int j = 0; j < n_joints; ++j) {
    const double h = 0.5 * (bounds->j_max[j] - bounds->j_min[j]);
    if (!(h > 0.0) || !is_fin(h)) return PRISM_EINVAL;
    if (j == 0 || h < jw) jw = h;
  }
  // 1.7 * (1, 1.25/H, 8, 10) was tuned (the slowest 16-sample group's iteration count at
  // residual 1e-3 with alpha = 1.8, over eight workload shapes) where the jerk bound in
  // velocity units, jw dt^2, is 60 * 0.02^2; the best uniform scale of the weights falls
  // in proportion as that bound widens
  const double ref = 60.0 * 0.02 * 0.02;
  double s = ref / (jw * dt * dt);
  s = std::min(std::max(s, std::exp2(-4.5)), std::exp2(1.5));
  w[0] = 1.7 * s;
  w[1] = 2.125 / H * s;
  w[2] = 13.6 * s;
  w[3] = 17.0 * s;
  return PRISM_OK;
}

prism_status_t prism_factor_host(int H, double rho, const double* w, double* K, double* k) {
  if (H < 2 || H > PRISM_MAX_H || !(rho > 0.0) || !is_fin(rho) || !K || !k || !valid_weights(w))
    return PRISM_EINVAL;
  std::vector<double> Kv, kv;
  if (!build_factor(H, rho, w, Kv, kv)) return PRISM_EINVAL;
  std::memcpy(K, Kv.data(), sizeof(double) * H * H);
  std::memcpy(k, kv.data(), sizeof(double) * H);
  return PRISM_OK;
}

prism_status_t prism_proj_create(int H, int n_joints, double dt, const prism_bounds_t* bounds,
                                 double rho, prism_proj_t* out) {
  return prism_proj_create_ex(H, n_joints, dt, bounds, rho, nullptr, out);
}

prism_status_t prism_proj_create_ex(int H, int n_joints, double dt, const prism_bounds_t* bounds,
                                    double rho, const double* block_weights, prism_proj_t* out) {
  if (!out || !bounds || !valid_weights(block_weights)) return PRISM_EINVAL;
  if (H < 2 || H > PRISM_MAX_H || n_joints < 1 || n_joints > PRISM_MAX_JOINTS) return PRISM_EINVAL;
  if (!(dt > 0.0) || !is_fin(dt) || !(rho > 0.0) || !is_fin(rho)) return PRISM_EINVAL;
  const double* arr[8] = {bounds->q_min, bounds->q_max, bounds->v_min, bounds->v_max,
                          bounds->a_min, bounds->a_max, bounds->j_min, bounds->j_max};
  for (auto a : arr)
    if (!a) return PRISM_EINVAL;
  for (int j = 0; j < n_joints; ++j)
    for (int b = 0; b < 8; b += 2) {
      const double lo = arr[b][j], hi = arr[b + 1][j];
      if (!is_fin(lo) || !is_fin(hi) || lo > hi) return PRISM_EINVAL;
    }
  prism_proj_s* p = new (std::nothrow) prism_proj_s();
  if (!p) return PRISM_ENOMEM;
  p->H = H;
  p->nj = n_joints;
  p->HQ = std::max(2, chunk_rows(H));
  p->dt = dt;
  p->rho = rho;
  if (block_weights)
    for (int b = 0; b < 4; ++b) p->w[b] = block_weights[b];
  p->bnd.resize(8 * n_joints);
  for (int b = 0; b < 8; ++b)
    for (int j = 0; j < n_joints; ++j) p->bnd[b * n_joints + j] = arr[b][j];
  prism_options_default(&p->opts);
  if (!build_factor(H, rho, p->w, p->K, p->k)) {
    delete p;
    return PRISM_EINVAL;
  }
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return PRISM_EDEVICE;
  }
  std::vector<float> f32, pf32;
  std::vector<uint16_t> bf, hf, pbf, phf;
  if (H >= kPairMinH) {
    p->HP = pair_chunk_rows(H);
    layout_pair_f32(p->K, H, p->HP, pf32);
    layout_pair_16(p->K, H, p->HP, true, pbf);
    layout_pair_16(p->K, H, p->HP, false, phf);
    p->pair_f32_bytes = (int)(pf32.size() * sizeof(float));
    p->pair_b16_bytes = (int)(pbf.size() * sizeof(uint16_t));
  }
  layout_f32(p->K, H, p->HQ, f32);
  layout_16(p->K, H, p->HQ, true, bf);
  layout_16(p->K, H, p->HQ, false, hf);
  p->f32_bytes = (int)(f32.size() * sizeof(float));
  p->b16_bytes = (int)(bf.size() * sizeof(uint16_t));
  const size_t tot = (size_t)p->f32_bytes + p->b16_bytes;
  prism_status_t st = PRISM_OK;
  if (hipMalloc(&p->frag_bf16, tot) != hipSuccess || hipMalloc(&p->frag_f16, tot) != hipSuccess ||
      hipMalloc((void**)&p->d_bounds, sizeof(double) * 8 * n_joints) != hipSuccess ||
      hipMalloc((void**)&p->d_counters, sizeof(int) * kCounterRing * kXcdQueues) != hipSuccess) {
    st = PRISM_ENOMEM;
  }
  if (st == PRISM_OK) {
    char* a = (char*)p->frag_bf16;
    char* b = (char*)p->frag_f16;
    if (hipMemcpy(a, f32.data(), p->f32_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(a + p->f32_bytes, bf.data(), p->b16_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b, f32.data(), p->f32_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b + p->f32_bytes, hf.data(), p->b16_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_bounds, p->bnd.data(), sizeof(double) * 8 * n_joints,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(p->d_counters, 0, sizeof(int) * kCounterRing * kXcdQueues) != hipSuccess)
      st = PRISM_EDEVICE;
  }
  if (st == PRISM_OK && p->HP > 0) {
    const size_t ptot = (size_t)p->pair_f32_bytes + p->pair_b16_bytes;
    if (hipMalloc(&p->pair_frag_bf16, ptot) != hipSuccess ||
        hipMalloc(&p->pair_frag_f16, ptot) != hipSuccess) {
      st = PRISM_ENOMEM;
    } else {
      char* a = (char*)p->pair_frag_bf16;
      char* b = (char*)p->pair_frag_f16;
      if (hipMemcpy(a, pf32.data(), p->pair_f32_bytes, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(a + p->pair_f32_bytes, pbf.data(), p->pair_b16_bytes, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b, pf32.data(), p->pair_f32_bytes, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b + p->pair_f32_bytes, phf.data(), p->pair_b16_bytes, hipMemcpyHostToDevice) != hipSuccess)
        st = PRISM_EDEVICE;
    }
  }
  for (int i = 0; st == PRISM_OK && i < kCounterRing; ++i)
    if (hipEventCreateWithFlags(&p->ring_ev[i], hipEventDisableTiming) != hipSuccess)
      st = PRISM_EDEVICE;
  if (st != PRISM_OK) {
    prism_proj_destroy(p);
    return st;
  }
  *out = p;
  return PRISM_OK;
}

void prism_proj_destroy(prism_proj_t p) {
  if (!p) return;
  if (p->frag_bf16) (void)hipFree(p->frag_bf16);
  if (p->frag_f16) (void)hipFree(p->frag_f16);
  if (p->d_bounds) (void)hipFree(p->d_bounds);
  if (p->d_counters) (void)hipFree(p->d_counters);
  if (p->pair_frag_bf16) (void)hipFree(p->pair_frag_bf16);
  if (p->pair_frag_f16) (void)hipFree(p->pair_frag_f16);
  for (hipEvent_t& e : p->ring_ev)
    if (e) (void)hipEventDestroy(e);
  release_literal_factors(p);
  delete p;
}

int prism_proj_horizon(prism_proj_t p) { return p ? p->H : -1; }
int prism_proj_joints(prism_proj_t p) { return p ? p->nj : -1; }

prism_status_t prism_proj_get_weights(prism_proj_t p, double* w) {
  if (!p || !w) return PRISM_EINVAL;
  for (int b = 0; b < 4; ++b) w[b] = p->w[b];
  return PRISM_OK;
}

prism_status_t prism_proj_get_factor(prism_proj_t p, double* K, double* k) {
  if (!p || !K || !k) return PRISM_EINVAL;
  std::memcpy(K, p->K.data(), sizeof(double) * p->H * p->H);
  std::memcpy(k, p->k.data(), sizeof(double) * p->H);
  return PRISM_OK;
}

prism_status_t prism_proj_set_options(prism_proj_t p, const prism_options_t* opts) {
  if (!p) return PRISM_EINVAL;
  const prism_status_t st = validate_options(opts);
  if (st != PRISM_OK) return st;
  p->opts = *opts;
  return PRISM_OK;
}

prism_status_t prism_proj_get_options(prism_proj_t p, prism_options_t* opts) {
  if (!p || !opts) return PRISM_EINVAL;
  *opts = p->opts;
  return PRISM_OK;
}

prism_status_t prism_proj_solve_ex(prism_proj_t p, const prism_solve_args_t* a, hipStream_t stream) {
  if (!p || !a) return PRISM_EINVAL;
  const prism_options_t* o = a->opts ? a->opts : &p->opts;
  prism_status_t st = validate_options(o);
  if (st != PRISM_OK) return st;
  if (a->N < 0 || a->iters < 0) return PRISM_EINVAL;
  if (!a->q0 || !a->v0) return PRISM_EINVAL;
  if (a->warm_shift != 0 && a->warm_shift != 1) return PRISM_EINVAL;
  if (a->warm_shift && a->state_warm && !a->x_warm) return PRISM_EINVAL;
  SolveKernelArgs K{};
  st = fill_joint_params(p, a->q0, a->v0, K.jp);
  if (st != PRISM_OK) return st;
  if (a->N == 0) return PRISM_OK;
  if (!a->v_samples || !a->v_out) return PRISM_EINVAL;
  if ((long long)a->N * p->H * p->nj > (1ll << 40)) return PRISM_EINVAL;
  st = check_device(p);
  if (st != PRISM_OK) return st;

  const bool exact = (4 * p->HQ == p->H);
  const bool pair_ok = !a->x_warm && !a->state_warm && !a->state_out;
  PairKernelFn pfn = (o->tile_waves == 2 && pair_ok) ? pick_pair_kernel(p, o->precision) : nullptr;
  if (o->tile_waves == 2 && !pfn) return PRISM_EUNSUPPORTED;
  SolveKernelFn fn = pfn ? nullptr : pick_kernel(p->HQ, exact, o->precision);
  if (!fn && !pfn) return PRISM_EUNSUPPORTED;
  K.xin = a->v_samples;
  K.xout = a->v_out;
  K.rp = a->r_primal;
  K.rd = a->r_dual;
  K.itout = a->iters_out;
  K.xw = a->x_warm;
  K.uw = a->state_warm;
  K.uout = a->state_out;
  K.shift = a->warm_shift;
  K.N = a->N;
  K.iters = a->iters;
  if (pfn) return launch_pair(p, K, o, pfn, stream);
  return launch_solve(p, K, o, fn, stream, nullptr, solve_waves(p->HQ, o->precision != PRISM_PREC_FP32));
}

prism_status_t prism_proj_solve(prism_proj_t p, const float* v_samples, int N, const double* q0,
                                const double* v0, int iters, float* v_out, float* r_primal,
                                float* r_dual, hipStream_t stream) {
  prism_solve_args_t a{};
  a.v_samples = v_samples;
  a.N = N;
  a.iters = iters;
  a.q0 = q0;
  a.v0 = v0;
  a.v_out = v_out;
  a.r_primal = r_primal;
  a.r_dual = r_dual;
  return prism_proj_solve_ex(p, &a, stream);
}

prism_status_t prism_proj_feasibility(prism_proj_t p, const float* v, int N, const double* q0,
                                      const double* v0, double* viol, hipStream_t stream) {
  if (!p || N < 0 || !q0 || !v0) return PRISM_EINVAL;
  for (int j = 0; j < p->nj; ++j)
    if (!is_fin(q0[j]) || !is_fin(v0[j])) return PRISM_EINVAL;
  if (N == 0) return PRISM_OK;
  if (!v || !viol) return PRISM_EINVAL;
  prism_status_t st = check_device(p);
  if (st != PRISM_OK) return st;
  FeasKernelArgs A{};
  A.x = v;
  A.viol = viol;
  A.bounds = p->d_bounds;
  A.N = N;
  A.H = p->H;
  A.nj = p->nj;
  A.dt = p->dt;
  for (int j = 0; j < p->nj; ++j) {
    A.q0[j] = q0[j];
    A.v0[j] = v0[j];
  }
  return launch_feasibility(A, stream) == hipSuccess ? PRISM_OK : PRISM_EDEVICE;
}

}  // extern "C"

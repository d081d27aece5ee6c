// Batched solve: many requests with their own factors in one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "admm_batch.h"
#include "kernel_args.h"
#include "prism_internal.h"
#include "prism_proj.h"

using namespace prism;

struct prism_batch_s {
  int device = 0;
  BatchReq* h_reqs = nullptr;        // pinned
  JointRowParams* h_jp = nullptr;    // pinned
  BatchReq* d_reqs = nullptr;
  JointRowParams* d_jp = nullptr;
  int* d_counters = nullptr;         // [cap_req][kXcdQueues] tile-queue counters
  size_t cap_req = 0, cap_jp = 0;
  hipEvent_t copied = nullptr;
  bool pending = false;
  // second launch of a split batch: an internal stream forked from the caller's stream
  // after the tables and counters are ready and joined back after its launch
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

__global__ void zero_ints_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void release_tables(prism_batch_s* b) {
  if (b->h_reqs) (void)hipHostFree(b->h_reqs);
  if (b->h_jp) (void)hipHostFree(b->h_jp);
  if (b->d_reqs) (void)hipFree(b->d_reqs);
  if (b->d_jp) (void)hipFree(b->d_jp);
  if (b->d_counters) (void)hipFree(b->d_counters);
  b->h_reqs = nullptr;
  b->h_jp = nullptr;
  b->d_reqs = nullptr;
  b->d_jp = nullptr;
  b->d_counters = nullptr;
  b->cap_req = b->cap_jp = 0;
}

prism_status_t reserve(prism_batch_s* b, size_t nreq, size_t njp) {
  if (nreq <= b->cap_req && njp <= b->cap_jp) return PRISM_OK;
  release_tables(b);
  const size_t cr = std::max<size_t>(64, nreq * 2), cj = std::max<size_t>(1024, njp * 2);
  if (hipHostMalloc((void**)&b->h_reqs, cr * sizeof(BatchReq), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->h_jp, cj * sizeof(JointRowParams), hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&b->d_reqs, cr * sizeof(BatchReq)) != hipSuccess ||
      hipMalloc((void**)&b->d_jp, cj * sizeof(JointRowParams)) != hipSuccess ||
      hipMalloc((void**)&b->d_counters, cr * kXcdQueues * sizeof(int)) != hipSuccess) {
    release_tables(b);
    return PRISM_ENOMEM;
  }
  b->cap_req = cr;
  b->cap_jp = cj;
  return PRISM_OK;
}

BatchKernelFn pick_batch_kernel(int set, int precision) {
  switch (precision) {
    case PRISM_PREC_FP32: return batch_kernel_f32(set);
    case PRISM_PREC_BF16: return batch_kernel_bf16(set);
    case PRISM_PREC_FP16: return batch_kernel_f16(set);
    default: return nullptr;
  }
}

}  // namespace

namespace prism {

prism_status_t enqueue_batch(prism_batch_s* b, const BatchDesc* reqs, int n_req,
                             const prism_options_t& opts, hipStream_t stream, int grid_pct) {
  prism_status_t st = validate_options(&opts);
  if (st != PRISM_OK) return st;
  if (opts.tile_waves == 2) return PRISM_EUNSUPPORTED;   // batched launches use one-wave tiles
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device) return PRISM_EDEVICE;

  // ---- validate every request before touching anything
  size_t n_jp = 0;
  std::vector<int> live;
  for (int r = 0; r < n_req; ++r) {
    const BatchDesc& q = reqs[r];
    const prism_proj_s* p = q.p;
    if (!p || q.N < 0 || q.iters < 0 || !q.q0 || !q.v0) return PRISM_EINVAL;
    if (q.shift != 0 && q.shift != 1) return PRISM_EINVAL;
    if (q.shift && q.uw && !q.xw) return PRISM_EINVAL;
    if (p->device != b->device) return PRISM_EDEVICE;
    JointRowParams tmp[kMaxJoints];
    st = fill_joint_params(p, q.q0, q.v0, tmp);
    if (st != PRISM_OK) return st;
    if (q.N == 0) continue;
    if (!q.xin || !q.xout) return PRISM_EINVAL;
    if ((long long)q.N * p->H * p->nj > (1ll << 40)) return PRISM_EINVAL;
    live.push_back(r);
    n_jp += p->nj;
  }
  if (live.empty()) return PRISM_OK;

  // longest work first: chunk^2 * tiles * iterations
  auto cost = [&](int r) {
    const prism_proj_s* p = reqs[r].p;
    const double tiles = (double)((reqs[r].N + kTileCols - 1) / kTileCols) * p->nj;
    return (double)p->HQ * p->HQ * tiles * std::max(1, reqs[r].iters);
  };
  std::stable_sort(live.begin(), live.end(), [&](int a, int c) { return cost(a) > cost(c); });

  // ---- which launches: sets 6 and 0 for chunks {5, 13, 25} only, else one per chunk class
  bool all_mpc = true;
  for (int r : live)
    if (!batch_set_has(0, reqs[r].p->HQ) && !batch_set_has(6, reqs[r].p->HQ)) all_mpc = false;
  std::vector<int> sets;
  if (all_mpc) {
    // horizons 97-100 (one wave per SIMD), then 17-20 and 49-52 (two waves per SIMD)
    for (int s : {6, 0})
      for (int r : live)
        if (batch_set_has(s, reqs[r].p->HQ)) {
          sets.push_back(s);
          break;
        }
  } else {
    for (int s : kBatchClasses)
      for (int r : live)
        if (batch_set_has(s, reqs[r].p->HQ)) {
          sets.push_back(s);
          break;
        }
  }

  if (b->pending) {
    if (hipEventSynchronize(b->copied) != hipSuccess) return PRISM_EDEVICE;
    b->pending = false;
  }
  st = reserve(b, live.size(), n_jp);
  if (st != PRISM_OK) return st;

  // ---- build the tables, grouped by launch
  struct Launch {
    int set, first, count, hq_max, frag_max;
    long long tiles;
    double work;
  };
  std::vector<Launch> launches;
  std::vector<int> live_of;   // request index of each table row
  size_t ri = 0, ji = 0;
  const bool tolmode = opts.tol > 0.0f;
  for (int s : sets) {
    Launch L{s, (int)ri, 0, 2, 0, 0, 0.0};
    for (int r : live) {
      const BatchDesc& q = reqs[r];
      const prism_proj_s* p = q.p;
      if (!batch_set_has(s, p->HQ)) continue;
      live_of.push_back(r);
      BatchReq& B = b->h_reqs[ri++];
      std::memset(&B, 0, sizeof(B));
      fill_joint_params(p, q.q0, q.v0, b->h_jp + ji);
      TileArgs& T = B.t;
      T.xin = q.xin;
      T.xout = q.xout;
      T.xsave = q.xsave;
      T.rp = q.rp;
      T.rd = q.rd;
      T.itout = q.itout;
      T.xw = q.xw;
      T.uw = q.uw;
      T.uout = q.uout;
      T.jp = b->d_jp + ji;
      T.N = q.N;
      T.H = p->H;
      T.nj = p->nj;
      T.iters = q.iters;
      T.check_every = opts.check_every;
      T.tolmode = tolmode ? 1 : 0;
      T.shift = q.shift;
      T.tail = (opts.precision == PRISM_PREC_FP32) ? 0
                                                   : std::min(opts.fp32_tail, tolmode ? opts.fp32_tail : q.iters);
      T.rho = (float)(p->rho * p->w[2]);
      T.alpha = opts.alpha;
      T.tol = opts.tol;
      T.cV = (float)(p->w[0] / p->w[2]);
      T.cQ = (float)(p->w[1] / p->w[2]);
      T.cJ = (float)(p->w[3] / p->w[2]);
      B.frag = (opts.precision == PRISM_PREC_FP16) ? p->frag_f16 : p->frag_bf16;
      B.HQ = p->HQ;
      B.frag_f32_bytes = p->f32_bytes;
      B.frag_16_bytes = p->b16_bytes;
      B.nblk = (q.N + kTileCols - 1) / kTileCols;
      B.wg_begin = 0;   // set below, once the launch's grid is known
      L.tiles += (long long)B.nblk * p->nj;
      L.work += cost(r);
      L.count++;
      L.hq_max = std::max(L.hq_max, p->HQ);
      L.frag_max = std::max(L.frag_max, solve_frag_bytes(p, opts.precision));
      ji += p->nj;
    }
    if (L.count > 0) launches.push_back(L);
  }

  // ---- per launch: kernel, grid, and each request's first home workgroup (workgroups
  // spread over the requests in proportion to their work, in launch order)
  struct Plan {
    BatchKernelFn fn;
    int grid, lds;
  };
  std::vector<Plan> plans;
  for (const Launch& L : launches) {
    Plan P{pick_batch_kernel(L.set, opts.precision), 1, 0};
    if (!P.fn) return PRISM_EUNSUPPORTED;
    P.lds = L.frag_max + kWaves * L.hq_max * 64 * (int)sizeof(float);
    const int bpc = kernel_blocks_per_cu((const void*)P.fn, P.lds);
    const long long slots = std::max(1ll, (long long)bpc * device_cus() * grid_pct / 100);
    P.grid = (int)std::max(1ll, std::min((L.tiles + kWaves - 1) / kWaves, slots));
    double before = 0.0;
    for (int k = 0; k < L.count; ++k) {
      BatchReq& B = b->h_reqs[L.first + k];
      B.wg_begin = (int)std::floor(before / L.work * P.grid);
      before += cost(live_of[(size_t)(L.first + k)]);
    }
    plans.push_back(P);
  }

  // ---- upload tables, clear counters, launch
  if (hipMemcpyAsync(b->d_jp, b->h_jp, ji * sizeof(JointRowParams), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipMemcpyAsync(b->d_reqs, b->h_reqs, ri * sizeof(BatchReq), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipEventRecord(b->copied, stream) != hipSuccess)
    return PRISM_EDEVICE;
  b->pending = true;
  const int n_ctr = (int)ri * kXcdQueues;
  hipLaunchKernelGGL(zero_ints_kernel, dim3((n_ctr + 255) / 256), dim3(256), 0, stream, b->d_counters,
                     n_ctr);
  if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  // The {5, 13, 25} split's two launches are independent (disjoint requests, counters
  // and outputs): the second runs on the internal stream, so its workgroups take the
  // CUs that the first launch's workgroups free while its last tiles finish. Other
  // mixes, and launches given a share of the GPU (the server's, which already overlap
  // on up to four streams of their own), run in order on the caller's stream.
  const bool fork = all_mpc && launches.size() == 2 && grid_pct >= 100;
  if (fork) {
    if (!b->side && (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
                     hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                     hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess))
      return PRISM_EDEVICE;
    if (hipEventRecord(b->fork, stream) != hipSuccess || hipStreamWaitEvent(b->side, b->fork, 0) != hipSuccess)
      return PRISM_EDEVICE;
  }
  for (size_t li = 0; li < launches.size(); ++li) {
    const Launch& L = launches[li];
    const Plan& P = plans[li];
    BatchKernelArgs A{};
    A.reqs = b->d_reqs + L.first;
    A.n_req = L.count;
    A.counter = b->d_counters + (size_t)L.first * kXcdQueues;
    A.xt_offset = L.frag_max;
    A.hq_max = L.hq_max;
    void* params[] = {&A};
    hipStream_t s = (fork && li == 1) ? b->side : stream;
    if (hipLaunchKernel((const void*)P.fn, dim3(P.grid), dim3(kWaves * 64), params, P.lds, s) != hipSuccess)
      return PRISM_EDEVICE;
    if (hipGetLastError() != hipSuccess) return PRISM_EDEVICE;
  }
  if (fork && (hipEventRecord(b->join, b->side) != hipSuccess ||
               hipStreamWaitEvent(stream, b->join, 0) != hipSuccess))
    return PRISM_EDEVICE;
  return PRISM_OK;
}

}  // namespace prism

extern "C" {

prism_status_t prism_batch_create(prism_batch_t* out) {
  if (!out) return PRISM_EINVAL;
  prism_batch_s* b = new (std::nothrow) prism_batch_s();
  if (!b) return PRISM_ENOMEM;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return PRISM_EDEVICE;
  }
  if (hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess) {
    prism_batch_destroy(b);
    return PRISM_ENOMEM;
  }
  *out = b;
  return PRISM_OK;
}

void prism_batch_destroy(prism_batch_t b) {
  if (!b) return;
  if (b->pending && b->copied) (void)hipEventSynchronize(b->copied);
  release_tables(b);
  if (b->copied) (void)hipEventDestroy(b->copied);
  if (b->side) {
    (void)hipStreamSynchronize(b->side);
    (void)hipStreamDestroy(b->side);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  delete b;
}

prism_status_t prism_proj_solve_batch(prism_batch_t b, int n_req, const prism_request_t* reqs,
                                      const prism_options_t* opts_in, hipStream_t stream) {
  if (!b || n_req < 0 || (n_req > 0 && !reqs)) return PRISM_EINVAL;
  prism_options_t opts;
  if (opts_in) opts = *opts_in;
  else prism_options_default(&opts);
  std::vector<BatchDesc> d((size_t)n_req);
  for (int r = 0; r < n_req; ++r) {
    const prism_request_t& q = reqs[r];
    BatchDesc& D = d[(size_t)r];
    D.p = q.proj;
    D.xin = q.v_samples;
    D.xout = q.v_out;
    D.xsave = nullptr;
    D.rp = q.r_primal;
    D.rd = q.r_dual;
    D.itout = q.iters_out;
    D.xw = q.x_warm;
    D.uw = q.state_warm;
    D.uout = q.state_out;
    D.N = q.N;
    D.iters = q.iters;
    D.shift = q.warm_shift;
    D.q0 = q.q0;
    D.v0 = q.v0;
  }
  return prism::enqueue_batch(b, d.data(), n_req, opts, stream);
}

}  // extern "C"

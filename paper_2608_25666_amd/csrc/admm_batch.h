// Persistent kernel for a batch of requests with different horizons, sample
// counts, joint counts, steps and factors, in one launch. A workgroup stages one
// request's factor in LDS and its waves claim that request's tiles one at a time,
// each on its own, from the request's per-XCD tile queues (their own XCD's queue
// first, so the tiles of one sample block, which share cache lines, meet in one
// L2). The workgroup waits for all its waves only when the request has no tiles
// left, and then moves to the first request in launch order (longest work first)
// that still has some. Each workgroup starts at a home request, the host spreading
// workgroups over the requests in proportion to their work. The chunk size is a
// runtime property of the request, dispatched over the compile-time list HQs.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "admm_tile.h"
#include "kernel_args.h"

namespace prism {

template <int GEMM, int HQ>
__device__ __forceinline__ void batch_tile(const TileArgs& T, int j, int s0, const float* kf32,
                                           const void* k16, float* xt) {
  TileSolver<HQ, false, GEMM> ts;
  ts.run(T, j, s0, kf32, k16, xt);
}

template <int GEMM, int... HQs>
__device__ __forceinline__ void batch_dispatch(int hq, const TileArgs& T, int j, int s0,
                                               const float* kf32, const void* k16, float* xt) {
  ((hq == HQs ? (batch_tile<GEMM, HQs>(T, j, s0, kf32, k16, xt), 0) : 0), ...);
}

// Tiles dealt to queue x of a request: its sample blocks x, x + 8, ... times its joints.
__device__ __forceinline__ int batch_queue_tiles(int nblk, int nj, int x) {
  return (nblk > x ? (nblk - x + kXcdQueues - 1) / kXcdQueues : 0) * nj;
}

template <int GEMM, int... HQs>
__device__ __forceinline__ void batch_body(const BatchKernelArgs& B) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ int s_next;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  float* xt_wave = reinterpret_cast<float*>(lds + B.xt_offset) + wave * (B.hq_max * 64);
  if (B.n_req <= 0) return;
  const int xq = blockIdx.x & (kXcdQueues - 1);   // workgroups are dealt to XCDs round-robin
  int r = 0;                                      // home: last request with wg_begin <= blockIdx
  {
    int lo = 0, hi = B.n_req - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.reqs[mid].wg_begin <= (int)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    r = lo;
  }
  const void* staged = nullptr;
  for (;;) {
    const BatchReq& R = B.reqs[r];                // r is uniform: request data in SGPRs
    if (R.frag != staged) {
      const int nbytes = R.frag_f32_bytes + (GEMM == GEMM_F32 ? 0 : R.frag_16_bytes);
      const v4u* src = reinterpret_cast<const v4u*>(R.frag);
      v4u* dst = reinterpret_cast<v4u*>(lds);
      // index from the wave and lane ids (kWaves * 64 threads): the work-item id
      // register need not stay live (at 256 registers the FP16 {5, 13} kernel spilled it)
      for (int i = wave * 64 + (int)__lane_id(); i < nbytes / 16; i += kWaves * 64) dst[i] = src[i];
      __syncthreads();
      staged = R.frag;
    }
    {
      int* ctr = B.counter + (size_t)r * kXcdQueues;
      const int nj = R.t.nj, nblk = R.nblk;
      int x = xq;
      for (int probed = 0; probed < kXcdQueues;) {
        const int in_queue = batch_queue_tiles(nblk, nj, x);
        int i = 0;
        if (lane == 0) i = atomicAdd(ctr + x, 1);
        i = __builtin_amdgcn_readfirstlane(i);
        if (i >= in_queue) {
          ++probed;
          x = (x + 1) & (kXcdQueues - 1);
          continue;
        }
        const int j = i % nj;
        const int sb = x + kXcdQueues * (i / nj);
        batch_dispatch<GEMM, HQs...>(R.HQ, R.t, j, sb * kTileCols, reinterpret_cast<const float*>(lds),
                                     lds + R.frag_f32_bytes, xt_wave);
      }
    }
    // Every wave has found request r drained and is done with its factor. Next: the
    // first request in launch order with a tile left in some queue. The counters are
    // read while other workgroups claim tiles; a stale read only sends this workgroup
    // to a request whose queues then turn out drained, and it looks again.
    if (threadIdx.x == 0) s_next = INT_MAX;
    __syncthreads();
    constexpr int kPerPass = kWaves * 64 / kXcdQueues;   // requests looked at per pass
    int found = INT_MAX;
    for (int base = 0; base < B.n_req; base += kPerPass) {
      const int rr = base + (int)threadIdx.x / kXcdQueues;
      const int x = threadIdx.x & (kXcdQueues - 1);
      if (rr < B.n_req) {
        const BatchReq& Q = B.reqs[rr];
        const int taken = __hip_atomic_load(B.counter + (size_t)rr * kXcdQueues + x, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        if (taken < batch_queue_tiles(Q.nblk, Q.t.nj, x)) atomicMin(&s_next, rr);
      }
      __syncthreads();
      found = __builtin_amdgcn_readfirstlane(s_next);
      __syncthreads();   // all have read s_next before the next pass may lower it
      if (found != INT_MAX) break;
    }
    if (found == INT_MAX) break;
    r = found;
  }
}

template <int GEMM, int... HQs>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void
admm_batch_kernel_2w(BatchKernelArgs B) {
  batch_body<GEMM, HQs...>(B);
}

template <int GEMM, int... HQs>
__global__ __launch_bounds__(256) void admm_batch_kernel(BatchKernelArgs B) {
  batch_body<GEMM, HQs...>(B);
}

using BatchKernelFn = void (*)(BatchKernelArgs);

// Kernels by chunk-size set: 0 = {5, 13} (horizons 17-20, 49-52; two waves per SIMD),
// 6 = {25} (horizons 97-100; one wave), 1 = chunks 2..8, 2 = 9..12 (two waves),
// 3 = 13..16, 4 = 17..24, 5 = 25..28, 7 = 29..30, 8 = 31, 9 = 32 (one wave; the last
// four split so that no class needs scratch). A batch whose chunks all fall in {5, 13, 25}
// runs sets 6 and 0; any other mix runs the classes it uses, in the order of kBatchClasses.
constexpr int kBatchClasses[] = {1, 2, 3, 4, 5, 7, 8, 9};
BatchKernelFn batch_kernel_f32(int set);
BatchKernelFn batch_kernel_bf16(int set);
BatchKernelFn batch_kernel_f16(int set);

inline bool batch_set_has(int set, int hq) {
  switch (set) {
    case 0: return hq == 5 || hq == 13;
    case 1: return hq >= 2 && hq <= 8;
    case 2: return hq >= 9 && hq <= 12;
    case 3: return hq >= 13 && hq <= 16;
    case 4: return hq >= 17 && hq <= 24;
    case 5: return hq >= 25 && hq <= 28;
    case 6: return hq == 25;
    case 7: return hq == 29 || hq == 30;
    case 8: return hq == 31;
    case 9: return hq == 32;
    default: return false;
  }
}

}  // namespace prism

// Persistent kernel for a batch of requests with different horizons, sample
// counts, joint counts, steps and factors, in one launch. Each request's tiles
// are grouped in work items of four tiles (one per wave) that share its factor;
// a workgroup pulls items from an atomic counter (the host orders items
// longest-first) and restages the factor in LDS only when it changes. The
// chunk size is a runtime property of the request, dispatched over the
// compile-time list HQs.
#pragma once

#include <hip/hip_runtime.h>

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

template <int GEMM, int... HQs>
__device__ __forceinline__ void batch_body(const BatchKernelArgs& B) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ int s_item;
  const int wave = threadIdx.x >> 6;
  float* xt_wave = reinterpret_cast<float*>(lds + B.xt_offset) + wave * (B.hq_max * 64);
  const void* staged = nullptr;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(B.counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);   // uniform: request data in SGPRs
    if (item >= B.n_items) break;
    int lo = 0, hi = B.n_req - 1;              // last request with item_begin <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.reqs[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    const BatchReq R = B.reqs[lo];
    if (R.frag != staged) {
      const int nbytes = R.frag_f32_bytes + (GEMM == GEMM_F32 ? 0 : R.frag_16_bytes);
      const v4u* src = reinterpret_cast<const v4u*>(R.frag);
      v4u* dst = reinterpret_cast<v4u*>(lds);
      for (int i = threadIdx.x; i < nbytes / 16; i += blockDim.x) dst[i] = src[i];
      __syncthreads();
      staged = R.frag;
    }
    const int tile = (item - R.item_begin) * kWaves + wave;
    if (tile < R.tiles) {
      const int j = tile % R.t.nj;
      const int s0 = (tile / R.t.nj) * kTileCols;
      batch_dispatch<GEMM, HQs...>(R.HQ, R.t, j, s0, reinterpret_cast<const float*>(lds),
                                   lds + R.frag_f32_bytes, xt_wave);
    }
    __syncthreads();   // every wave is done with this factor before the next item
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

// Kernels by chunk-size set: 0 = {5, 13, 25} (horizons 17-20, 49-52, 97-100),
// 1 = chunks 2..8, 2 = 9..12, 3 = 13..16, 4 = 17..24, 5 = 25..32.
BatchKernelFn batch_kernel_f32(int set);
BatchKernelFn batch_kernel_bf16(int set);
BatchKernelFn batch_kernel_f16(int set);

inline bool batch_set_has(int set, int hq) {
  switch (set) {
    case 0: return hq == 5 || hq == 13 || hq == 25;
    case 1: return hq >= 2 && hq <= 8;
    case 2: return hq >= 9 && hq <= 12;
    case 3: return hq >= 13 && hq <= 16;
    case 4: return hq >= 17 && hq <= 24;
    case 5: return hq >= 25 && hq <= 32;
    default: return false;
  }
}

}  // namespace prism

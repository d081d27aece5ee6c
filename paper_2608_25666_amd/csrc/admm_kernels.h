// Persistent ADMM kernels: a workgroup of four waves stages the permuted
// inverse K in LDS once, then each wave pulls tiles (16 samples of one joint)
// until none are left. HBM is touched only to load the samples and store the
// projected trajectories and residuals.
//
// Tiles are queued per XCD: queue x holds the sample blocks b = x, x + 8, ...
// (all joints of a block in a row), and workgroup w serves queue w mod 8, the
// XCD it is dispatched to. The joints of one sample share cache lines in the
// [N][H][joints] layout, so a block is then read and written through a single
// L2. A wave whose queue is empty takes tiles from the next queues.
#pragma once

#include <hip/hip_runtime.h>

#include "admm_tile.h"
#include "kernel_args.h"

namespace prism {

// Chunk sizes up to this one fit in 256 registers per lane, so two waves share
// each SIMD and each covers the other's dependency waits (the SIMD does not run
// one wave's VALU work beside the other's MFMA work).
constexpr int kMaxHQTwoWaves = 16;

template <int HQ, bool EXACT, int GEMM, bool PLAN = false>
__device__ __forceinline__ void solve_body(const SolveKernelArgs& A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  {
    // stage FP32 fragments, then the 16-bit fragments of the reduced forms
    const int nbytes = A.frag_f32_bytes + (GEMM == GEMM_F32 ? 0 : A.frag_16_bytes);
    const v4u* src = reinterpret_cast<const v4u*>(A.frag);
    v4u* dst = reinterpret_cast<v4u*>(lds);
    for (int i = threadIdx.x; i < nbytes / 16; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const float* kf32 = reinterpret_cast<const float*>(lds);
  const void* k16 = lds + A.frag_f32_bytes;
  const int frag_bytes = A.frag_f32_bytes + (GEMM == GEMM_F32 ? 0 : A.frag_16_bytes);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float* xt_wave = reinterpret_cast<float*>(lds + frag_bytes) + wave * (HQ * 64);
  TileArgs T;
  T.xin = A.xin;
  T.xout = A.xout;
  T.rp = A.rp;
  T.rd = A.rd;
  T.itout = A.itout;
  T.xw = A.xw;
  T.uw = A.uw;
  T.uout = A.uout;
  T.jp = A.jp;
  T.xsave = nullptr;
  T.shift = A.shift;
  T.gen_on = A.gen_on;
  T.cost_on = A.cost_on;
  T.gen = A.gen;
  T.cost = A.cost;
  T.N = A.N;
  T.H = A.H;
  T.nj = A.nj;
  T.iters = A.iters;
  T.check_every = A.check_every;
  T.tail = A.tail;
  T.tolmode = A.tolmode;
  T.rho = A.rho;
  T.alpha = A.alpha;
  T.tol = A.tol;
  T.cV = A.cV;
  T.cQ = A.cQ;
  T.cJ = A.cJ;
  const int nblk = (A.N + kTileCols - 1) / kTileCols;
  int x = blockIdx.x & (kXcdQueues - 1);
  for (int probed = 0; probed < kXcdQueues;) {
    const int in_queue = (nblk > x ? (nblk - x + kXcdQueues - 1) / kXcdQueues : 0) * A.nj;
    int i = 0;
    if (lane == 0) i = atomicAdd(A.counter + x, 1);
    i = __builtin_amdgcn_readfirstlane(i);
    if (i >= in_queue) {
      ++probed;
      x = (x + 1) & (kXcdQueues - 1);
      continue;
    }
    const int j = i % A.nj;
    const int sb = x + kXcdQueues * (i / A.nj);
    TileSolver<HQ, EXACT, GEMM, PLAN> ts;
    ts.run(T, j, sb * kTileCols, kf32, k16, xt_wave);
  }
}

template <int HQ, bool EXACT, int GEMM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void
admm_solve_kernel_2w(SolveKernelArgs A) {
  solve_body<HQ, EXACT, GEMM>(A);
}

template <int HQ, bool EXACT, int GEMM>
__global__ __launch_bounds__(256) void admm_solve_kernel(SolveKernelArgs A) {
  solve_body<HQ, EXACT, GEMM>(A);
}

// Eight waves per workgroup (solve_waves): two per SIMD, one staged factor for all.
template <int HQ, bool EXACT, int GEMM>
__global__ __launch_bounds__(512) void admm_solve_kernel_8w(SolveKernelArgs A) {
  solve_body<HQ, EXACT, GEMM>(A);
}

using SolveKernelFn = void (*)(SolveKernelArgs);

template <int HQ, bool EXACT, int GEMM>
SolveKernelFn kernel_for() {
  if constexpr (HQ <= kMaxHQTwoWaves) return admm_solve_kernel_2w<HQ, EXACT, GEMM>;
  else if constexpr (solve_waves(HQ, GEMM != GEMM_F32) == 8) return admm_solve_kernel_8w<HQ, EXACT, GEMM>;
  else return admm_solve_kernel<HQ, EXACT, GEMM>;
}

// Optimizer-step variant: samples drawn in the load, tracking cost in the
// epilogue (used by prism_plan_step). The sampling and cost code need registers of
// their own: two waves per SIMD fit without spills up to chunk 13 with the FP32
// x-update and chunk 12 with the 16-bit ones.
constexpr int max_hq_two_waves_plan(int gemm) { return gemm == GEMM_F32 ? 13 : 12; }
template <int HQ, int GEMM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void
admm_plan_kernel_2w(SolveKernelArgs A) {
  solve_body<HQ, false, GEMM, true>(A);
}

template <int HQ, int GEMM>
__global__ __launch_bounds__(256) void admm_plan_kernel(SolveKernelArgs A) {
  solve_body<HQ, false, GEMM, true>(A);
}

template <int HQ, int GEMM>
SolveKernelFn plan_kernel_for() {
  if constexpr (HQ <= max_hq_two_waves_plan(GEMM)) return admm_plan_kernel_2w<HQ, GEMM>;
  else return admm_plan_kernel<HQ, GEMM>;
}

SolveKernelFn plan_kernel_f32(int HQ);
SolveKernelFn plan_kernel_bf16(int HQ);
SolveKernelFn plan_kernel_f16(int HQ);

// Two-wave tile kernels (admm_pair.h) by chunk size HP = ceil(H/8); null if not built.
// The launch takes kPairWaves waves per workgroup and pair_lds_words(HP) 32-bit words of
// LDS per pair after the factor fragments.
constexpr int kPairWaves = 8;
constexpr int pair_lds_words(int HP) { return 244 + 4 * HP * 64; }
using PairKernelFn = void (*)(SolveKernelArgs);
PairKernelFn pair_kernel_f32(int HP);
PairKernelFn pair_kernel_bf16(int HP);
PairKernelFn pair_kernel_f16(int HP);

// Kernel for chunk size HQ (2..32), exact fit (4*HQ == H) and GEMM precision.
SolveKernelFn solve_kernel_f32(int HQ, bool exact);
SolveKernelFn solve_kernel_bf16(int HQ, bool exact);
SolveKernelFn solve_kernel_f16(int HQ, bool exact);

}  // namespace prism

// Fused ADMM tile solver for gfx950 (CDNA4), device code.
//
// One wavefront projects a tile of 16 columns: samples s0..s0+15 of one joint
// (Sec. III-D "Joint-wise separability": every (sample, joint) column is an
// independent H-step QP with the same matrices). Lane l = 16*g + c owns column
// c and the HQ consecutive steps g*HQ .. g*HQ+HQ-1 ("chunk g"). This is the
// accumulator layout of v_mfma_f32_16x16x4_f32 once the shared inverse K has
// its rows and columns permuted on the host, so the x-update x += K d
// (Sec. III-D "Step 2: Primal update", in incremental form) runs on MFMA with
// both operands coming straight from registers, while the row stencils run on
// the VALU with only a handful of cross-lane reads per iteration.
//
// ADMM state per column, all FP32 in registers:
//   x  (H)       primal iterate (MFMA accumulator),
//   x~ (H)       the sample (kept in LDS, read once per iteration),
//   q  (4 x H)   q = (1 - alpha) z + u per constraint row (u = y / rho),
//   sw (H)       C^T w, then the defect d = (x~ - x) + rho C^T w.
// Constraint rows per step k (velocity units, see JointRowParams):
//   V: x_k   Q: sum_{i<=k} x_i   A: x_k - x_{k-1}   J: A_k - A_{k-1}.
// One iteration (rows updated with the current s = C x):
//   t = alpha s + q,  z = clip(t, lb, ub),  q' = t - alpha z,
//   w = 2 z - t - s  (= z - s - u'),  d = (x~ - x) + C^T R w,  x += K d,
// with R = rho diag(w_V, w_Q, w_A, w_J) the block penalty (one weight per
// block; the weights enter the transposed sums as FMA coefficients).
// This is the scaled ADMM of the paper's splitting (slack clip = Step 1,
// primal solve = Step 2, multiplier update = Step 3, multiplier carried in the
// constraint space), written with one state per row and an incremental
// primal step so that reduced-precision GEMM operands only round the defect.
//
// Residuals (check iterations): e = z - s per row,
//   r_p = max |e|,  r_d = max_{step >= 2} |rho C^T e - d|,
// which equals |x - x~ + rho C^T u| (the stationarity gap) in exact arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include <type_traits>

#include "kernel_args.h"

namespace prism {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Standard normal for sample element e: Philox4x32-10 (Salmon et al., SC'11) at
// counter (e, stream) with key (seed); Box-Muller of its first two words as
// 23-bit uniforms (exact in FP32).
__device__ __forceinline__ float philox_normal(unsigned long long e, const SampleGen& G) {
  unsigned c0 = (unsigned)e, c1 = (unsigned)(e >> 32), c2 = G.stream_lo, c3 = G.stream_hi;
  unsigned k0 = G.seed_lo, k1 = G.seed_hi;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const unsigned lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  const float u0 = ((float)(c0 >> 9) + 0.5f) * (1.0f / 8388608.0f);
  const float u1 = ((float)(c1 >> 9) + 0.5f) * (1.0f / 8388608.0f);
  return sqrtf(-2.0f * logf(u0)) * cospif(2.0f * u1);
}

__device__ __forceinline__ float lane_read(float v, int src_byte_addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_byte_addr, __float_as_int(v)));
}

__device__ __forceinline__ float med3(float t, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(t, lo, hi);
}

// Hide a value from loop-invariant code motion and CSE. Per-row addresses are
// cheap to recompute but, if hoisted out of the iteration loop, each one would
// occupy registers for the whole solve.
template <typename T>
__device__ __forceinline__ T opaque(T v) {
  __asm__ volatile("" : "+v"(v));
  return v;
}

// Write-only target for stores of lanes whose row or column lies outside the
// problem (padding rows of the last chunk, samples past N). Redirecting those
// stores keeps every store unconditional, so the solver has no divergent
// branches. Large enough for any per-lane row offset (4 blocks x PRISM_MAX_H).
static __device__ float g_store_sink[4 * 128 + 64];

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

template <int HQ, bool EXACT, int GEMM, bool PLAN = false>
struct TileSolver {
  static constexpr int NB = (HQ + 3) / 4;    // 16-row output blocks (4 registers each)
  static constexpr int NJ4 = (HQ + 3) / 4;   // FP32 k-steps, grouped by four
  static constexpr int NJ8 = (HQ + 7) / 8;   // 16-bit k-steps of eight

  v4f xb[NB];
  float* xt_lds;     // this wave's copy of the samples in LDS, [HQ][64]
  float qv[HQ], qq[HQ], qa[HQ], qj[HQ];
  float sw[HQ];
  float se[HQ];
  float sfw[3], sfe[3];   // higher chunks' transposed position sums (raw reads)
  static constexpr int kXtAhead = HQ <= 13 ? (PLAN ? (HQ < 4 ? HQ : 4) : HQ) : (HQ <= 24 ? 4 : 1);
  float xt_ahead[kXtAhead];   // first samples of the chunk, read ahead of the defect stage
  float rpm, rdm;

  int lane, g, nvalid;
  int a_prev, a_next, a_prev2, a_next2;   // ds_bpermute byte addresses
  float lbV, ubV, lbQ, ubQ, lbA, ubA, lbJ, ubJ, v0;
  // bounds of the jerk row in chunk position 0: for chunk 0 that row (step 1) is
  // outside the problem (jerk rows are steps 2..H) and identically zero, so its
  // bounds are widened to hold 0 and the row stays inert (z = s = 0, q = 0)
  float lbJ0, ubJ0;
  float rho, alpha, oma;
  float cV, cQ, cJ;   // block penalties relative to the acceleration block

  __device__ __forceinline__ float X(int i) const { return xb[i >> 2][i & 3]; }

  // Rows past the horizon (only in the last chunk(s)) must not feed back.
  __device__ __forceinline__ bool row_ok(int i) const {
    if (EXACT || i < HQ - 3) return true;
    return i < nvalid;
  }
  __device__ __forceinline__ float mask(int i, float v) const {
    if (EXACT || i < HQ - 3) return v;
    return i < nvalid ? v : 0.0f;
  }

  // Sums over the lower / higher chunks of the column. The three partner reads are
  // independent (one LDS round trip); the sum is formed as T_near + (T_mid + T_far).
  __device__ __forceinline__ float excl_prefix(float T) const {   // sum over lower chunks
    float a = lane_read(T, a_prev);    // chunk g-1
    float b = lane_read(T, a_prev2);   // chunk g-2
    float c = lane_read(T, a_next);    // chunk g-3 (lane - 48 = lane + 16 mod 64)
    a = (g == 0) ? 0.0f : a;
    b = (g < 2) ? 0.0f : b;
    c = (g < 3) ? 0.0f : c;
    return a + (b + c);
  }
  // Sum over the higher chunks in two parts: the reads are issued where T is known
  // and summed where the result is needed, so the LDS round trip overlaps other rows.
  __device__ __forceinline__ void suffix_reads(float T, float (&r)[3]) const {
    r[0] = lane_read(T, a_next);    // chunk g+1
    r[1] = lane_read(T, a_next2);   // chunk g+2
    r[2] = lane_read(T, a_prev);    // chunk g+3 (lane + 48 = lane - 16 mod 64)
  }
  __device__ __forceinline__ float suffix_sum(const float (&r)[3]) const {
    const float a = (g == 3) ? 0.0f : r[0];
    const float b = (g >= 2) ? 0.0f : r[1];
    const float c = (g >= 1) ? 0.0f : r[2];
    return a + (b + c);
  }

  // One constraint row: slack clip and multiplier update from s = (C x)_row.
  template <bool CHECK>
  __device__ __forceinline__ float rowop(float s, float& q, float lb, float ub, float& e,
                                         float& u) const {
    q = fmaf(alpha, s, q);                     // t, computed in place
    const float z = med3(q, lb, ub);
    const float w = fmaf(2.0f, z, -q) - s;
    if constexpr (CHECK) { e = z - s; u = q - z; }
    q = fmaf(-alpha, z, q);                    // q' = t - alpha z
    // On check iterations the stop test follows: keep q' computed here. Left free, the
    // compiler sinks this update past the residual reduction, keeping t and z alive
    // across it instead of q' (about 100 more registers at HQ = 25). Empty asm: no code.
    if constexpr (CHECK) asm volatile("" : "+v"(q));
    return w;
  }

  // Row update for every block and transposed accumulation sw = C^T w
  // (se = C^T e and the primal residual on check iterations).
  template <bool CHECK>
  __device__ __forceinline__ void row_update() {
    float e = 0.0f, u = 0.0f;
    if constexpr (CHECK) rpm = 0.0f;
    auto track = [&](int i, float ev, float uv, int blk) {
      (void)i;
      (void)uv;
      (void)blk;
      if constexpr (CHECK) rpm = fmaxf(rpm, fabsf(ev));
    };
    // the acceleration/jerk block's boundary values depend only on x: read them first
    const float xprev_r = lane_read(X(HQ - 1), a_prev);
    const float aprev_r = lane_read(X(HQ - 1) - X(HQ - 2), a_prev);
    // ---- position block: s = prefix sum (chunk prefix + lower chunks' totals)
    {
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < HQ; ++i) { acc += X(i); sw[i] = acc; }
      const float off = excl_prefix(acc);
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        const float s = sw[i] + off;
        float w = rowop<CHECK>(s, qq[i], lbQ, ubQ, e, u);
        w = mask(i, w);
        sw[i] = w;
        if constexpr (CHECK) { e = mask(i, e); se[i] = e; track(i, e, u, 1); }
      }
      // C_Q^T: suffix sums within the chunk, higher chunks' totals added to d later
      float suf = 0.0f, sufe = 0.0f;
#pragma unroll
      for (int i = HQ - 1; i >= 0; --i) {
        suf = fmaf(cQ, sw[i], suf);
        sw[i] = suf;
        if constexpr (CHECK) { sufe = fmaf(cQ, se[i], sufe); se[i] = sufe; }
      }
      suffix_reads(suf, sfw);
      if constexpr (CHECK) suffix_reads(sufe, sfe);
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- velocity block: s = x
#pragma unroll
    for (int i = 0; i < HQ; ++i) {
      float w = rowop<CHECK>(X(i), qv[i], lbV, ubV, e, u);
      sw[i] = fmaf(cV, mask(i, w), sw[i]);
      if constexpr (CHECK) { e = mask(i, e); se[i] = fmaf(cV, e, se[i]); track(i, e, u, 0); }
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- acceleration and jerk blocks, streamed along the chunk.
    // C_A^T w_A + cJ C_J^T w_J = D^T v with v_k = wA_k + cJ (wJ_k - wJ_{k+1}),
    // (D^T v)_k = v_k - v_{k+1}.
    {
      // the defect stage's first samples come from LDS while these rows run
#pragma unroll
      for (int i = 0; i < kXtAhead; ++i) xt_ahead[i] = xt_lds[i * 64 + lane];
      __builtin_amdgcn_sched_barrier(0);   // keep the reads here, ahead of the rows
      float xprev = (g == 0) ? v0 : xprev_r;
      float aprev = (g == 0) ? 0.0f : aprev_r;
      float wa_p = 0.0f, wj_p = 0.0f, wj_0 = 0.0f, v_0 = 0.0f, v_pm = 0.0f;
      float ea_p = 0.0f, ej_p = 0.0f, ej_0 = 0.0f, ve_0 = 0.0f, ve_pm = 0.0f;
      // the next chunk's first terms are read as soon as they exist (step 2 of the
      // chunk) and used after the loop
      float wj_nr = 0.0f, v_nr = 0.0f, ej_nr = 0.0f, ve_nr = 0.0f;
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        const float sa = X(i) - xprev;
        const float sj = sa - aprev;
        xprev = X(i);
        aprev = sa;
        float ea = 0.0f, ej = 0.0f, ua = 0.0f, uj = 0.0f;
        float wa = mask(i, rowop<CHECK>(sa, qa[i], lbA, ubA, ea, ua));
        float wj = mask(i, rowop<CHECK>(sj, qj[i], i == 0 ? lbJ0 : lbJ, i == 0 ? ubJ0 : ubJ,
                                        ej, uj));
        if constexpr (CHECK) {
          ea = mask(i, ea);
          ej = mask(i, ej);
          track(i, ea, ua, 2);
          track(i, ej, uj, 3);
        }
        if (i == 0) {
          wj_0 = wj;
          if constexpr (CHECK) ej_0 = ej;
        } else {
          const float v = fmaf(cJ, wj_p - wj, wa_p);
          float ve = 0.0f;
          if constexpr (CHECK) ve = fmaf(cJ, ej_p - ej, ea_p);
          if (i == 1) {
            v_0 = v;
            wj_nr = lane_read(wj_0, a_next);
            v_nr = lane_read(v_0, a_next);
            if constexpr (CHECK) {
              ve_0 = ve;
              ej_nr = lane_read(ej_0, a_next);
              ve_nr = lane_read(ve_0, a_next);
            }
          } else {
            sw[i - 2] += v_pm - v;
            if constexpr (CHECK) se[i - 2] += ve_pm - ve;
          }
          v_pm = v;
          if constexpr (CHECK) ve_pm = ve;
        }
        wa_p = wa;
        wj_p = wj;
        if constexpr (CHECK) { ea_p = ea; ej_p = ej; }
      }
      const float wj_n = (g == 3) ? 0.0f : wj_nr;
      const float v_last = fmaf(cJ, wj_p - wj_n, wa_p);
      sw[HQ - 2] += v_pm - v_last;
      const float v_n = (g == 3) ? 0.0f : v_nr;
      sw[HQ - 1] += v_last - v_n;
      if constexpr (CHECK) {
        const float ej_n = (g == 3) ? 0.0f : ej_nr;
        const float ve_last = fmaf(cJ, ej_p - ej_n, ea_p);
        se[HQ - 2] += ve_pm - ve_last;
        const float ve_n = (g == 3) ? 0.0f : ve_nr;
        se[HQ - 1] += ve_last - ve_n;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- defect d = (x~ - x) + rho C^T w; dual residual on check iterations
    if constexpr (CHECK) rdm = 0.0f;
    const float offw = suffix_sum(sfw);
    float offe = 0.0f;
    if constexpr (CHECK) offe = suffix_sum(sfe);
#pragma unroll
    for (int i = 0; i < HQ; ++i) {
      const float xt = i < kXtAhead ? xt_ahead[i] : xt_lds[i * 64 + lane];
      const float d = fmaf(rho, sw[i] + offw, xt - X(i));
      sw[i] = d;
      if constexpr (CHECK) {
        float r = fabsf(fmaf(rho, se[i] + offe, -d));
        r = mask(i, r);
        if (i == 0) r = (g == 0) ? 0.0f : r;     // step 1: absorbed by x_1 = v0
        rdm = fmaxf(rdm, r);
      }
    }
  }

  // x += K d with FP32 operands (v_mfma_f32_16x16x4_f32). Fragments stream
  // from LDS ahead of use; the barriers keep the scheduler from hoisting
  // the whole of K into registers.
  __device__ __forceinline__ void gemm_f32(const float* __restrict__ kf) {
    __asm__ volatile("" ::: "memory");
    const v4f* k4 = reinterpret_cast<const v4f*>(kf) + lane;
    // two fragments in flight (one for chunks above 24, where the registers are
    // spoken for): a block's last group can hold a single MFMA, too little cover
    // for one LDS round trip. Slots rotate by group index (compile-time after
    // unrolling), so no register moves.
    constexpr int total = NB * NJ4;
    constexpr int ahead = HQ <= 24 ? 2 : 1;
    v4f f[ahead + 1];
    f[0] = k4[0];
    if (ahead == 2 && total > 1) f[1] = k4[64];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int jj = 0; jj < NJ4; ++jj) {
        const int idx = b * NJ4 + jj;
        if (idx + ahead < total) f[(idx + ahead) % (ahead + 1)] = k4[(idx + ahead) * 64];
        const v4f a = f[idx % (ahead + 1)];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 4 * jj + e;
          if (j < HQ) xb[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], sw[j], xb[b], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // x += K d with 16-bit operands and FP32 accumulation (v_mfma_f32_16x16x32_*).
  __device__ __forceinline__ void gemm_16(const void* __restrict__ kl) {
    __asm__ volatile("" ::: "memory");
    const v4u* k16 = reinterpret_cast<const v4u*>(kl) + lane;
    using VT = typename std::conditional<GEMM == GEMM_BF16, v8bf, v8h>::type;
    using ST = typename std::conditional<GEMM == GEMM_BF16, __bf16, _Float16>::type;
    VT dv[NJ8];
#pragma unroll
    for (int jj = 0; jj < NJ8; ++jj)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = 8 * jj + e;
        dv[jj][e] = (j < HQ) ? (ST)sw[j] : (ST)0.0f;
      }
    // K fragments stream from LDS up to kDepth ahead of their MFMA, so the LDS
    // latency is paid about once per GEMM instead of once per MFMA
    constexpr int NT = NB * NJ8;
    constexpr int kDepth = NT < 8 ? NT : (HQ >= 15 ? 4 : 8);
    v4u ring[kDepth];
#pragma unroll
    for (int t = 0; t < kDepth; ++t) ring[t] = k16[t * 64];
#pragma unroll
    for (int idx = 0; idx < NT; ++idx) {
      const int b = idx / NJ8, jj = idx % NJ8;
      const v4u a = ring[idx % kDepth];
      if (idx + kDepth < NT) ring[idx % kDepth] = k16[(idx + kDepth) * 64];
      if constexpr (GEMM == GEMM_BF16)
        xb[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), dv[jj], xb[b], 0, 0, 0);
      else
        xb[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), dv[jj], xb[b], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // q <- c C x + q for every row, with x_0 := vb in the first acceleration and
  // jerk rows (c = 1 - alpha adds the slack of x to the relaxed state).
  __device__ __forceinline__ void prep_q(float c, float vb) {
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < HQ; ++i) { acc += X(i); sw[i] = acc; }
    const float off = excl_prefix(acc);
    float xprev = lane_read(X(HQ - 1), a_prev);
    float aprev = lane_read(X(HQ - 1) - X(HQ - 2), a_prev);
    xprev = (g == 0) ? vb : xprev;
    aprev = (g == 0) ? 0.0f : aprev;
#pragma unroll
    for (int i = 0; i < HQ; ++i) {
      const float sa = X(i) - xprev;
      const float sj = sa - aprev;
      xprev = X(i);
      aprev = sa;
      qv[i] = fmaf(c, X(i), qv[i]);
      qq[i] = fmaf(c, sw[i] + off, qq[i]);
      qa[i] = fmaf(c, sa, qa[i]);
      qj[i] = fmaf(c, sj, qj[i]);
    }
  }

  // Cold state from the sample held in LDS: x = x~ with x_1 = v0, q = (1 - alpha) C x.
  __device__ __forceinline__ void restart_cold() {
#pragma unroll
    for (int i = 0; i < 4 * NB; ++i) xb[i >> 2][i & 3] = (i < HQ) ? xt_lds[i * 64 + lane] : 0.0f;
    if (g == 0) xb[0][0] = v0;
#pragma unroll
    for (int i = 0; i < HQ; ++i) { qv[i] = 0.0f; qq[i] = 0.0f; qa[i] = 0.0f; qj[i] = 0.0f; }
    if (oma != 0.0f) prep_q(oma, v0);
  }

  // Advance a row block held as this lane's chunk (steps g*HQ .. g*HQ+HQ-1) by
  // one step: step k takes step k+1, the last step H-1 keeps its value, rows
  // past H stay zero. The chunk boundary comes from the next lane group.
  __device__ __forceinline__ void shift_rows(float (&r)[HQ], int H) {
    const float nxt_raw = lane_read(r[0], a_next);
    const float nxt = (g == 3) ? 0.0f : nxt_raw;
    const int lastrel = H - 1 - g * HQ;          // in [0, HQ) only for the group holding H-1
    constexpr int kLo = HQ > 4 ? HQ - 4 : 0;     // H >= 4 HQ - 3 puts lastrel here when HQ > 2
    float keep[HQ - kLo];
#pragma unroll
    for (int i = kLo; i < HQ; ++i) keep[i - kLo] = r[i];
#pragma unroll
    for (int i = 0; i + 1 < HQ; ++i) r[i] = r[i + 1];
    r[HQ - 1] = nxt;
#pragma unroll
    for (int i = kLo; i < HQ; ++i) r[i] = (i == lastrel) ? keep[i - kLo] : r[i];
  }

  __device__ void run(const TileArgs& A, int j, int s0, const float* __restrict__ kf32,
                      const void* __restrict__ k16, float* xt_wave) {
    xt_lds = xt_wave;
    lane = threadIdx.x & 63;
    g = lane >> 4;
    const int c = lane & 15;
    a_prev = ((lane - 16) & 63) << 2;
    a_next = ((lane + 16) & 63) << 2;
    a_prev2 = ((lane - 32) & 63) << 2;
    a_next2 = ((lane + 32) & 63) << 2;
    const int H = A.H, nj = A.nj;
    const int s = s0 + c;
    const bool col_ok = s < A.N;
    const int s_ld = col_ok ? s : A.N - 1;     // loads always read a valid column
    {
      const int nv = H - g * HQ;
      nvalid = nv < 0 ? 0 : (nv > HQ ? HQ : nv);
    }
    const JointRowParams& jp = A.jp[j];
    lbV = jp.lb[0]; ubV = jp.ub[0];
    lbQ = jp.lb[1]; ubQ = jp.ub[1];
    lbA = jp.lb[2]; ubA = jp.ub[2];
    lbJ = jp.lb[3]; ubJ = jp.ub[3];
    lbJ0 = (g == 0) ? fminf(lbJ, 0.0f) : lbJ;
    ubJ0 = (g == 0) ? fmaxf(ubJ, 0.0f) : ubJ;
    v0 = jp.v0;
    rho = A.rho;
    alpha = A.alpha;
    oma = 1.0f - A.alpha;
    cV = A.cV;
    cQ = A.cQ;
    cJ = A.cJ;

    // ---- load the sample (and warm state). Lane bases include the chunk
    // offset so the per-row offsets i*nj are wave-uniform; rows past H read
    // row 0 of the column and are zeroed.
    const size_t colbase = (size_t)s_ld * H * nj + j;
    const size_t chunk = (size_t)(g * HQ) * nj;
    auto ld_row = [&](const float* p, int i) -> float {
      if (EXACT || i < HQ - 3) return p[i * nj];
      const int r = (i < nvalid) ? i : -g * HQ;  // row 0 of this column
      const float v = p[r * nj];
      return (i < nvalid) ? v : 0.0f;
    };
    if (PLAN && A.gen_on) {
      // draw the samples: x~ = nu + sigma * z, one generator call per element
      const SampleGen& G = A.gen;
#pragma unroll 1
      for (int i = 0; i < HQ; ++i) {
        const bool ok = EXACT || i < nvalid;
        const int k = ok ? g * HQ + i : 0;
        const float z = philox_normal(((unsigned long long)s_ld * H + k) * nj + j, G);
        const int pj = k * nj + j;
        xt_lds[i * 64 + lane] = ok ? fmaf(G.sigma[pj], z, G.nu[pj]) : 0.0f;
      }
#pragma unroll
      for (int i = 0; i < 4 * NB; ++i) xb[i >> 2][i & 3] = (i < HQ) ? xt_lds[i * 64 + lane] : 0.0f;
      if (G.xs_out != nullptr) {
        float* po = opaque(col_ok ? G.xs_out + colbase + chunk : g_store_sink);
        const int st = col_ok ? nj : 0;
#pragma unroll
        for (int i = 0; i < HQ; ++i) {
          float* dst = po + i * st;
          if (!(EXACT || i < HQ - 3)) dst = (i < nvalid) ? dst : g_store_sink;
          *dst = X(i);
        }
      }
    } else {
      const float* px = opaque(A.xin + colbase + chunk);
#pragma unroll
      for (int i = 0; i < 4 * NB; ++i) {
        const float v = (i < HQ) ? ld_row(px, i) : 0.0f;
        xb[i >> 2][i & 3] = v;
        if (i < HQ) xt_lds[i * 64 + lane] = v;
      }
    }
    const bool shift = A.shift != 0 && A.xw != nullptr;
    if (A.xw != nullptr) {
      const float* pw = opaque(A.xw + colbase + chunk);
#pragma unroll
      for (int i = 0; i < 4 * NB; ++i) xb[i >> 2][i & 3] = (i < HQ) ? ld_row(pw, i) : 0.0f;
    }
    const size_t ubase = ((size_t)s_ld * nj + j) * 4 * H;
    if (A.uw != nullptr) {
      // warm state: q = (1 - alpha) z + u of the previous solve
      const float* pu = opaque(A.uw + ubase + g * HQ);
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        const int r = (EXACT || i < HQ - 3 || i < nvalid) ? i : -g * HQ;
        const bool ok = EXACT || i < HQ - 3 || i < nvalid;
        qv[i] = ok ? pu[0 * H + r] : 0.0f;
        qq[i] = ok ? pu[1 * H + r] : 0.0f;
        qa[i] = ok ? pu[2 * H + r] : 0.0f;
        qj[i] = ok ? pu[3 * H + r] : 0.0f;
      }
      if (g == 0) { qa[0] = 0.0f; qj[0] = 0.0f; }   // rows fixed by x_1 = v0 carry no dual
    } else {
#pragma unroll
      for (int i = 0; i < HQ; ++i) { qv[i] = 0.0f; qq[i] = 0.0f; qa[i] = 0.0f; qj[i] = 0.0f; }
    }
    if (shift) {
      // Next MPC step: the multiplier and the slack's deviation from C x move one
      // step ahead (last step repeating) and the slack is rebuilt on the shifted
      // iterate: q' = (1 - alpha) C x' + shift(q - (1 - alpha) C x). The previous
      // boundary value is the warm iterate's first step.
      if (A.uw != nullptr && A.alpha != 1.0f) prep_q(-oma, lane_read(X(0), c << 2));
      if (A.uw != nullptr) {
        shift_rows(qv, H);
        shift_rows(qq, H);
        shift_rows(qa, H);
        shift_rows(qj, H);
        if (g == 0) { qa[0] = 0.0f; qj[0] = 0.0f; }
      }
      float r[HQ];
#pragma unroll
      for (int i = 0; i < HQ; ++i) r[i] = X(i);
      shift_rows(r, H);
#pragma unroll
      for (int i = 0; i < HQ; ++i) xb[i >> 2][i & 3] = r[i];
    }
    if (g == 0) xb[0][0] = v0;                 // x_1 = v0 (eq. (A_b_def))
    // cold start or shifted state: q += (1 - alpha) C x0 (the slack of x0)
    if ((A.uw == nullptr || shift) && A.alpha != 1.0f) prep_q(oma, v0);

    const bool tolmode = A.tolmode != 0;
    // the tolerance as a uniform value: the batch kernel reads its arguments from a
    // table in global memory, and a per-lane copy made the stop test a divergent branch
    const float tol = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, A.tol)));
    const bool reduced = GEMM != GEMM_F32;
    const int iters = A.iters;
    const int ce = A.check_every;
    // Fixed count: the last `tail` iterations run the FP32 GEMM. Residual-driven:
    // the reduced GEMM runs until the tile meets the tolerance, then `tail` FP32
    // iterations follow (check points inside the tail do not stop it) and the tile
    // stops at the end of the tail if it still meets the tolerance there, else at the
    // first later check point that does (FP32 iterations, checked every check_every).
    // Reduced forms in residual mode: the rounded x-update perturbs the iteration map,
    // and near alpha = 2 that can outweigh the contraction, so that the iterates
    // diverge, or hold them at a rounding floor above tol. A tile whose residual at a
    // check point exceeds kReducedRise times the lowest it had at an earlier one
    // (exact iterations rise by at most about 15x on the way down) restarts there from
    // the sample with a cold state and the FP32 GEMM: from then on it runs the FP32
    // form, which stops at the first check point that meets tol (continuing from the
    // diverged state in FP32 was measured to need thousands of iterations). A tile
    // whose residual has set no new low for kReducedStall iterations (exact iterations
    // go at most about 130 without one) goes on from its state in FP32, as after
    // convergence: `tail` iterations at least, then the first check point meeting tol.
    const int f32_from = !reduced ? 0 : (tolmode ? INT_MAX : iters - A.tail);
    float rlow = __builtin_inff();   // lowest tile residual at the check points so far
    int it_low = 0;                  // the check point that set it
    bool f32p = !reduced;
    int it = 0;
    int tail_end = -1;           // iteration that ends the FP32 tail after convergence
    // Check points (residuals computed): iteration 0, every check_every in residual
    // mode, the end of the tail, and the cap. Between them the plain iterations run
    // in branch-free inner loops, one per GEMM precision.
    for (;;) {
      row_update<true>();
      if (tolmode) {
        // Every lane holds the maximum; read back as uniform, the stop test and the GEMM
        // switch are scalar branches, so the iteration counter and the inner loops stay
        // scalar (with a per-lane maximum they became execution-masked vector loops).
        const float r = col_ok ? fmaxf(rpm, rdm) : 0.0f;
        const float rm = __builtin_bit_cast(
            float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, wave_max(r))));
        if constexpr (GEMM == GEMM_F32) {
          if (rm <= tol) break;
        } else {
          if (rm <= tol) {
            // the FP32 tail has run (or there is none): done
            if (A.tail <= 0 || (f32p && it >= tail_end)) break;
            if (!f32p) {
              f32p = true;
              tail_end = it + A.tail;
            }
          } else if (it == tail_end) {
            tail_end = -1;
          }
          if (!f32p && it < iters) {
            if (rm > kReducedRise * rlow) {
              restart_cold();
              f32p = true;
              tail_end = -1;
              continue;   // rows of the restarted state at this check point
            }
            if (rm < rlow) {
              rlow = rm;
              it_low = it;
            } else if (it - it_low >= kReducedStall) {
              f32p = true;
              tail_end = it + A.tail;
            }
          }
        }
      }
      if (it == iters) break;
      int next = iters;
      if (tolmode) {
        const int c = (it / ce + 1) * ce;
        next = c < next ? c : next;
        if (tail_end > it && tail_end < next) next = tail_end;
      }
      if constexpr (GEMM == GEMM_F32) {
        gemm_f32(kf32);
        ++it;
        while (it < next) {
          row_update<false>();
          gemm_f32(kf32);
          ++it;
        }
      } else {
        if (f32p || it >= f32_from) gemm_f32(kf32);
        else gemm_16(k16);
        ++it;
        if (!f32p) {
          const int e = f32_from < next ? f32_from : next;
          while (it < e) {
            row_update<false>();
            gemm_16(k16);
            ++it;
          }
        }
        while (it < next) {
          row_update<false>();
          gemm_f32(kf32);
          ++it;
        }
      }
    }

    if (PLAN && A.cost_on) {
      // tracking cost of this column: w_pos (theta_k - ref_k)^2 + w_vel x_k^2 with
      // theta_k = q0 + dt * (sum of x up to step k); rows past H hold x = 0
      const CostArgs& Cg = A.cost;
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        acc += X(i);
        sw[i] = acc;
      }
      const float off = excl_prefix(acc);
      const float q0j = A.jp[j].q0;
      float c = 0.0f;
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        const bool ok = EXACT || i < nvalid;
        const int k = ok ? g * HQ + i : 0;
        const float d = fmaf(Cg.dt, sw[i] + off, q0j - Cg.ref[k * nj + j]);
        const float t = fmaf(Cg.w_pos * d, d, Cg.w_vel * X(i) * X(i));
        c += ok ? t : 0.0f;
      }
      c += __shfl_xor(c, 16, 64);
      c += __shfl_xor(c, 32, 64);
      if (g == 0 && col_ok) Cg.cost[(size_t)s * nj + j] = c;
    }

    // ---- store x and the per-column residuals
    bool bad = false;
    {
      float* po = opaque(col_ok ? A.xout + colbase + chunk : g_store_sink);
      const int st = col_ok ? nj : 0;
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        const float v = X(i);
        bad |= (v != v);
        float* dst = po + i * st;
        if (!(EXACT || i < HQ - 3)) dst = (i < nvalid) ? dst : g_store_sink;
        *dst = v;
      }
    }
    if (A.xsave != nullptr) {
      float* po = opaque(col_ok ? A.xsave + colbase + chunk : g_store_sink);
      const int st = col_ok ? nj : 0;
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        float* dst = po + i * st;
        if (!(EXACT || i < HQ - 3)) dst = (i < nvalid) ? dst : g_store_sink;
        *dst = X(i);
      }
    }
    if (A.uout != nullptr) {
      // relaxed dual state q = (1 - alpha) z + u per row, for warm-starting
      float* qb = opaque(col_ok ? A.uout + ubase + g * HQ : g_store_sink);
      const int bs = col_ok ? H : 0;
#pragma unroll
      for (int i = 0; i < HQ; ++i) {
        float* d0 = qb + 0 * bs + i;
        float* d1 = qb + 1 * bs + i;
        float* d2 = qb + 2 * bs + i;
        float* d3 = qb + 3 * bs + i;
        if (!(EXACT || i < HQ - 3)) {
          const bool ok = i < nvalid;
          d0 = ok ? d0 : g_store_sink;
          d1 = ok ? d1 : g_store_sink;
          d2 = ok ? d2 : g_store_sink;
          d3 = ok ? d3 : g_store_sink;
        }
        *d0 = qv[i];
        *d1 = qq[i];
        *d2 = qa[i];
        *d3 = qj[i];
      }
    }
    float rp = rpm, rd = rdm;
    rp = fmaxf(rp, __shfl_xor(rp, 16, 64));
    rp = fmaxf(rp, __shfl_xor(rp, 32, 64));
    rd = fmaxf(rd, __shfl_xor(rd, 16, 64));
    rd = fmaxf(rd, __shfl_xor(rd, 32, 64));
    int anybad = bad ? 1 : 0;
    anybad |= __shfl_xor(anybad, 16, 64);
    anybad |= __shfl_xor(anybad, 32, 64);
    if (anybad) { rp = __builtin_nanf(""); rd = __builtin_nanf(""); }
    if (g == 0 && col_ok) {
      const size_t o = (size_t)s * nj + j;
      if (A.rp) A.rp[o] = rp;
      if (A.rd) A.rd[o] = rd;
      if (A.itout) A.itout[o] = it;
    }
  }
};

}  // namespace prism

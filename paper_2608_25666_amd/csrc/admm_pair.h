// Two-wave tiles for gfx950: one tile (16 samples of one joint) is projected by a
// pair of waves of one workgroup, each holding half of the steps, so that the rows and
// the x-update of one iteration are split between two SIMDs.
//
// Measured on MI355X (per iteration, a lone tile, FP32): H = 100 3.8 us against 4.2 us
// for one wave; H = 50 2.1 against 1.6; H = 20 1.4 against 0.6. The iteration's
// dependency chain (member 1's rows and defect, a hand-over, member 0's defect, a
// hand-over, the x-update) keeps the per-iteration shuffles and LDS round trips serial,
// and below H = 100 they outweigh the halved row and GEMM work; with many tiles in
// flight the one-wave kernel is faster at every H. Hence opt-in (tile_waves = 2).
//
// A tile's H steps are cut into eight chunks of HP = ceil(H/8) rows. Member m of the
// pair (m = 0, 1) holds chunks 4m .. 4m+3: lane l = 16 g + c owns column c and the
// steps (4m + g) HP .. (4m + g) HP + HP - 1, in the same register layout as the
// one-wave solver (admm_tile.h, which also states the iteration). Each member updates
// its own constraint rows and computes its own rows of the x-update on MFMA; its
// A-operand fragments cover its output rows against the k-steps of both members
// (factor.h, layout_pair_*), the B operand being its own defect registers and then
// its partner's defect read from LDS.
//
// What crosses between the members in one iteration (per column, through LDS):
//   S1, member 0 -> 1: the sum of x over member 0's steps (position rows of member 1),
//       member 0's last x and last first difference (acceleration and jerk rows of
//       member 1's first step);
//   S2, member 1 -> 0: its weighted sums of the position rows' w (the transposed
//       position rows of member 0), the jerk and acceleration terms of its first two
//       steps (the transposed rows of member 0's last two steps), its defect, and on
//       check iterations its residuals and NaN flags;
//   S3, member 0 -> 1: its defect (and residuals, NaN flags on check iterations).
// Each hand-over is a flag in LDS raised after the data is written (release fence)
// and awaited by the partner (acquire fence). Waits are bounded: a wait that exceeds
// kPairSpinLimit polls ends the kernel for that pair, with NaN residuals for its tile.
// Both members take every decision (stop, tail) from the same exchanged values, so
// their control flow, and with it the sequence of hand-overs, is identical.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "admm_kernels.h"
#include "admm_tile.h"
#include "kernel_args.h"

namespace prism {

constexpr int kPairSpinLimit = 1 << 22;   // polls of a partner's flag before giving up

// Per-pair LDS block (32-bit words), placed after the factor fragments.
template <int HP>
struct PairLds {
  static constexpr int FLAG0 = 0, FLAG1 = 1;     // hand-over counters of member 0 / 1
  static constexpr int TILE = 2, QUEUE = 3;      // next tile index (-1: none), its queue
  static constexpr int T0 = 4;                   // [16] sum of x over member 0
  static constexpr int XL = T0 + 16;             // [16] member 0's last x
  static constexpr int AL = XL + 16;             // [16] member 0's last first difference
  static constexpr int W1 = AL + 16;             // [16] member 1's weighted position sums (w)
  static constexpr int W1E = W1 + 16;            // [16] the same for e (check iterations)
  static constexpr int WJ = W1E + 16;            // [16] member 1: jerk w of its first step
  static constexpr int VN = WJ + 16;             // [16] member 1: v of its second step
  static constexpr int EJ = VN + 16;             // [16] check: jerk e of its first step
  static constexpr int VEN = EJ + 16;            // [16] check: ve of its second step
  static constexpr int RP = VEN + 16;            // [2][16] per-column r_p of each member
  static constexpr int RD = RP + 32;             // [2][16] per-column r_d of each member
  static constexpr int BAD = RD + 32;            // [2][16] per-column NaN flags
  static constexpr int D = BAD + 32;             // [2][HP][64] defect of each member
  static constexpr int XT = D + 2 * HP * 64;     // [2][HP][64] samples of each member
  static constexpr int WORDS = XT + 2 * HP * 64;
  static_assert(WORDS == pair_lds_words(HP), "pair_lds_words matches the block");
};

// Maximum over the wave, read back with readfirstlane: every lane holds it after the
// butterfly, and saying so keeps the stop test (and with it the loop counters and the
// hand-over sequence numbers) uniform, so the hand-over waits are scalar loops.
__device__ __forceinline__ float pair_wave_max(float v) {
  v = wave_max(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ void pair_signal(int* flag, int v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(flag, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until *flag >= v; false if the partner did not get there within the bound.
__device__ __forceinline__ bool pair_wait(int* flag, int v) {
  for (int n = 0; n < kPairSpinLimit; ++n) {
    const int f = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (f >= v) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      return true;
    }
  }
  return false;
}

template <int HP, int GEMM>
struct PairSolver {
  using L = PairLds<HP>;
  static constexpr int NB = (HP + 3) / 4;     // 16-row output blocks (4 registers each)
  static constexpr int NJ4 = (HP + 3) / 4;    // FP32 k-steps, grouped by four
  static constexpr int NJ8 = (HP + 7) / 8;    // 16-bit k-steps of eight
  // Steps past H exist only in member 1's chunks, and only in their last 7 registers
  // (8 HP - H <= 7); earlier registers need no mask.
  static constexpr int kMaskFrom = HP > 7 ? HP - 7 : 0;

  v4f xb[NB];
  float qv[HP], qq[HP], qa[HP], qj[HP];
  float sw[HP], se[HP];
  float sfw[3], sfe[3];
  float rpm, rdm;
  // the next chunk's first jerk / v terms and what the streamed rows leave for them
  float wj_nr, v_nr, ej_nr, ve_nr;
  float v_pm, wj_p, wa_p, ve_pm, ej_p, ea_p;
  float wj_first, v_second, ej_first, ve_second;   // this lane group's own first terms

  int lane, g, c, m, nvalid;
  int a_prev, a_next, a_prev2, a_next2;
  float lbV, ubV, lbQ, ubQ, lbA, ubA, lbJ, ubJ, lbJ0, ubJ0, v0;
  float rho, alpha, oma, cV, cQ, cJ;
  float* P;      // this pair's LDS block
  int* Pi;       // the same, as ints
  float* xt;     // this member's samples in LDS, [HP][64]

  __device__ __forceinline__ float X(int i) const { return xb[i >> 2][i & 3]; }
  __device__ __forceinline__ float mask(int i, float v) const {
    if (i < kMaskFrom) return v;
    return i < nvalid ? v : 0.0f;
  }

  __device__ __forceinline__ float excl_prefix(float T) const {   // lower chunks of the member
    float a = lane_read(T, a_prev);
    float b = lane_read(T, a_prev2);
    float d = lane_read(T, a_next);
    a = (g == 0) ? 0.0f : a;
    b = (g < 2) ? 0.0f : b;
    d = (g < 3) ? 0.0f : d;
    return a + (b + d);
  }
  __device__ __forceinline__ void suffix_reads(float T, float (&r)[3]) const {
    r[0] = lane_read(T, a_next);
    r[1] = lane_read(T, a_next2);
    r[2] = lane_read(T, a_prev);
  }
  __device__ __forceinline__ float suffix_sum(const float (&r)[3]) const {   // higher chunks of the member
    const float a = (g == 3) ? 0.0f : r[0];
    const float b = (g >= 2) ? 0.0f : r[1];
    const float d = (g >= 1) ? 0.0f : r[2];
    return a + (b + d);
  }
  // sum over the member's four lane groups (every lane gets its column's total)
  __device__ __forceinline__ float member_sum(float v) const {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
  }
  __device__ __forceinline__ float member_max(float v) const {
    v = fmaxf(v, __shfl_xor(v, 16, 64));
    v = fmaxf(v, __shfl_xor(v, 32, 64));
    return v;
  }

  template <bool CHECK>
  __device__ __forceinline__ float rowop(float s, float& q, float lb, float ub, float& e) const {
    q = fmaf(alpha, s, q);
    const float z = med3(q, lb, ub);
    const float w = fmaf(2.0f, z, -q) - s;
    if constexpr (CHECK) e = z - s;
    q = fmaf(-alpha, z, q);
    return w;
  }

  // Constraint rows of this member at the current x: slack clip, multiplier update and
  // the transposed sums of w (and e on check iterations) into sw (se), all but the
  // terms that come from the next member (member 0's last two steps and position sums).
  // t0: sum of x over member 0 (member 1; 0 for member 0); xl, al: member 0's last x and
  // last difference (member 1).
  template <bool CHECK>
  __device__ __forceinline__ void rows(float t0, float xl, float al) {
    float e = 0.0f;
    if constexpr (CHECK) rpm = 0.0f;
    const float xprev_r = lane_read(X(HP - 1), a_prev);
    const float aprev_r = lane_read(X(HP - 1) - X(HP - 2), a_prev);
    // ---- position block
    {
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < HP; ++i) { acc += X(i); sw[i] = acc; }
      const float off = excl_prefix(acc) + t0;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        const float s = sw[i] + off;
        float w = rowop<CHECK>(s, qq[i], lbQ, ubQ, e);
        sw[i] = mask(i, w);
        if constexpr (CHECK) { e = mask(i, e); se[i] = e; rpm = fmaxf(rpm, fabsf(e)); }
      }
      float suf = 0.0f, sufe = 0.0f;
#pragma unroll
      for (int i = HP - 1; i >= 0; --i) {
        suf = fmaf(cQ, sw[i], suf);
        sw[i] = suf;
        if constexpr (CHECK) { sufe = fmaf(cQ, se[i], sufe); se[i] = sufe; }
      }
      suffix_reads(suf, sfw);
      if constexpr (CHECK) suffix_reads(sufe, sfe);
      // member 1 hands its position sums to member 0 (every lane: its column's total)
      if (m == 1) {
        const float tw = member_sum(suf);
        float te = 0.0f;
        if constexpr (CHECK) te = member_sum(sufe);
        if (g == 0) {
          P[L::W1 + c] = tw;
          if constexpr (CHECK) P[L::W1E + c] = te;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- velocity block
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      float w = rowop<CHECK>(X(i), qv[i], lbV, ubV, e);
      sw[i] = fmaf(cV, mask(i, w), sw[i]);
      if constexpr (CHECK) { e = mask(i, e); se[i] = fmaf(cV, e, se[i]); rpm = fmaxf(rpm, fabsf(e)); }
    }
    __builtin_amdgcn_sched_barrier(0);
    // ---- acceleration and jerk blocks, streamed along the chunk (see admm_tile.h)
    {
      float xprev = (g == 0) ? (m == 0 ? v0 : xl) : xprev_r;
      float aprev = (g == 0) ? (m == 0 ? 0.0f : al) : aprev_r;
      float wj_0 = 0.0f, v_0 = 0.0f, ej_0 = 0.0f, ve_0 = 0.0f;
      float wa_pp = 0.0f, wj_pp = 0.0f, vpm = 0.0f, ea_pp = 0.0f, ej_pp = 0.0f, vepm = 0.0f;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        const float sa = X(i) - xprev;
        const float sj = sa - aprev;
        xprev = X(i);
        aprev = sa;
        float ea = 0.0f, ej = 0.0f;
        const float wa = mask(i, rowop<CHECK>(sa, qa[i], lbA, ubA, ea));
        const float wj = mask(i, rowop<CHECK>(sj, qj[i], i == 0 ? lbJ0 : lbJ,
                                              i == 0 ? ubJ0 : ubJ, ej));
        if constexpr (CHECK) {
          ea = mask(i, ea);
          ej = mask(i, ej);
          rpm = fmaxf(rpm, fmaxf(fabsf(ea), fabsf(ej)));
        }
        if (i == 0) {
          wj_0 = wj;
          if constexpr (CHECK) ej_0 = ej;
        } else {
          const float v = fmaf(cJ, wj_pp - wj, wa_pp);
          float ve = 0.0f;
          if constexpr (CHECK) ve = fmaf(cJ, ej_pp - ej, ea_pp);
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
            sw[i - 2] += vpm - v;
            if constexpr (CHECK) se[i - 2] += vepm - ve;
          }
          vpm = v;
          if constexpr (CHECK) vepm = ve;
        }
        wa_pp = wa;
        wj_pp = wj;
        if constexpr (CHECK) { ea_pp = ea; ej_pp = ej; }
      }
      v_pm = vpm;
      wj_p = wj_pp;
      wa_p = wa_pp;
      if constexpr (CHECK) { ve_pm = vepm; ej_p = ej_pp; ea_p = ea_pp; }
      wj_first = wj_0;
      v_second = v_0;
      if constexpr (CHECK) { ej_first = ej_0; ve_second = ve_0; }
      // member 1's first chunk hands its first terms to member 0's last chunk
      if (m == 1 && g == 0) {
        P[L::WJ + c] = wj_0;
        P[L::VN + c] = v_0;
        if constexpr (CHECK) { P[L::EJ + c] = ej_0; P[L::VEN + c] = ve_0; }
      }
    }
  }

  // The transposed acceleration/jerk terms of the chunk's last two steps, which need
  // the next chunk's first terms (wj_n, v_n; ej_n, ve_n on check iterations).
  template <bool CHECK>
  __device__ __forceinline__ void close_chunk(float wj_n, float v_n, float ej_n, float ve_n) {
    const float v_last = fmaf(cJ, wj_p - wj_n, wa_p);
    sw[HP - 2] += v_pm - v_last;
    sw[HP - 1] += v_last - v_n;
    if constexpr (CHECK) {
      const float ve_last = fmaf(cJ, ej_p - ej_n, ea_p);
      se[HP - 2] += ve_pm - ve_last;
      se[HP - 1] += ve_last - ve_n;
    }
  }

  // d = (x~ - x) + rho (C^T w), with the higher chunks' position sums; dual residual on
  // check iterations (step 1 excluded: absorbed by x_1 = v0).
  template <bool CHECK>
  __device__ __forceinline__ void defect(float w_more, float e_more) {
    if constexpr (CHECK) rdm = 0.0f;
    const float offw = suffix_sum(sfw) + w_more;
    float offe = 0.0f;
    if constexpr (CHECK) offe = suffix_sum(sfe) + e_more;
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      const float d = fmaf(rho, sw[i] + offw, xt[i * 64 + lane] - X(i));
      sw[i] = d;
      if constexpr (CHECK) {
        float r = fabsf(fmaf(rho, se[i] + offe, -d));
        r = mask(i, r);
        if (i == 0) r = (m == 0 && g == 0) ? 0.0f : r;
        rdm = fmaxf(rdm, r);
      }
    }
  }

  // x += K d for this member's rows: own defect from registers, the partner's from LDS.
  __device__ __forceinline__ void gemm_f32(const float* __restrict__ kf) {
    float pd[HP];
    const float* dp = P + L::D + (1 - m) * HP * 64 + lane;
#pragma unroll
    for (int j = 0; j < HP; ++j) pd[j] = dp[j * 64];
    __asm__ volatile("" ::: "memory");
    const v4f* k4 = reinterpret_cast<const v4f*>(kf) + lane;
    constexpr int total = NB * 2 * NJ4;
    constexpr int ahead = 2;
    v4f f[ahead + 1];
    f[0] = k4[0];
    if (total > 1) f[1] = k4[64];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int jj = 0; jj < NJ4; ++jj) {
          const int idx = (b * 2 + s) * NJ4 + jj;
          if (idx + ahead < total) f[(idx + ahead) % (ahead + 1)] = k4[(idx + ahead) * 64];
          const v4f a = f[idx % (ahead + 1)];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int j = 4 * jj + e;
            if (j < HP)
              xb[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], s == 0 ? sw[j] : pd[j], xb[b], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
  }

  __device__ __forceinline__ void gemm_16(const void* __restrict__ kl) {
    using VT = typename std::conditional<GEMM == GEMM_BF16, v8bf, v8h>::type;
    using ST = typename std::conditional<GEMM == GEMM_BF16, __bf16, _Float16>::type;
    VT dv[2][NJ8];
    const float* dp = P + L::D + (1 - m) * HP * 64 + lane;
#pragma unroll
    for (int jj = 0; jj < NJ8; ++jj)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = 8 * jj + e;
        dv[0][jj][e] = (j < HP) ? (ST)sw[j] : (ST)0.0f;
        dv[1][jj][e] = (j < HP) ? (ST)dp[j * 64] : (ST)0.0f;
      }
    __asm__ volatile("" ::: "memory");
    const v4u* k16 = reinterpret_cast<const v4u*>(kl) + lane;
    constexpr int NT = NB * 2 * NJ8;
    constexpr int kDepth = NT < 4 ? NT : 4;
    v4u ring[kDepth];
#pragma unroll
    for (int t = 0; t < kDepth; ++t) ring[t] = k16[t * 64];
#pragma unroll
    for (int idx = 0; idx < NT; ++idx) {
      const int b = idx / (2 * NJ8), s = (idx / NJ8) % 2, jj = idx % NJ8;
      const v4u a = ring[idx % kDepth];
      if (idx + kDepth < NT) ring[idx % kDepth] = k16[(idx + kDepth) * 64];
      if constexpr (GEMM == GEMM_BF16)
        xb[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), dv[s][jj], xb[b], 0, 0, 0);
      else
        xb[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), dv[s][jj], xb[b], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // q <- c C x + q for every row of this member (cold start with relaxation).
  __device__ __forceinline__ void prep_q(float cf, float t0, float xl, float al) {
    float acc = 0.0f;
#pragma unroll
    for (int i = 0; i < HP; ++i) { acc += X(i); sw[i] = acc; }
    const float off = excl_prefix(acc) + t0;
    float xprev = lane_read(X(HP - 1), a_prev);
    float aprev = lane_read(X(HP - 1) - X(HP - 2), a_prev);
    xprev = (g == 0) ? (m == 0 ? v0 : xl) : xprev;
    aprev = (g == 0) ? (m == 0 ? 0.0f : al) : aprev;
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      const float sa = X(i) - xprev;
      const float sj = sa - aprev;
      xprev = X(i);
      aprev = sa;
      qv[i] = fmaf(cf, X(i), qv[i]);
      qq[i] = fmaf(cf, sw[i] + off, qq[i]);
      qa[i] = fmaf(cf, sa, qa[i]);
      qj[i] = fmaf(cf, sj, qj[i]);
    }
  }

  // One iteration's rows, hand-overs and defect. Returns false if a wait timed out.
  // On check iterations res_out gets the tile's max(r_p, r_d) over valid columns and the
  // per-column values (rp_c, rd_c, bad_c) for the store.
  template <bool CHECK>
  __device__ __forceinline__ bool step(int& seq0, int& seq1, bool col_ok, bool prep, float& res_out,
                                       float& rp_c, float& rd_c, int& bad_c) {
    float t0 = 0.0f, xl = 0.0f, al = 0.0f;
    int badl = 0;
    if constexpr (CHECK) {
#pragma unroll
      for (int i = 0; i < HP; ++i) badl |= (X(i) != X(i)) ? 1 : 0;
    }
    // S1: member 0's sums and boundary values
    if (m == 0) {
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < HP; ++i) acc += X(i);
      const float tot = member_sum(acc);
      if (g == 0) P[L::T0 + c] = tot;
      if (g == 3) {
        P[L::XL + c] = X(HP - 1);
        P[L::AL + c] = X(HP - 1) - X(HP - 2);
      }
      pair_signal(Pi + L::FLAG0, ++seq0);
    } else {
      if (!pair_wait(Pi + L::FLAG0, ++seq0)) return false;
      t0 = P[L::T0 + c];
      xl = P[L::XL + c];
      al = P[L::AL + c];
    }
    if (prep) prep_q(oma, t0, xl, al);
    rows<CHECK>(t0, xl, al);
    float rp_own = 0.0f, rd_own = 0.0f;
    if (m == 1) {
      // member 1's last chunk has no successor
      const float z = 0.0f;
      close_chunk<CHECK>(g == 3 ? z : wj_nr, g == 3 ? z : v_nr, g == 3 ? z : ej_nr,
                         g == 3 ? z : ve_nr);
      defect<CHECK>(0.0f, 0.0f);
#pragma unroll
      for (int j = 0; j < HP; ++j) P[L::D + HP * 64 + j * 64 + lane] = sw[j];
      if constexpr (CHECK) {
        rp_own = member_max(rpm);
        rd_own = member_max(rdm);
        const int bm = (badl | __shfl_xor(badl, 16, 64) | __shfl_xor(badl, 32, 64));
        if (g == 0) {
          P[L::RP + 16 + c] = rp_own;
          P[L::RD + 16 + c] = rd_own;
          Pi[L::BAD + 16 + c] = bm;
        }
        badl = bm;
      }
      pair_signal(Pi + L::FLAG1, ++seq1);
      // S3: member 0's defect (read in the GEMM) and residuals
      if (!pair_wait(Pi + L::FLAG0, ++seq0)) return false;
    } else {
      if (!pair_wait(Pi + L::FLAG1, ++seq1)) return false;
      const float wjn = (g == 3) ? P[L::WJ + c] : wj_nr;
      const float vn = (g == 3) ? P[L::VN + c] : v_nr;
      float ejn = 0.0f, ven = 0.0f, e_more = 0.0f;
      if constexpr (CHECK) {
        ejn = (g == 3) ? P[L::EJ + c] : ej_nr;
        ven = (g == 3) ? P[L::VEN + c] : ve_nr;
        e_more = P[L::W1E + c];
      }
      close_chunk<CHECK>(wjn, vn, ejn, ven);
      defect<CHECK>(P[L::W1 + c], e_more);
#pragma unroll
      for (int j = 0; j < HP; ++j) P[L::D + j * 64 + lane] = sw[j];
      if constexpr (CHECK) {
        rp_own = member_max(rpm);
        rd_own = member_max(rdm);
        const int bm = (badl | __shfl_xor(badl, 16, 64) | __shfl_xor(badl, 32, 64));
        if (g == 0) {
          P[L::RP + c] = rp_own;
          P[L::RD + c] = rd_own;
          Pi[L::BAD + c] = bm;
        }
        badl = bm;
      }
      pair_signal(Pi + L::FLAG0, ++seq0);
    }
    if constexpr (CHECK) {
      const int o = (1 - m) * 16 + c;
      rp_c = fmaxf(rp_own, P[L::RP + o]);
      rd_c = fmaxf(rd_own, P[L::RD + o]);
      bad_c = badl | Pi[L::BAD + o];
      // uniform stop test up to HP = 7; at HP = 13 the scalar registers it frees are not
      // worth the vector registers it costs there (256 with 13 spilled)
      const float rmax = col_ok ? fmaxf(rp_c, rd_c) : 0.0f;
      if constexpr (HP <= 7) res_out = pair_wave_max(rmax);
      else res_out = wave_max(rmax);
    }
    return true;
  }

  // Projects one tile; false if a hand-over timed out (the tile's residuals are NaN
  // and the pair must stop: its hand-over counters no longer match).
  __device__ bool run(const SolveKernelArgs& A, int j, int s0, const float* __restrict__ kf32,
                      const void* __restrict__ k16, int& seq0, int& seq1) {
    lane = threadIdx.x & 63;
    g = lane >> 4;
    c = lane & 15;
    a_prev = ((lane - 16) & 63) << 2;
    a_next = ((lane + 16) & 63) << 2;
    a_prev2 = ((lane - 32) & 63) << 2;
    a_next2 = ((lane + 32) & 63) << 2;
    xt = P + L::XT + m * HP * 64;
    const int H = A.H, nj = A.nj;
    const int G = 4 * m + g;                       // chunk
    const int s = s0 + c;
    const bool col_ok = s < A.N;
    const int s_ld = col_ok ? s : A.N - 1;
    {
      const int nv = H - G * HP;
      nvalid = nv < 0 ? 0 : (nv > HP ? HP : nv);
    }
    const JointRowParams& jp = A.jp[j];
    lbV = jp.lb[0]; ubV = jp.ub[0];
    lbQ = jp.lb[1]; ubQ = jp.ub[1];
    lbA = jp.lb[2]; ubA = jp.ub[2];
    lbJ = jp.lb[3]; ubJ = jp.ub[3];
    lbJ0 = (m == 0 && g == 0) ? fminf(lbJ, 0.0f) : lbJ;
    ubJ0 = (m == 0 && g == 0) ? fmaxf(ubJ, 0.0f) : ubJ;
    v0 = jp.v0;
    rho = A.rho;
    alpha = A.alpha;
    oma = 1.0f - A.alpha;
    cV = A.cV;
    cQ = A.cQ;
    cJ = A.cJ;

    // ---- load this member's rows of the sample (rows past H read row 0 and are zeroed)
    const size_t colbase = (size_t)s_ld * H * nj + j;
    const size_t chunk = (size_t)(G * HP) * nj;
    {
      const float* px = opaque(A.xin + colbase + chunk);
#pragma unroll
      for (int i = 0; i < 4 * NB; ++i) {
        float v = 0.0f;
        if (i < HP) {
          if (i < kMaskFrom) {
            v = px[i * nj];
          } else {
            const int r = (i < nvalid) ? i : -G * HP;
            v = px[r * nj];
            v = (i < nvalid) ? v : 0.0f;
          }
          xt[i * 64 + lane] = v;
        }
        xb[i >> 2][i & 3] = v;
      }
    }
    if (m == 0 && g == 0) xb[0][0] = v0;           // x_1 = v0 (eq. (A_b_def))
#pragma unroll
    for (int i = 0; i < HP; ++i) { qv[i] = 0.0f; qq[i] = 0.0f; qa[i] = 0.0f; qj[i] = 0.0f; }

    const bool tolmode = A.tolmode != 0;
    const bool reduced = GEMM != GEMM_F32;
    const int iters = A.iters;
    const int ce = A.check_every;
    // reduced forms in residual mode, as in the one-wave tile: at the first check point
    // whose residual exceeds kReducedRise times the lowest before it both members
    // restart from the sample with a cold state in the FP32 form; after kReducedStall
    // iterations with no new lowest residual they go on in FP32 as after convergence
    const int f32_from = !reduced ? 0 : (tolmode ? INT_MAX : iters - A.tail);
    float rlow = __builtin_inff();
    int it_low = 0;
    bool f32p = !reduced;
    int it = 0;
    int tail_end = -1;
    bool prep = A.alpha != 1.0f;                   // cold start: q += (1 - alpha) C x0
    float rp_c = 0.0f, rd_c = 0.0f;
    int bad_c = 0;
    bool ok = true;
    for (;;) {
      const bool chk = it == 0 || it == iters ||
                       (tolmode && (it % ce == 0 || it == tail_end));
      float r = 0.0f;
      if (chk) ok = step<true>(seq0, seq1, col_ok, prep, r, rp_c, rd_c, bad_c);
      else ok = step<false>(seq0, seq1, col_ok, prep, r, rp_c, rd_c, bad_c);
      prep = false;
      if (!ok) break;
      if (chk && tolmode) {
        if (r <= A.tol) {
          if (A.tail <= 0 || (f32p && it >= tail_end)) break;
          if (!f32p) {
            f32p = true;
            tail_end = it + A.tail;
          }
        } else if (it == tail_end) {
          tail_end = -1;
        }
        if constexpr (GEMM != GEMM_F32) {
          const float ru = __builtin_bit_cast(
              float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, r)));
          if (!f32p && it < iters) {
            if (ru > kReducedRise * rlow) {
#pragma unroll
              for (int i = 0; i < 4 * NB; ++i) xb[i >> 2][i & 3] = (i < HP) ? xt[i * 64 + lane] : 0.0f;
              if (m == 0 && g == 0) xb[0][0] = v0;
#pragma unroll
              for (int i = 0; i < HP; ++i) { qv[i] = 0.0f; qq[i] = 0.0f; qa[i] = 0.0f; qj[i] = 0.0f; }
              prep = A.alpha != 1.0f;
              f32p = true;
              tail_end = -1;
              continue;   // both members take this branch: the same tile residual
            }
            if (ru < rlow) {
              rlow = ru;
              it_low = it;
            } else if (it - it_low >= kReducedStall) {
              f32p = true;
              tail_end = it + A.tail;
            }
          }
        }
      }
      if (it == iters) break;
      if constexpr (GEMM == GEMM_F32) {
        gemm_f32(kf32);
      } else {
        if (f32p || it >= f32_from) gemm_f32(kf32);
        else gemm_16(k16);
      }
      ++it;
    }

    // ---- store this member's rows, then the column outputs (member 0, lane group 0)
    {
      float* po = opaque(col_ok ? A.xout + colbase + chunk : g_store_sink);
      const int st = col_ok ? nj : 0;
#pragma unroll
      for (int i = 0; i < HP; ++i) {
        float* dst = po + i * st;
        if (i >= kMaskFrom) dst = (i < nvalid) ? dst : g_store_sink;
        *dst = X(i);
      }
    }
    if (!ok || bad_c) {
      rp_c = __builtin_nanf("");
      rd_c = __builtin_nanf("");
    }
    if (m == 0 && g == 0 && col_ok) {
      const size_t o = (size_t)s * nj + j;
      if (A.rp) A.rp[o] = rp_c;
      if (A.rd) A.rd[o] = rd_c;
      if (A.itout) A.itout[o] = it;
    }
    return ok;
  }
};

// Persistent pair kernel: eight waves (four pairs) stage the pair-layout factor in LDS
// once; each pair takes tiles from the XCD queues as the one-wave kernel does (member 0
// takes the tile and hands it to member 1) until none are left.
template <int HP, int GEMM>
__device__ __forceinline__ void pair_body(const SolveKernelArgs& A) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  using L = PairLds<HP>;
  const int frag_bytes = A.frag_f32_bytes + (GEMM == GEMM_F32 ? 0 : A.frag_16_bytes);
  {
    const v4u* src = reinterpret_cast<const v4u*>(A.frag);
    v4u* dst = reinterpret_cast<v4u*>(lds);
    for (int i = threadIdx.x; i < frag_bytes / 16; i += blockDim.x) dst[i] = src[i];
  }
  // the wave index is uniform: readfirstlane lets the compiler branch on it with scalar
  // control flow instead of execution masks
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int pair = wave >> 1;
  const int m = wave & 1;
  float* P = reinterpret_cast<float*>(lds + frag_bytes) + pair * L::WORDS;
  int* Pi = reinterpret_cast<int*>(P);
  if (m == 0 && lane == 0) {
    Pi[L::FLAG0] = 0;
    Pi[L::FLAG1] = 0;
  }
  __syncthreads();
  // member m's fragments: FP32 region m, then (reduced forms) 16-bit region m
  const float* kf32 = reinterpret_cast<const float*>(lds) + (size_t)m * (A.frag_f32_bytes / 8);
  const void* k16 = lds + A.frag_f32_bytes + (size_t)m * (A.frag_16_bytes / 2);
  int seq0 = 0, seq1 = 0;
  const int nblk = (A.N + kTileCols - 1) / kTileCols;
  int x = blockIdx.x & (kXcdQueues - 1);
  int probed = 0;
  for (;;) {
    int tile = -1, queue = 0;
    if (m == 0) {
      while (probed < kXcdQueues) {
        const int in_queue = (nblk > x ? (nblk - x + kXcdQueues - 1) / kXcdQueues : 0) * A.nj;
        int i = 0;
        if (lane == 0) i = atomicAdd(A.counter + x, 1);
        i = __builtin_amdgcn_readfirstlane(i);
        if (i < in_queue) {
          tile = i;
          queue = x;
          break;
        }
        ++probed;
        x = (x + 1) & (kXcdQueues - 1);
      }
      if (lane == 0) {
        Pi[L::TILE] = tile;
        Pi[L::QUEUE] = queue;
      }
      pair_signal(Pi + L::FLAG0, ++seq0);
    } else {
      if (!pair_wait(Pi + L::FLAG0, ++seq0)) return;
      tile = __builtin_amdgcn_readfirstlane(Pi[L::TILE]);
      queue = __builtin_amdgcn_readfirstlane(Pi[L::QUEUE]);
    }
    if (tile < 0) return;
    const int j = tile % A.nj;
    const int sb = queue + kXcdQueues * (tile / A.nj);
    PairSolver<HP, GEMM> ps;
    ps.m = m;
    ps.P = P;
    ps.Pi = Pi;
    if (!ps.run(A, j, sb * kTileCols, kf32, k16, seq0, seq1)) return;
  }
}

template <int HP, int GEMM>
__global__ __launch_bounds__(kPairWaves * 64) __attribute__((amdgpu_waves_per_eu(2))) void
admm_pair_kernel(SolveKernelArgs A) {
  pair_body<HP, GEMM>(A);
}

}  // namespace prism

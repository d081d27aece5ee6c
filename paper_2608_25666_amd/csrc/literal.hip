// The Bregman iteration exactly as Sec. III-D prints it (eqs. (admm_zeta),
// (admm_primal)/(admm_KKT), (admm_dual)), on the GPU in FP64 (declared in
// include/prism_proj.h as prism_proj_literal).
//
// This is NOT the projection. The multiplier lives in the primal space and the
// slack step does not see it, so every feasible x with lambda = x - x~ is a
// fixed point: a fixed number of passes heads for a feasible trajectory near the
// sample, not the nearest one. It is the fast mode behind the paper's remark that
// ten to twenty iterations suffice (Sec. III-D "Convergence").
//
// Printed steps, with G = [C; -C] and h in the paper's physical row scaling and
// penalty delta:
//   zeta'  = max(0, h - G x)
//   x'     : (I + delta G^T G) x' + A^T mu = x~ + lambda + delta G^T (h - zeta'),  A x' = b
//   lambda' = lambda - (delta/2) G^T (G x' - h + zeta')
// Here rows are carried in the velocity units of the projection kernel (row
// block b scaled by S_b = 1, 1/dt, dt, dt^2 for velocity, position,
// acceleration, jerk), with W = S^-2 = diag(1, dt^2, dt^-2, dt^-4) per block and
// s = C x - c the affine row values (c: the v0 terms of the first acceleration
// and jerk rows). Writing both bound rows of G out gives, exactly,
//   G^T (h - zeta') = C^T W (m + 2c),      m = min(ub, s) + max(lb, s),
//   G^T G           = 2 C^T W C,
//   G^T (G x' - h + zeta') = C^T W (2 s' - m),
// so with w = lambda + x~ (x~ only ever enters through this sum) Steps 1 and 2 are
//   u  = C^T W m(x),  rhs = w + delta u + 2 delta C^T W c,  x' = K rhs + k v0,
// where x' = K r + k v0 solves the equality-constrained system with
// P = I + 2 delta C^T W C (the projection's factor with rho = 2 delta and block
// weights W). C^T W c is nonzero only at steps 1 and 2 (1-based); step 1 of
// rhs is absorbed by the equality multiplier, leaving -2 delta W_J v0 at step 2.
// K's column of step 1 is zero (the step is pinned), so it carries k instead and
// rhs_1 is set to v0: x' = K rhs + k v0 is one product.
// Step 3 is then w' = w + (delta/2) u - delta C^T W s(x'); since x' solves
// P x' + e_1 mu = rhs, delta C^T W C x' = (rhs - x' - e_1 mu) / 2, and Step 3
// reduces exactly to w' = (w + x') / 2 on steps 2..H, which the kernel uses.
//
// Layout: one wave per tile of 16 columns (samples s0..s0+15 of one joint);
// lane l = 16 g + c holds steps g*HQ .. g*HQ+HQ-1 of column c. K sits in LDS as
// v_mfma_f64_16x16x4_f64 A-operand fragments whose rows follow that
// instruction's accumulator (row g + 4e of a block in item e of lane group g),
// so x' = K rhs runs on the matrix cores with rhs and x' in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "factor.h"
#include "prism_internal.h"
#include "prism_proj.h"

namespace prism {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int kLitWaves = 4;       // tiles (waves) per workgroup, sharing K in LDS
constexpr int kLitMinHQ = 2;       // at least two steps per lane group
constexpr int kLitMaxHQ = 32;      // H <= 128
constexpr int kLitMaxFactors = 64; // distinct penalties kept per handle

int literal_hq(int H) { return std::max(kLitMinHQ, (H + 3) / 4); }

struct LitJoint {
  double lbQ, ubQ;   // position rows in velocity units: (q_min - q0) / dt, (q_max - q0) / dt
  double v0, q0;
};

struct LitArgs {
  const float* xin;     // [N][H][nj]
  const float* xinit;   // [N][H][nj] or null (start from the samples)
  float* xout;          // [N][H][nj]
  double* viol;         // [N][nj] or null
  const double* frag;   // layout_f64 fragments (k in the column of step 1)
  const double* bnd;    // physical bounds [8][nj]
  int N, H, nj, iters, ntiles;
  double delta, dt;
  LitJoint jp[kMaxJoints];
};

__device__ __forceinline__ double lane_read_d(double v, int byte_addr) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(unsigned)u);
  const int hi = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(unsigned)(u >> 32));
  return __longlong_as_double(
      (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo));
}

template <int HQ>
struct LitTile {
  static constexpr int NB = (HQ + 3) / 4;   // 16-row output blocks
  static constexpr int NJ2 = (HQ + 1) / 2;  // pairs of k-steps per fragment load

  v4d xb[NB];     // x (MFMA accumulator), item 4b + e = step g*HQ + 4b + e
  double w[HQ];   // lambda + x~
  double r[HQ];   // right-hand side / transposed row sums

  int g, nvalid;
  int a_prev, a_next, a_far;   // ds_bpermute addresses of lanes l-16, l+16, l+32
  double lb[4], ub[4];
  double v0, wQ, wA, wJ;

  __device__ __forceinline__ double X(int i) const { return xb[i >> 2][i & 3]; }
  // Steps past the horizon sit only in the last three registers of the last lane
  // group once HQ = ceil(H/4) >= 3; with the minimum HQ = 2 whole groups may lie past it.
  __device__ __forceinline__ bool valid(int i) const {
    if (HQ > 2 && i < HQ - 3) return true;
    return i < nvalid;
  }

  __device__ __forceinline__ double excl_prefix(double T) const {   // lower chunks
    const double a = lane_read_d(T, a_prev);
    const double b = lane_read_d(T, a_far);
    const double c = lane_read_d(T, a_next);   // chunk g-3 = g+1 (mod 4)
    return (g >= 1 ? a : 0.0) + ((g >= 2 ? b : 0.0) + (g >= 3 ? c : 0.0));
  }
  __device__ __forceinline__ double excl_suffix(double T) const {   // higher chunks
    const double a = lane_read_d(T, a_next);
    const double b = lane_read_d(T, a_far);
    const double c = lane_read_d(T, a_prev);   // chunk g+3 = g-1 (mod 4)
    return (g <= 2 ? a : 0.0) + ((g <= 1 ? b : 0.0) + (g == 0 ? c : 0.0));
  }

  template <bool CLIP>
  __device__ __forceinline__ double rowval(double s, int b) const {
    if (CLIP) return fmin(ub[b], s) + fmax(lb[b], s);
    return s;
  }

  // out = C^T W m over this chunk's steps, m per row = min(ub, s) + max(lb, s)
  // (CLIP) or s, rows taken at the current x. Transposes: velocity rows map to
  // their own step, position rows to every earlier step (suffix sums), the
  // acceleration row of step k to steps k and k-1, the jerk row to k, k-1, k-2.
  template <bool CLIP>
  __device__ __forceinline__ void transpose_rows(double (&out)[HQ]) const {
    double T = 0.0;
#pragma unroll
    for (int i = 0; i < HQ; ++i) T += X(i);
    double P = excl_prefix(T);
    const double xl = lane_read_d(X(HQ - 1), a_prev);
    const double al = lane_read_d(X(HQ - 1) - X(HQ - 2), a_prev);
    double xp = g == 0 ? v0 : xl;
    double ap = g == 0 ? 0.0 : al;
    double mq = 0.0;                        // position rows of this chunk so far
    double send1 = 0.0, send2 = 0.0;        // owed to the previous chunk's last two steps
#pragma unroll
    for (int i = 0; i < HQ; ++i) {
      const double x = X(i);
      P += x;
      const double sA = x - xp;
      const double sJ = sA - ap;
      xp = x;
      ap = sA;
      const bool ok = valid(i);
      const bool okJ = ok && (g > 0 || i > 0);
      const double mV = ok ? rowval<CLIP>(x, 0) : 0.0;
      const double mQ = ok ? rowval<CLIP>(P, 1) : 0.0;
      const double mA = ok ? rowval<CLIP>(sA, 2) : 0.0;
      const double mJ = okJ ? rowval<CLIP>(sJ, 3) : 0.0;
      out[i] = mV + wA * mA + wJ * mJ - wQ * mq;
      mq += mQ;
      const double b1 = -(wA * mA + 2.0 * wJ * mJ);   // to step i-1
      const double b2 = wJ * mJ;                       // to step i-2
      if (i >= 1) out[i - 1] += b1;
      else send1 += b1;
      if (i >= 2) out[i - 2] += b2;
      else if (i == 1) send1 += b2;
      else send2 += b2;
    }
    const double Sq = excl_suffix(mq);
    const double r1 = lane_read_d(send1, a_next);
    const double r2 = lane_read_d(send2, a_next);
    const double add = wQ * (mq + Sq);
#pragma unroll
    for (int i = 0; i < HQ; ++i) out[i] += add;
    out[HQ - 1] += g <= 2 ? r1 : 0.0;
    out[HQ - 2] += g <= 2 ? r2 : 0.0;
#pragma unroll
    for (int i = 0; i < HQ; ++i) out[i] = valid(i) ? out[i] : 0.0;
  }
};

// Waves per SIMD asked of the register allocator: as many as the registers allow
// without spills; above HQ = 24 the K fragments (over 80 KB of LDS) leave room
// for one workgroup per CU anyway.
constexpr int literal_waves_per_simd(int HQ) {
  return HQ <= 9 ? 4 : HQ <= 16 ? 3 : HQ <= 24 ? 2 : 1;
}

template <int HQ>
__global__ __launch_bounds__(64 * kLitWaves, literal_waves_per_simd(HQ)) void literal_kernel(
    LitArgs A) {
  using T = LitTile<HQ>;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  double* lds = reinterpret_cast<double*>(lds_raw);
  constexpr int ntot2 = T::NB * T::NJ2 * 64;
  for (int i = threadIdx.x; i < ntot2; i += 64 * kLitWaves)
    reinterpret_cast<v2d*>(lds)[i] = reinterpret_cast<const v2d*>(A.frag)[i];
  __syncthreads();

  // workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // run of tiles so that the joints of one sample block share an L2
  const int G = gridDim.x, B = blockIdx.x, xcd = B & 7;
  const int L = xcd * (G >> 3) + min(xcd, G & 7) + (B >> 3);
  // wave-uniform: the joint's bounds and weights then live in scalar registers
  const int tile = __builtin_amdgcn_readfirstlane(L * kLitWaves + (int)(threadIdx.x >> 6));
  if (tile >= A.ntiles) return;
  const int j = tile % A.nj;
  const int s0 = (tile / A.nj) * 16;

  T S;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15;
  S.g = lane >> 4;
  S.nvalid = min(max(A.H - S.g * HQ, 0), HQ);
  S.a_prev = ((lane + 48) & 63) << 2;
  S.a_next = ((lane + 16) & 63) << 2;
  S.a_far = ((lane + 32) & 63) << 2;
  const int nj = A.nj;
  const double dt = A.dt;
  S.lb[0] = A.bnd[2 * nj + j];
  S.ub[0] = A.bnd[3 * nj + j];
  S.lb[1] = A.jp[j].lbQ;
  S.ub[1] = A.jp[j].ubQ;
  S.lb[2] = A.bnd[4 * nj + j] * dt;
  S.ub[2] = A.bnd[5 * nj + j] * dt;
  S.lb[3] = A.bnd[6 * nj + j] * dt * dt;
  S.ub[3] = A.bnd[7 * nj + j] * dt * dt;
  S.v0 = A.jp[j].v0;
  S.wQ = dt * dt;
  S.wA = 1.0 / (dt * dt);
  S.wJ = S.wA * S.wA;
  const double delta = A.delta;

  const int s = s0 + c;
  const bool col = s < A.N;
  const size_t base = (size_t)(col ? s : 0) * A.H * nj + j;
  const int k0 = S.g * HQ;
#pragma unroll
  for (int i = 0; i < HQ; ++i) {
    const bool ok = col && S.valid(i);
    const size_t at = base + (size_t)(k0 + i) * nj;
    const double xt = ok ? (double)A.xin[at] : 0.0;
    S.w[i] = xt;   // lambda_0 = 0
    S.xb[i >> 2][i & 3] = ok ? (A.xinit ? (double)A.xinit[at] : xt) : 0.0;
  }
#pragma unroll
  for (int i = HQ; i < 4 * T::NB; ++i) S.xb[i >> 2][i & 3] = 0.0;
  if (S.g == 0) S.xb[0][0] = S.v0;   // x_1 = v0 (eq. (A_b_def))

  const v2d* kf = reinterpret_cast<const v2d*>(lds) + lane;
  for (int it = 0; it < A.iters; ++it) {
    // Steps 1 and 2: slack from x, right-hand side, primal solve
    S.template transpose_rows<true>(S.r);
#pragma unroll
    for (int i = 0; i < HQ; ++i) S.r[i] = S.w[i] + delta * S.r[i];
    if (S.g == 0) {
      S.r[1] -= 2.0 * delta * S.wJ * S.v0;
      S.r[0] = S.v0;   // step 1's entry is absorbed by the equality; K carries k there
    }
#pragma unroll
    for (int b = 0; b < T::NB; ++b) S.xb[b] = v4d{0.0, 0.0, 0.0, 0.0};
    // fragments stream from LDS one pair ahead; the barriers keep the scheduler
    // from hoisting all of K into registers
    __asm__ volatile("" ::: "memory");
    v2d a = kf[0];
#pragma unroll
    for (int b = 0; b < T::NB; ++b) {
#pragma unroll
      for (int jp = 0; jp < T::NJ2; ++jp) {
        const int idx = b * T::NJ2 + jp;
        v2d an = a;
        if (idx + 1 < T::NB * T::NJ2) an = kf[(idx + 1) * 64];
        S.xb[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], S.r[2 * jp], S.xb[b], 0, 0, 0);
        if (2 * jp + 1 < HQ)
          S.xb[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], S.r[2 * jp + 1], S.xb[b], 0, 0, 0);
        a = an;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // Step 3: lambda' = lambda - (delta/2) G^T (G x' - h + zeta') equals
    // (lambda + x' - x~) / 2 on every free step because x' solves Step 2's system;
    // in w = lambda + x~ that is w' = (w + x') / 2 (step 1 of w is never read)
#pragma unroll
    for (int i = 0; i < HQ; ++i) S.w[i] = 0.5 * (S.w[i] + S.X(i));
  }

  // largest bound violation of the returned iterate, physical units
  double T0 = 0.0;
#pragma unroll
  for (int i = 0; i < HQ; ++i) T0 += S.X(i);
  double P = S.excl_prefix(T0);
  const double xl = lane_read_d(S.X(HQ - 1), S.a_prev);
  const double al = lane_read_d(S.X(HQ - 1) - S.X(HQ - 2), S.a_prev);
  double xp = S.g == 0 ? S.v0 : xl;
  double ap = S.g == 0 ? 0.0 : al;
  const double q0 = A.jp[j].q0;
  const double qmin = A.bnd[j], qmax = A.bnd[nj + j];
  const double vmin = A.bnd[2 * nj + j], vmax = A.bnd[3 * nj + j];
  const double amin = A.bnd[4 * nj + j], amax = A.bnd[5 * nj + j];
  const double jmin = A.bnd[6 * nj + j], jmax = A.bnd[7 * nj + j];
  double worst = 0.0;
#pragma unroll
  for (int i = 0; i < HQ; ++i) {
    const double x = S.X(i);
    P += x;
    const double sA = x - xp;
    const double sJ = sA - ap;
    xp = x;
    ap = sA;
    if (S.valid(i)) {
      const double th = q0 + dt * P;
      const double ac = sA / dt;
      worst = fmax(worst, fmax(x - vmax, vmin - x));
      worst = fmax(worst, fmax(th - qmax, qmin - th));
      worst = fmax(worst, fmax(ac - amax, amin - ac));
      if (S.g > 0 || i > 0) {
        const double je = sJ / (dt * dt);
        worst = fmax(worst, fmax(je - jmax, jmin - je));
      }
    }
  }
  worst = fmax(worst, __shfl_xor(worst, 16));
  worst = fmax(worst, __shfl_xor(worst, 32));
  if (col) {
#pragma unroll
    for (int i = 0; i < HQ; ++i)
      if (S.valid(i)) A.xout[base + (size_t)(k0 + i) * nj] = (float)S.X(i);
    if (A.viol && S.g == 0) A.viol[(size_t)s * nj + j] = worst;
  }
}

typedef void (*LitKernelFn)(LitArgs);

template <int... I>
constexpr std::array<LitKernelFn, sizeof...(I)> literal_table(std::integer_sequence<int, I...>) {
  return {{&literal_kernel<I + kLitMinHQ>...}};
}

LitKernelFn pick_literal(int HQ) {
  static const auto table =
      literal_table(std::make_integer_sequence<int, kLitMaxHQ - kLitMinHQ + 1>{});
  if (HQ < kLitMinHQ || HQ > kLitMaxHQ) return nullptr;
  return table[HQ - kLitMinHQ];
}

size_t literal_values(int HQ) { return f64_frag_count(HQ); }

// Device copy of the printed iteration's factor for penalty delta, built on the
// first call with that delta and kept until the handle is destroyed.
prism_status_t literal_factor(prism_proj_s* p, double delta, const double** out) {
  std::lock_guard<std::mutex> lock(p->lit_mu);
  for (const auto& e : p->lit)
    if (e.first == delta) {
      *out = e.second;
      return PRISM_OK;
    }
  if ((int)p->lit.size() >= kLitMaxFactors) return PRISM_ENOMEM;
  const double dt = p->dt;
  const double w[4] = {1.0, dt * dt, 1.0 / (dt * dt), 1.0 / (dt * dt * dt * dt)};
  std::vector<double> K, k, host;
  if (!build_factor(p->H, 2.0 * delta, w, K, k)) return PRISM_EINVAL;
  const int HQ = literal_hq(p->H);
  layout_f64(K, k, p->H, HQ, host);
  double* d = nullptr;
  const size_t bytes = host.size() * sizeof(double);
  if (hipMalloc(&d, bytes) != hipSuccess) return PRISM_ENOMEM;
  if (hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return PRISM_EDEVICE;
  }
  p->lit.emplace_back(delta, d);
  *out = d;
  return PRISM_OK;
}

}  // namespace

void release_literal_factors(prism_proj_s* p) {
  std::lock_guard<std::mutex> lock(p->lit_mu);
  for (auto& e : p->lit) (void)hipFree(e.second);
  p->lit.clear();
}

}  // namespace prism

using namespace prism;

extern "C" {

prism_status_t prism_proj_literal(prism_proj_t p, const prism_literal_args_t* a,
                                  hipStream_t stream) {
  if (!p || !a) return PRISM_EINVAL;
  if (a->N < 0 || a->iters < 0 || !a->q0 || !a->v0) return PRISM_EINVAL;
  if (!std::isfinite(a->delta) || a->delta <= 0.0) return PRISM_EINVAL;
  JointRowParams check[kMaxJoints];
  prism_status_t st = fill_joint_params(p, a->q0, a->v0, check);
  if (st != PRISM_OK) return st;
  if (a->N == 0) return PRISM_OK;
  if (!a->v_samples || !a->v_out) return PRISM_EINVAL;
  if ((long long)a->N * p->H * p->nj > (1ll << 40)) return PRISM_EINVAL;
  const long long ntiles = (long long)((a->N + 15) / 16) * p->nj;
  if (ntiles > INT_MAX - kLitWaves) return PRISM_EINVAL;
  st = check_device(p);
  if (st != PRISM_OK) return st;
  const int HQ = literal_hq(p->H);
  LitKernelFn fn = pick_literal(HQ);
  if (!fn) return PRISM_EUNSUPPORTED;
  const double* frag = nullptr;
  st = literal_factor(p, a->delta, &frag);
  if (st != PRISM_OK) return st;

  LitArgs A{};
  A.xin = a->v_samples;
  A.xinit = a->x_init;
  A.xout = a->v_out;
  A.viol = a->violation;
  A.frag = frag;
  A.bnd = p->d_bounds;
  A.N = a->N;
  A.H = p->H;
  A.nj = p->nj;
  A.iters = a->iters;
  A.ntiles = (int)ntiles;
  A.delta = a->delta;
  A.dt = p->dt;
  for (int j = 0; j < p->nj; ++j) {
    const double qmin = p->bnd[0 * p->nj + j], qmax = p->bnd[1 * p->nj + j];
    A.jp[j].lbQ = (qmin - a->q0[j]) / p->dt;
    A.jp[j].ubQ = (qmax - a->q0[j]) / p->dt;
    A.jp[j].v0 = a->v0[j];
    A.jp[j].q0 = a->q0[j];
  }
  const int lds = (int)(literal_values(HQ) * sizeof(double));
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return PRISM_EDEVICE;
  const int grid = (int)((ntiles + kLitWaves - 1) / kLitWaves);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * kLitWaves), lds, stream, A);
  return hipGetLastError() == hipSuccess ? PRISM_OK : PRISM_EDEVICE;
}

}  // extern "C"

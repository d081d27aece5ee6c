// Launch arguments shared by the host library and the device kernels.
#pragma once

#include <cstdint>

namespace prism {

constexpr int kMaxJoints = 64;   // PRISM_MAX_JOINTS
constexpr int kWaves = 4;        // waves per workgroup
// Waves per workgroup of a single-solve launch. The reduced forms with chunks 22..25
// (H = 85..100) fit in 256 registers, but a four-wave workgroup's staged factor and
// samples (about 104 KB of LDS at chunk 25) leave room for one workgroup per CU; eight
// waves sharing one staged factor (about 129 KB) run two waves per SIMD instead.
constexpr int solve_waves(int HQ, bool reduced) { return (reduced && HQ >= 22 && HQ <= 25) ? 8 : kWaves; }
constexpr int kTileCols = 16;    // samples per tile (MFMA N dimension)
constexpr int kXcdQueues = 8;    // tile queues, one per XCD (MI355X has 8)
constexpr float kReducedRise = 64.0f;    // residual mode: a reduced-form tile whose residual
                                          // rises this far above its lowest restarts in FP32
constexpr int kReducedStall = 500;       // residual mode: a reduced-form tile with no new
                                          // lowest residual for this many iterations goes on
                                          // in FP32

enum GemmPrec : int { GEMM_F32 = 0, GEMM_BF16 = 1, GEMM_F16 = 2 };

// Row bounds of one joint in velocity units, in the kernel's affine form:
//   velocity  s = x_k                          in [v_min, v_max]
//   position  s = sum_{i<=k} x_i               in [(q_min-q0)/dt, (q_max-q0)/dt]
//   accel.    s = x_k - x_{k-1}, x_0 := v0     in [a_min dt, a_max dt]
//   jerk      s = a_k - a_{k-1}, a_1 := 0      in [j_min dt^2, j_max dt^2]
// (1-based steps; the kernel's jerk row of step 1 is identically zero and its
// bounds are widened to contain 0, so it is inert: jerk rows are steps 2..H).
struct JointRowParams {
  float lb[4];
  float ub[4];
  float v0;
  float q0;          // start position (used by the tracking cost)
  float pad[2];
};

// Samples drawn in the load instead of read: x~ = nu + sigma * z, z standard
// normal from Philox4x32-10 (counter: element index, stream; key: seed).
struct SampleGen {
  const float* nu;      // [H][nj]
  const float* sigma;   // [H][nj]
  float* xs_out;        // drawn samples [N][H][nj] or null
  unsigned seed_lo, seed_hi, stream_lo, stream_hi;
};

// Tracking cost of each projected column, written per (sample, joint).
struct CostArgs {
  const float* ref;     // theta_ref [H][nj]
  float* cost;          // [N][nj]
  float w_pos, w_vel, dt;
};

// What one tile needs to know about its request (single solve or batch entry).
struct TileArgs {
  const float* xin;
  float* xout;
  float* rp;
  float* rd;
  int* itout;
  const float* xw;
  const float* uw;
  float* uout;
  const JointRowParams* jp;   // n_joints entries
  float* xsave;               // second copy of x [N][H][nj] or null
  int N, H, nj, iters, check_every, tail, tolmode;
  int shift;                  // 1: warm x and q are read one step ahead (last step repeated)
  float rho, alpha, tol, cV, cQ, cJ;
  int gen_on, cost_on;        // sample in the load / cost in the epilogue
  SampleGen gen;
  CostArgs cost;
};

struct SolveKernelArgs {
  const float* xin;      // [N][H][nj]
  float* xout;           // [N][H][nj]
  float* rp;             // [N][nj] or null
  float* rd;             // [N][nj] or null
  int* itout;            // [N][nj] or null
  const float* xw;       // warm x [N][H][nj] or null
  const float* uw;       // warm dual state q [N][nj][4][H] or null
  float* uout;           // dual state q out [N][nj][4][H] or null
  const void* frag;      // FP32 fragments, then 16-bit fragments (reduced forms)
  int* counter;          // kXcdQueues tile-queue counters, zero at launch
  int N, H, nj, ntiles;
  int shift;             // warm state read one step ahead
  int gen_on, cost_on;
  SampleGen gen;
  CostArgs cost;
  int iters, check_every, tail, tolmode;
  float rho, alpha, tol;          // rho: penalty of the acceleration block (rho * w_A)
  float cV, cQ, cJ;               // block weights relative to the acceleration block
  int frag_f32_bytes, frag_16_bytes;
  JointRowParams jp[kMaxJoints];
};

// One request of a batched launch (device memory). Its sample blocks are dealt to
// kXcdQueues tile queues (block b to queue b mod kXcdQueues), as in a single solve.
struct BatchReq {
  TileArgs t;
  const void* frag;          // FP32 fragments, then 16-bit fragments
  int HQ;
  int frag_f32_bytes, frag_16_bytes;
  int nblk;                  // ceil(N / 16) sample blocks
  int wg_begin;              // first workgroup whose home is this request
};

struct BatchKernelArgs {
  const BatchReq* reqs;      // longest work first; wg_begin non-decreasing
  int n_req;
  int* counter;              // [n_req][kXcdQueues] tile-queue counters, zero at launch
  int xt_offset;             // LDS byte offset of the per-wave sample copies
  int hq_max;                // largest chunk size in this launch
};

struct FeasKernelArgs {
  const float* x;        // [N][H][nj]
  double* viol;          // [N][nj][5]
  const double* bounds;  // device [8][nj]: q_min, q_max, v_min, v_max, a_min, a_max, j_min, j_max
  int N, H, nj;
  double dt;
  double q0[kMaxJoints], v0[kMaxJoints];
};

}  // namespace prism

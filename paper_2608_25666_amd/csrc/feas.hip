// FP64 feasibility check of projected trajectories (one thread per column).
//
// Positions by forward-Euler integration from q0 (Sec. III-D eq. (pos_stack)),
// accelerations by backward differences with the velocity before step 1 equal
// to v0 (eq. (acc_stack)), jerks as differences of consecutive accelerations
// for steps 2..H (eq. (jerk_stack)), and the boundary equality x_1 = v0
// (eq. (A_b_def)). Writes the largest violation of each bound in its own unit.
#include <hip/hip_runtime.h>

#include "kernel_args.h"

namespace prism {

__global__ __launch_bounds__(256) void feasibility_kernel(FeasKernelArgs A) {
  const long col = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= (long)A.N * A.nj) return;
  const int j = (int)(col % A.nj);
  const long s = col / A.nj;
  const int nj = A.nj;
  const double qmin = A.bounds[0 * nj + j], qmax = A.bounds[1 * nj + j];
  const double vmin = A.bounds[2 * nj + j], vmax = A.bounds[3 * nj + j];
  const double amin = A.bounds[4 * nj + j], amax = A.bounds[5 * nj + j];
  const double jmin = A.bounds[6 * nj + j], jmax = A.bounds[7 * nj + j];
  const double dt = A.dt;
  const double v0 = A.v0[j];
  double q = A.q0[j], vprev = v0, aprev = 0.0;
  double vp = 0.0, vv = 0.0, va = 0.0, vj = 0.0;
  bool nan = false;
  const float* x = A.x + s * (long)A.H * nj + j;
  for (int k = 0; k < A.H; ++k) {
    const double v = (double)x[(long)k * nj];
    nan |= (v != v);
    q += dt * v;
    const double a = (v - vprev) / dt;
    vv = fmax(vv, fmax(v - vmax, vmin - v));
    vp = fmax(vp, fmax(q - qmax, qmin - q));
    va = fmax(va, fmax(a - amax, amin - a));
    if (k >= 1) {
      const double jk = (a - aprev) / dt;
      vj = fmax(vj, fmax(jk - jmax, jmin - jk));
    }
    vprev = v;
    aprev = a;
  }
  const double eq = fabs((double)x[0] - v0);
  double* o = A.viol + col * 5;
  const double nanv = __builtin_nan("");
  o[0] = nan ? nanv : fmax(vp, 0.0);
  o[1] = nan ? nanv : fmax(vv, 0.0);
  o[2] = nan ? nanv : fmax(va, 0.0);
  o[3] = nan ? nanv : fmax(vj, 0.0);
  o[4] = nan ? nanv : eq;
}

hipError_t launch_feasibility(const FeasKernelArgs& a, hipStream_t stream) {
  const long cols = (long)a.N * a.nj;
  const int blocks = (int)((cols + 255) / 256);
  hipLaunchKernelGGL(feasibility_kernel, dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace prism

// Instantiations of the persistent ADMM kernel: f16 x-update operands, chunk sizes 10..17.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_f16_1(int HQ, bool exact) {
  switch (HQ) {
    case 10: return exact ? (SolveKernelFn)admm_solve_kernel<10, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<10, false, GEMM_F16>;
    case 11: return exact ? (SolveKernelFn)admm_solve_kernel<11, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<11, false, GEMM_F16>;
    case 12: return exact ? (SolveKernelFn)admm_solve_kernel<12, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<12, false, GEMM_F16>;
    case 13: return exact ? (SolveKernelFn)admm_solve_kernel<13, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<13, false, GEMM_F16>;
    case 14: return exact ? (SolveKernelFn)admm_solve_kernel<14, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<14, false, GEMM_F16>;
    case 15: return exact ? (SolveKernelFn)admm_solve_kernel<15, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<15, false, GEMM_F16>;
    case 16: return exact ? (SolveKernelFn)admm_solve_kernel<16, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<16, false, GEMM_F16>;
    case 17: return exact ? (SolveKernelFn)admm_solve_kernel<17, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<17, false, GEMM_F16>;
    default: return nullptr;
  }
}

}  // namespace prism

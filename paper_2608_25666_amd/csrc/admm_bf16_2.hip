// Instantiations of the persistent ADMM kernel: bf16 x-update operands, chunk sizes 18..25.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_bf16_2(int HQ, bool exact) {
  switch (HQ) {
    case 18: return exact ? (SolveKernelFn)admm_solve_kernel<18, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<18, false, GEMM_BF16>;
    case 19: return exact ? (SolveKernelFn)admm_solve_kernel<19, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<19, false, GEMM_BF16>;
    case 20: return exact ? (SolveKernelFn)admm_solve_kernel<20, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<20, false, GEMM_BF16>;
    case 21: return exact ? (SolveKernelFn)admm_solve_kernel<21, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<21, false, GEMM_BF16>;
    case 22: return exact ? (SolveKernelFn)admm_solve_kernel<22, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<22, false, GEMM_BF16>;
    case 23: return exact ? (SolveKernelFn)admm_solve_kernel<23, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<23, false, GEMM_BF16>;
    case 24: return exact ? (SolveKernelFn)admm_solve_kernel<24, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<24, false, GEMM_BF16>;
    case 25: return exact ? (SolveKernelFn)admm_solve_kernel<25, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<25, false, GEMM_BF16>;
    default: return nullptr;
  }
}

}  // namespace prism

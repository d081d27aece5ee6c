// Instantiations of the persistent ADMM kernel: bf16 x-update operands, chunk sizes 26..32.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_bf16_3(int HQ, bool exact) {
  switch (HQ) {
    case 26: return exact ? (SolveKernelFn)admm_solve_kernel<26, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<26, false, GEMM_BF16>;
    case 27: return exact ? (SolveKernelFn)admm_solve_kernel<27, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<27, false, GEMM_BF16>;
    case 28: return exact ? (SolveKernelFn)admm_solve_kernel<28, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<28, false, GEMM_BF16>;
    case 29: return exact ? (SolveKernelFn)admm_solve_kernel<29, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<29, false, GEMM_BF16>;
    case 30: return exact ? (SolveKernelFn)admm_solve_kernel<30, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<30, false, GEMM_BF16>;
    case 31: return exact ? (SolveKernelFn)admm_solve_kernel<31, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<31, false, GEMM_BF16>;
    case 32: return exact ? (SolveKernelFn)admm_solve_kernel<32, true, GEMM_BF16> : (SolveKernelFn)admm_solve_kernel<32, false, GEMM_BF16>;
    default: return nullptr;
  }
}

}  // namespace prism

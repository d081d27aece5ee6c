// Instantiations of the persistent ADMM kernel: f16 x-update operands, chunk sizes 2..9.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_f16_0(int HQ, bool exact) {
  switch (HQ) {
    case 2: return exact ? (SolveKernelFn)admm_solve_kernel<2, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<2, false, GEMM_F16>;
    case 3: return exact ? (SolveKernelFn)admm_solve_kernel<3, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<3, false, GEMM_F16>;
    case 4: return exact ? (SolveKernelFn)admm_solve_kernel<4, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<4, false, GEMM_F16>;
    case 5: return exact ? (SolveKernelFn)admm_solve_kernel<5, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<5, false, GEMM_F16>;
    case 6: return exact ? (SolveKernelFn)admm_solve_kernel<6, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<6, false, GEMM_F16>;
    case 7: return exact ? (SolveKernelFn)admm_solve_kernel<7, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<7, false, GEMM_F16>;
    case 8: return exact ? (SolveKernelFn)admm_solve_kernel<8, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<8, false, GEMM_F16>;
    case 9: return exact ? (SolveKernelFn)admm_solve_kernel<9, true, GEMM_F16> : (SolveKernelFn)admm_solve_kernel<9, false, GEMM_F16>;
    default: return nullptr;
  }
}

}  // namespace prism

// Instantiations of the persistent ADMM kernel: bf16 x-update operands, chunk sizes 10..17.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_bf16_1(int HQ, bool exact) {
  switch (HQ) {
    case 10: return exact ? kernel_for<10, true, GEMM_BF16>() : kernel_for<10, false, GEMM_BF16>();
    case 11: return exact ? kernel_for<11, true, GEMM_BF16>() : kernel_for<11, false, GEMM_BF16>();
    case 12: return exact ? kernel_for<12, true, GEMM_BF16>() : kernel_for<12, false, GEMM_BF16>();
    case 13: return exact ? kernel_for<13, true, GEMM_BF16>() : kernel_for<13, false, GEMM_BF16>();
    case 14: return exact ? kernel_for<14, true, GEMM_BF16>() : kernel_for<14, false, GEMM_BF16>();
    case 15: return exact ? kernel_for<15, true, GEMM_BF16>() : kernel_for<15, false, GEMM_BF16>();
    case 16: return exact ? kernel_for<16, true, GEMM_BF16>() : kernel_for<16, false, GEMM_BF16>();
    case 17: return exact ? kernel_for<17, true, GEMM_BF16>() : kernel_for<17, false, GEMM_BF16>();
    default: return nullptr;
  }
}

}  // namespace prism

// Instantiations of the persistent ADMM kernel: bf16 x-update operands, chunk sizes 2..9.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_bf16_0(int HQ, bool exact) {
  switch (HQ) {
    case 2: return exact ? kernel_for<2, true, GEMM_BF16>() : kernel_for<2, false, GEMM_BF16>();
    case 3: return exact ? kernel_for<3, true, GEMM_BF16>() : kernel_for<3, false, GEMM_BF16>();
    case 4: return exact ? kernel_for<4, true, GEMM_BF16>() : kernel_for<4, false, GEMM_BF16>();
    case 5: return exact ? kernel_for<5, true, GEMM_BF16>() : kernel_for<5, false, GEMM_BF16>();
    case 6: return exact ? kernel_for<6, true, GEMM_BF16>() : kernel_for<6, false, GEMM_BF16>();
    case 7: return exact ? kernel_for<7, true, GEMM_BF16>() : kernel_for<7, false, GEMM_BF16>();
    case 8: return exact ? kernel_for<8, true, GEMM_BF16>() : kernel_for<8, false, GEMM_BF16>();
    case 9: return exact ? kernel_for<9, true, GEMM_BF16>() : kernel_for<9, false, GEMM_BF16>();
    default: return nullptr;
  }
}

}  // namespace prism

// Instantiations of the persistent ADMM kernel: f16 x-update operands, chunk sizes 18..25.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_f16_2(int HQ, bool exact) {
  switch (HQ) {
    case 18: return exact ? kernel_for<18, true, GEMM_F16>() : kernel_for<18, false, GEMM_F16>();
    case 19: return exact ? kernel_for<19, true, GEMM_F16>() : kernel_for<19, false, GEMM_F16>();
    case 20: return exact ? kernel_for<20, true, GEMM_F16>() : kernel_for<20, false, GEMM_F16>();
    case 21: return exact ? kernel_for<21, true, GEMM_F16>() : kernel_for<21, false, GEMM_F16>();
    case 22: return exact ? kernel_for<22, true, GEMM_F16>() : kernel_for<22, false, GEMM_F16>();
    case 23: return exact ? kernel_for<23, true, GEMM_F16>() : kernel_for<23, false, GEMM_F16>();
    case 24: return exact ? kernel_for<24, true, GEMM_F16>() : kernel_for<24, false, GEMM_F16>();
    case 25: return exact ? kernel_for<25, true, GEMM_F16>() : kernel_for<25, false, GEMM_F16>();
    default: return nullptr;
  }
}

}  // namespace prism

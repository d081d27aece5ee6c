// Instantiations of the persistent ADMM kernel: f16 x-update operands, chunk sizes 26..32.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_f16_3(int HQ, bool exact) {
  switch (HQ) {
    case 26: return exact ? kernel_for<26, true, GEMM_F16>() : kernel_for<26, false, GEMM_F16>();
    case 27: return exact ? kernel_for<27, true, GEMM_F16>() : kernel_for<27, false, GEMM_F16>();
    case 28: return exact ? kernel_for<28, true, GEMM_F16>() : kernel_for<28, false, GEMM_F16>();
    case 29: return exact ? kernel_for<29, true, GEMM_F16>() : kernel_for<29, false, GEMM_F16>();
    case 30: return exact ? kernel_for<30, true, GEMM_F16>() : kernel_for<30, false, GEMM_F16>();
    case 31: return exact ? kernel_for<31, true, GEMM_F16>() : kernel_for<31, false, GEMM_F16>();
    case 32: return exact ? kernel_for<32, true, GEMM_F16>() : kernel_for<32, false, GEMM_F16>();
    default: return nullptr;
  }
}

}  // namespace prism

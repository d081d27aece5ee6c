// Optimizer-step kernels (sampling in the load, cost in the epilogue), bf16 x-update.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn plan_kernel_bf16(int HQ) {
  switch (HQ) {
    case 2: return plan_kernel_for<2, GEMM_BF16>();
    case 3: return plan_kernel_for<3, GEMM_BF16>();
    case 4: return plan_kernel_for<4, GEMM_BF16>();
    case 5: return plan_kernel_for<5, GEMM_BF16>();
    case 6: return plan_kernel_for<6, GEMM_BF16>();
    case 7: return plan_kernel_for<7, GEMM_BF16>();
    case 8: return plan_kernel_for<8, GEMM_BF16>();
    case 9: return plan_kernel_for<9, GEMM_BF16>();
    case 10: return plan_kernel_for<10, GEMM_BF16>();
    case 11: return plan_kernel_for<11, GEMM_BF16>();
    case 12: return plan_kernel_for<12, GEMM_BF16>();
    case 13: return plan_kernel_for<13, GEMM_BF16>();
    case 14: return plan_kernel_for<14, GEMM_BF16>();
    case 15: return plan_kernel_for<15, GEMM_BF16>();
    case 16: return plan_kernel_for<16, GEMM_BF16>();
    case 17: return plan_kernel_for<17, GEMM_BF16>();
    case 18: return plan_kernel_for<18, GEMM_BF16>();
    case 19: return plan_kernel_for<19, GEMM_BF16>();
    case 20: return plan_kernel_for<20, GEMM_BF16>();
    case 21: return plan_kernel_for<21, GEMM_BF16>();
    case 22: return plan_kernel_for<22, GEMM_BF16>();
    case 23: return plan_kernel_for<23, GEMM_BF16>();
    case 24: return plan_kernel_for<24, GEMM_BF16>();
    case 25: return plan_kernel_for<25, GEMM_BF16>();
    case 26: return plan_kernel_for<26, GEMM_BF16>();
    case 27: return plan_kernel_for<27, GEMM_BF16>();
    case 28: return plan_kernel_for<28, GEMM_BF16>();
    case 29: return plan_kernel_for<29, GEMM_BF16>();
    case 30: return plan_kernel_for<30, GEMM_BF16>();
    case 31: return plan_kernel_for<31, GEMM_BF16>();
    case 32: return plan_kernel_for<32, GEMM_BF16>();
    default: return nullptr;
  }
}

}  // namespace prism

// Optimizer-step kernels (sampling in the load, cost in the epilogue), bf16 x-update.
#include "admm_kernels.h"

namespace prism {

SolveKernelFn plan_kernel_bf16(int HQ) {
  switch (HQ) {
    case 2: return admm_plan_kernel<2, GEMM_BF16>;
    case 3: return admm_plan_kernel<3, GEMM_BF16>;
    case 4: return admm_plan_kernel<4, GEMM_BF16>;
    case 5: return admm_plan_kernel<5, GEMM_BF16>;
    case 6: return admm_plan_kernel<6, GEMM_BF16>;
    case 7: return admm_plan_kernel<7, GEMM_BF16>;
    case 8: return admm_plan_kernel<8, GEMM_BF16>;
    case 9: return admm_plan_kernel<9, GEMM_BF16>;
    case 10: return admm_plan_kernel<10, GEMM_BF16>;
    case 11: return admm_plan_kernel<11, GEMM_BF16>;
    case 12: return admm_plan_kernel<12, GEMM_BF16>;
    case 13: return admm_plan_kernel<13, GEMM_BF16>;
    case 14: return admm_plan_kernel<14, GEMM_BF16>;
    case 15: return admm_plan_kernel<15, GEMM_BF16>;
    case 16: return admm_plan_kernel<16, GEMM_BF16>;
    case 17: return admm_plan_kernel<17, GEMM_BF16>;
    case 18: return admm_plan_kernel<18, GEMM_BF16>;
    case 19: return admm_plan_kernel<19, GEMM_BF16>;
    case 20: return admm_plan_kernel<20, GEMM_BF16>;
    case 21: return admm_plan_kernel<21, GEMM_BF16>;
    case 22: return admm_plan_kernel<22, GEMM_BF16>;
    case 23: return admm_plan_kernel<23, GEMM_BF16>;
    case 24: return admm_plan_kernel<24, GEMM_BF16>;
    case 25: return admm_plan_kernel<25, GEMM_BF16>;
    case 26: return admm_plan_kernel<26, GEMM_BF16>;
    case 27: return admm_plan_kernel<27, GEMM_BF16>;
    case 28: return admm_plan_kernel<28, GEMM_BF16>;
    case 29: return admm_plan_kernel<29, GEMM_BF16>;
    case 30: return admm_plan_kernel<30, GEMM_BF16>;
    case 31: return admm_plan_kernel<31, GEMM_BF16>;
    case 32: return admm_plan_kernel<32, GEMM_BF16>;
    default: return nullptr;
  }
}

}  // namespace prism

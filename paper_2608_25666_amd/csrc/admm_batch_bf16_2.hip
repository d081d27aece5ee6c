// Batched persistent ADMM kernels with bf16 x-update operands (part 2).
#include "admm_batch.h"

namespace prism {

BatchKernelFn batch_kernel_bf16_2(int set) {
  if (set == 4) return admm_batch_kernel<GEMM_BF16, 17, 18, 19, 20, 21, 22, 23, 24>;
  if (set == 5) return admm_batch_kernel<GEMM_BF16, 25, 26, 27, 28>;
  if (set == 7) return admm_batch_kernel<GEMM_BF16, 29, 30>;
  if (set == 8) return admm_batch_kernel<GEMM_BF16, 31>;
  if (set == 9) return admm_batch_kernel<GEMM_BF16, 32>;
  return nullptr;
}

}  // namespace prism

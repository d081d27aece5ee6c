// Batched persistent ADMM kernels with bf16 x-update operands (part 1).
#include "admm_batch.h"

namespace prism {

BatchKernelFn batch_kernel_bf16_1(int set) {
  if (set == 2) return admm_batch_kernel_2w<GEMM_BF16, 9, 10, 11, 12>;
  if (set == 3) return admm_batch_kernel<GEMM_BF16, 13, 14, 15, 16>;
  return nullptr;
}

}  // namespace prism

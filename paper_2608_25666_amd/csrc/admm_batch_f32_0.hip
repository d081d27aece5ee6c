// Batched persistent ADMM kernels with f32 x-update operands (part 0).
#include "admm_batch.h"

namespace prism {

BatchKernelFn batch_kernel_f32_0(int set) {
  if (set == 0) return admm_batch_kernel_2w<GEMM_F32, 5, 13>;
  if (set == 1) return admm_batch_kernel_2w<GEMM_F32, 2, 3, 4, 5, 6, 7, 8>;
  if (set == 6) return admm_batch_kernel<GEMM_F32, 25>;
  return nullptr;
}

}  // namespace prism

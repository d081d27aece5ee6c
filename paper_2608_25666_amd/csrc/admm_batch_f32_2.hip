// Batched persistent ADMM kernels with f32 x-update operands (part 2).
#include "admm_batch.h"

namespace prism {

BatchKernelFn batch_kernel_f32_2(int set) {
  if (set == 4) return admm_batch_kernel<GEMM_F32, 17, 18, 19, 20, 21, 22, 23, 24>;
  if (set == 5) return admm_batch_kernel<GEMM_F32, 25, 26, 27, 28>;
  if (set == 7) return admm_batch_kernel<GEMM_F32, 29, 30>;
  if (set == 8) return admm_batch_kernel<GEMM_F32, 31>;
  if (set == 9) return admm_batch_kernel<GEMM_F32, 32>;
  return nullptr;
}

}  // namespace prism

// Instantiations of the two-wave tile kernel, f32 x-update operands.
#include "admm_pair.h"

namespace prism {

PairKernelFn pair_kernel_f32(int HP) {
  switch (HP) {
    case 3: return admm_pair_kernel<3, GEMM_F32>;
    case 7: return admm_pair_kernel<7, GEMM_F32>;
    case 13: return admm_pair_kernel<13, GEMM_F32>;
    default: return nullptr;
  }
}

}  // namespace prism

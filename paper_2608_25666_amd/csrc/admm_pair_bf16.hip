// Instantiations of the two-wave tile kernel, bf16 x-update operands.
#include "admm_pair.h"

namespace prism {

PairKernelFn pair_kernel_bf16(int HP) {
  switch (HP) {
    case 3: return admm_pair_kernel<3, GEMM_BF16>;
    case 7: return admm_pair_kernel<7, GEMM_BF16>;
    case 13: return admm_pair_kernel<13, GEMM_BF16>;
    default: return nullptr;
  }
}

}  // namespace prism

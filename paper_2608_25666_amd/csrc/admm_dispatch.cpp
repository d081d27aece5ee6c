// Chunk-size dispatch over the instantiation files (split for parallel builds).
#include "admm_batch.h"
#include "admm_kernels.h"

namespace prism {

SolveKernelFn solve_kernel_f32_0(int HQ, bool exact);
SolveKernelFn solve_kernel_f32_1(int HQ, bool exact);
SolveKernelFn solve_kernel_f32_2(int HQ, bool exact);
SolveKernelFn solve_kernel_f32_3(int HQ, bool exact);

SolveKernelFn solve_kernel_f32(int HQ, bool exact) {
  if (HQ >= 2 && HQ <= 9) return solve_kernel_f32_0(HQ, exact);
  if (HQ >= 10 && HQ <= 17) return solve_kernel_f32_1(HQ, exact);
  if (HQ >= 18 && HQ <= 25) return solve_kernel_f32_2(HQ, exact);
  if (HQ >= 26 && HQ <= 32) return solve_kernel_f32_3(HQ, exact);
  return nullptr;
}

SolveKernelFn solve_kernel_bf16_0(int HQ, bool exact);
SolveKernelFn solve_kernel_bf16_1(int HQ, bool exact);
SolveKernelFn solve_kernel_bf16_2(int HQ, bool exact);
SolveKernelFn solve_kernel_bf16_3(int HQ, bool exact);

SolveKernelFn solve_kernel_bf16(int HQ, bool exact) {
  if (HQ >= 2 && HQ <= 9) return solve_kernel_bf16_0(HQ, exact);
  if (HQ >= 10 && HQ <= 17) return solve_kernel_bf16_1(HQ, exact);
  if (HQ >= 18 && HQ <= 25) return solve_kernel_bf16_2(HQ, exact);
  if (HQ >= 26 && HQ <= 32) return solve_kernel_bf16_3(HQ, exact);
  return nullptr;
}

SolveKernelFn solve_kernel_f16_0(int HQ, bool exact);
SolveKernelFn solve_kernel_f16_1(int HQ, bool exact);
SolveKernelFn solve_kernel_f16_2(int HQ, bool exact);
SolveKernelFn solve_kernel_f16_3(int HQ, bool exact);

SolveKernelFn solve_kernel_f16(int HQ, bool exact) {
  if (HQ >= 2 && HQ <= 9) return solve_kernel_f16_0(HQ, exact);
  if (HQ >= 10 && HQ <= 17) return solve_kernel_f16_1(HQ, exact);
  if (HQ >= 18 && HQ <= 25) return solve_kernel_f16_2(HQ, exact);
  if (HQ >= 26 && HQ <= 32) return solve_kernel_f16_3(HQ, exact);
  return nullptr;
}

BatchKernelFn batch_kernel_f32_0(int set);
BatchKernelFn batch_kernel_f32_1(int set);
BatchKernelFn batch_kernel_f32_2(int set);
BatchKernelFn batch_kernel_bf16_0(int set);
BatchKernelFn batch_kernel_bf16_1(int set);
BatchKernelFn batch_kernel_bf16_2(int set);
BatchKernelFn batch_kernel_f16_0(int set);
BatchKernelFn batch_kernel_f16_1(int set);
BatchKernelFn batch_kernel_f16_2(int set);

BatchKernelFn batch_kernel_f32(int set) {
  if (set <= 1 || set == 6) return batch_kernel_f32_0(set);
  return set <= 3 ? batch_kernel_f32_1(set) : batch_kernel_f32_2(set);
}
BatchKernelFn batch_kernel_bf16(int set) {
  if (set <= 1 || set == 6) return batch_kernel_bf16_0(set);
  return set <= 3 ? batch_kernel_bf16_1(set) : batch_kernel_bf16_2(set);
}
BatchKernelFn batch_kernel_f16(int set) {
  if (set <= 1 || set == 6) return batch_kernel_f16_0(set);
  return set <= 3 ? batch_kernel_f16_1(set) : batch_kernel_f16_2(set);
}

}  // namespace prism

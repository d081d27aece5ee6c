// Host-side construction of the reusable x-update factor and its on-chip layouts.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace prism {

// Rows of one lane group ("chunk") for horizon H: the 4 lane groups of a wave
// each hold HQ consecutive steps of a column, HQ = ceil(H / 4).
inline int chunk_rows(int H) { return (H + 3) / 4; }

// K (H*H, row-major) and k (H) of x = K r + k v0, the solution of the
// equality-constrained primal system with P = I + C^T R C, C = [I; L; D1; D2]
// and R = rho * diag(w) (w: one positive weight per constraint block, in the
// order velocity, position, acceleration, jerk; null = all ones).
// Returns false if P is not positive definite (cannot happen for rho, w > 0).
bool build_factor(int H, double rho, const double* w, std::vector<double>& K, std::vector<double>& k);

// FP32 A-operand fragments for v_mfma_f32_16x16x4_f32, read as one float4 per
// lane per (output block b, group of four k-steps jj):
//   index ((b * NJ4 + jj) * 64 + lane) * 4 + e,   k-step j = 4*jj + e.
// NB = ceil(HQ/4) output blocks, NJ4 = ceil(HQ/4).
void layout_f32(const std::vector<double>& K, int H, int HQ, std::vector<float>& out);

// 16-bit A-operand fragments for v_mfma_f32_16x16x32_{bf16,f16}: 8 values per
// lane per (b, k-step jj), index ((b * NJ8 + jj) * 64 + lane) * 8 + e,
// NJ8 = ceil(HQ/8). bf16 = true selects bfloat16, otherwise IEEE half. RNE.
void layout_16(const std::vector<double>& K, int H, int HQ, bool bf16, std::vector<uint16_t>& out);

// FP64 A-operand fragments for v_mfma_f64_16x16x4_f64, whose accumulator puts
// row g + 4e of a 16x16 block in item e of lane group g (the FP32 form uses
// row 4g + e). Two k-steps per lane per (output block b, pair jp), read as one
// 16-byte load: index ((b * NJ2 + jp) * 64 + lane) * 2 + e, k-step j = 2*jp + e,
// NB = ceil(HQ/4), NJ2 = ceil(HQ/2). Column 0 of K (identically zero: step 1 is
// fixed by the equality) holds k instead, so that x = K r + k v0 is one product
// with r_1 set to v0.
void layout_f64(const std::vector<double>& K, const std::vector<double>& k, int H, int HQ,
                std::vector<double>& out);
inline size_t f64_frag_count(int HQ) {
  return (size_t)((HQ + 3) / 4) * ((HQ + 1) / 2) * 64 * 2;
}

// Two-wave tiles: a tile's H steps are cut into eight chunks of HP = ceil(H / 8) rows;
// member m of the pair of waves holds chunks 4m .. 4m+3 (lane group g: chunk 4m + g).
// Member m's A-operand fragments cover its own output rows (NB = ceil(HP/4) blocks)
// against the k-steps of both members' chunks, its own first (source s = 0) and then
// its partner's (s = 1):
//   FP32:   index m*F + (((b*2 + s)*NJ4 + jj)*64 + lane)*4 + e,  k-step j = 4jj + e,
//   16-bit: index m*F + (((b*2 + s)*NJ8 + jj)*64 + lane)*8 + e,  k-step j = 8jj + e,
// with F the per-member fragment count. Row and column steps past H are zero.
inline int pair_chunk_rows(int H) { return (H + 7) / 8; }
void layout_pair_f32(const std::vector<double>& K, int H, int HP, std::vector<float>& out);
void layout_pair_16(const std::vector<double>& K, int H, int HP, bool bf16,
                    std::vector<uint16_t>& out);
inline size_t pair_f32_frag_count(int HP) {   // per member
  return (size_t)((HP + 3) / 4) * 2 * ((HP + 3) / 4) * 64 * 4;
}
inline size_t pair_16_frag_count(int HP) {    // per member
  return (size_t)((HP + 3) / 4) * 2 * ((HP + 7) / 8) * 64 * 8;
}

// Byte sizes of the two layouts.
inline size_t f32_frag_bytes(int HQ) {
  const int nb = (HQ + 3) / 4;
  return (size_t)nb * ((HQ + 3) / 4) * 64 * 4 * sizeof(float);
}
inline size_t b16_frag_bytes(int HQ) {
  const int nb = (HQ + 3) / 4;
  return (size_t)nb * ((HQ + 7) / 8) * 64 * 8 * sizeof(uint16_t);
}

uint16_t float_to_bf16_rne(float f);
uint16_t float_to_f16_rne(float f);

}  // namespace prism

// Host check of the two-wave tile fragment layouts (layout_pair_f32, layout_pair_16).
//
// Emulates v_mfma_f32_16x16x4_f32 (A row r, k-column kk from lane 16*kk + r; B k-row kk,
// column n from lane 16*kk + n; item e of lane 16*g + n holds accumulator row 4g + e)
// and v_mfma_f32_16x16x32_* (A row r, k-columns 8*kk + e from lane 16*kk + r, item e;
// B k-rows 8*kk + e, column n from lane 16*kk + n) over the fragments of each member
// of a pair. Each member feeds its own defect registers (source 0) and its partner's
// (source 1) as B, the way the kernel does, and must end with x = K d on every lane for
// its steps (4m + g) * HP + i. The 16-bit layout is checked with the fragments widened
// back to float, against K rounded the same way. Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "factor.h"

using namespace prism;

static float from_bf16(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
static float from_f16(uint16_t h) {
  _Float16 v;
  std::memcpy(&v, &h, 2);
  return (float)v;
}

static int check(int H, bool sixteen, bool bf16, unsigned seed) {
  const int HP = pair_chunk_rows(H);
  const double w[4] = {1.7, 2.125 / H, 13.6, 17.0};
  std::vector<double> K, k;
  if (!build_factor(H, 1.0, w, K, k)) return 1;
  std::vector<float> f32;
  std::vector<uint16_t> f16;
  if (sixteen) layout_pair_16(K, H, HP, bf16, f16);
  else layout_pair_f32(K, H, HP, f32);
  const int NB = (HP + 3) / 4, NJ = sixteen ? (HP + 7) / 8 : (HP + 3) / 4, KW = sixteen ? 8 : 4;
  const size_t per = sixteen ? pair_16_frag_count(HP) : pair_f32_frag_count(HP);
  std::mt19937 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  const int C = 16;
  std::vector<double> d((size_t)8 * HP * C, 0.0);
  for (int c = 0; c < C; ++c)
    for (int s = 0; s < H; ++s) d[(size_t)s * C + c] = nd(gen);
  // register j of lane (g, c) of member m holds d at step (4m + g) * HP + j
  auto dreg = [&](int m, int lane, int j) {
    const int s = (4 * m + (lane >> 4)) * HP + j;
    return (j < HP && s < H) ? d[(size_t)s * C + (lane & 15)] : 0.0;
  };
  auto frag = [&](int m, int b, int src, int jj, int lane, int e) -> double {
    const size_t i = m * per + ((((size_t)b * 2 + src) * NJ + jj) * 64 + lane) * KW + e;
    if (!sixteen) return f32[i];
    return bf16 ? from_bf16(f16[i]) : from_f16(f16[i]);
  };
  auto kval = [&](int r, int c) -> double {
    const float v = (float)K[(size_t)r * H + c];
    if (!sixteen) return v;
    return bf16 ? from_bf16(float_to_bf16_rne(v)) : from_f16(float_to_f16_rne(v));
  };
  double worst = 0.0;
  for (int m = 0; m < 2; ++m) {
    std::vector<double> acc((size_t)64 * 4 * NB, 0.0);
    for (int b = 0; b < NB; ++b)
      for (int src = 0; src < 2; ++src) {
        const int ms = src == 0 ? m : 1 - m;
        for (int jj = 0; jj < NJ; ++jj) {
          double D[16][16] = {};
          for (int r = 0; r < 16; ++r)
            for (int n = 0; n < 16; ++n)
              for (int kk = 0; kk < 4; ++kk)
                for (int e = 0; e < KW; ++e) {
                  const int j = KW * jj + e;
                  D[r][n] += frag(m, b, src, jj, 16 * kk + r, e) * dreg(ms, 16 * kk + n, j);
                }
          for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 4; ++e)
              acc[(size_t)lane * 4 * NB + 4 * b + e] += D[4 * (lane >> 4) + e][lane & 15];
        }
      }
    for (int lane = 0; lane < 64; ++lane)
      for (int i = 0; i < 4 * NB; ++i) {
        const int s = (4 * m + (lane >> 4)) * HP + i;
        double want = 0.0;
        if (i < HP && s < H)
          for (int t = 0; t < H; ++t) want += kval(s, t) * d[(size_t)t * C + (lane & 15)];
        worst = std::fmax(worst, std::fabs(acc[(size_t)lane * 4 * NB + i] - want));
      }
  }
  std::printf("H=%d HP=%d %s: max |emulated - K d| = %.3e\n", H, HP,
              sixteen ? (bf16 ? "bf16" : "f16") : "f32", worst);
  return worst <= 1e-9 ? 0 : 3;
}

int main() {
  int bad = 0;
  const int Hs[] = {16, 20, 23, 49, 50, 56, 64, 97, 100, 104, 128};
  for (int H : Hs) {
    bad |= check(H, false, false, 3u + H);
    bad |= check(H, true, true, 5u + H);
    bad |= check(H, true, false, 7u + H);
  }
  std::printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}

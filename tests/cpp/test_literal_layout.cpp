// Host check of the FP64 fragment layout of the printed-iteration kernel.
//
// Emulates v_mfma_f64_16x16x4_f64 with its lane layout (A row m, k-column kk from lane
// 16*kk + m; B k-row kk, column n from lane 16*kk + n; item e of lane 16*g + n holds
// accumulator row g + 4e) over the fragments layout_f64 writes, feeding each lane's
// own right-hand-side registers as B the way the kernel does, and checks that every
// lane ends with x = K r + k v0 for its steps g*HQ + i. Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <random>
#include <vector>

#include "factor.h"

using namespace prism;

static int check(int H, int HQ, double rho, const double* w, unsigned seed) {
  std::vector<double> K, k, frag;
  if (!build_factor(H, rho, w, K, k)) return 1;
  layout_f64(K, k, H, HQ, frag);
  const int NB = (HQ + 3) / 4, NJ2 = (HQ + 1) / 2;
  if (frag.size() != f64_frag_count(HQ)) return 2;
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  const int C = 16;
  // r[step][col]; step 0 (pinned by the equality) carries v0 in the kernel
  std::vector<double> r((size_t)4 * HQ * C, 0.0), v0(C);
  for (int c = 0; c < C; ++c) {
    v0[c] = nd(gen);
    for (int s = 0; s < H; ++s) r[(size_t)s * C + c] = s == 0 ? v0[c] : nd(gen);
  }
  // lane registers: reg[lane][i] = r at step g*HQ + i
  auto rreg = [&](int lane, int i) {
    const int g = lane >> 4, c = lane & 15, s = g * HQ + i;
    return (i < HQ && s < H) ? r[(size_t)s * C + c] : 0.0;
  };
  // x[lane][4b+e] accumulators
  std::vector<double> acc((size_t)64 * 4 * NB, 0.0);
  for (int b = 0; b < NB; ++b)
    for (int j = 0; j < HQ; ++j) {
      const int jp = j / 2, e2 = j % 2;
      double D[16][16] = {};
      for (int m = 0; m < 16; ++m)
        for (int n = 0; n < 16; ++n)
          for (int kk = 0; kk < 4; ++kk) {
            const double a = frag[(((size_t)b * NJ2 + jp) * 64 + 16 * kk + m) * 2 + e2];
            const double bb = rreg(16 * kk + n, j);
            D[m][n] += a * bb;
          }
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 4; ++e)
          acc[(size_t)lane * 4 * NB + 4 * b + e] += D[(lane >> 4) + 4 * e][lane & 15];
    }
  double worst = 0.0;
  for (int lane = 0; lane < 64; ++lane) {
    const int g = lane >> 4, c = lane & 15;
    for (int i = 0; i < 4 * NB; ++i) {
      const int s = g * HQ + i;
      double want = 0.0;
      if (i < HQ && s < H) {
        want = k[s] * v0[c];
        for (int t = 1; t < H; ++t) want += K[(size_t)s * H + t] * r[(size_t)t * C + c];
      }
      const double got = acc[(size_t)lane * 4 * NB + i];
      worst = std::fmax(worst, std::fabs(got - want));
    }
  }
  std::printf("H=%d HQ=%d rho=%g: max |emulated - K r - k v0| = %.3e\n", H, HQ, rho, worst);
  return worst <= 1e-9 ? 0 : 3;
}

int main() {
  const double dt = 0.02;
  const double wl[4] = {1.0, dt * dt, 1.0 / (dt * dt), 1.0 / (dt * dt * dt * dt)};
  const double wd[4] = {1.7, 2.125 / 50, 13.6, 17.0};
  int bad = 0;
  const int Hs[] = {2, 5, 8, 9, 13, 50, 51, 69, 100, 128};
  for (int H : Hs) {
    const int HQ = std::max(2, (H + 3) / 4);
    bad |= check(H, HQ, 1.0, wd, 7u + H);
    bad |= check(H, HQ, 2.0, wl, 11u + H);   // the printed iteration's factor (delta = 1)
  }
  std::printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}

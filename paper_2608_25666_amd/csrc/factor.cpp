// FP64 host construction of the reusable x-update factor.
//
// Sec. III-D, "Step 2: Primal update" (eqs. (admm_primal), (admm_KKT)) solves
//   [P  e1][x ]   [r ]
//   [e1' 0][mu] = [v0],   P = I + rho C^T C (scalar penalty),
// and "Pre-computable factorization" factors it once. With a diagonal block
// penalty R = rho diag(w) in place of the scalar penalty, P = I + C^T R C.
// Eliminating mu gives
//   x = K r + k v0,  K = Pi - Pi e1 e1' Pi / Pi_11,  k = Pi e1 / Pi_11,  Pi = P^-1.
// C = [I; L; D1; D2] are the constraint rows after scaling every block to
// velocity units (cumulative sum L, first difference D1, second difference D2
// of Sec. III-D eqs. (pos_stack), (acc_stack), (D2_def)), so K depends on H,
// rho and the block weights only. K is symmetric, K e1 = 0 (the fixed first
// step never moves) and K P = I - k e1'.
#include "factor.h"

#include <cmath>
#include <cstring>

namespace prism {

namespace {

// G = C^T diag(w) C for C = [I; L; D1; D2], assembled from the row definitions
// (w[b] weights every row of block b).
void gram(int H, const double w[4], std::vector<double>& G) {
  G.assign((size_t)H * H, 0.0);
  auto add_row = [&](double wb, const std::vector<std::pair<int, double>>& row) {
    for (auto& a : row)
      for (auto& b : row) G[(size_t)a.first * H + b.first] += wb * a.second * b.second;
  };
  for (int i = 0; i < H; ++i) add_row(w[0], {{i, 1.0}});                 // velocity rows
  for (int i = 0; i < H; ++i) {                                           // position rows
    std::vector<std::pair<int, double>> row;
    for (int c = 0; c <= i; ++c) row.push_back({c, 1.0});
    add_row(w[1], row);
  }
  for (int i = 0; i < H; ++i) {                                           // acceleration rows
    if (i == 0) add_row(w[2], {{0, 1.0}});
    else add_row(w[2], {{i, 1.0}, {i - 1, -1.0}});
  }
  for (int r = 0; r + 1 < H; ++r) {                                       // jerk rows, steps 2..H
    if (r == 0) add_row(w[3], {{0, -2.0}, {1, 1.0}});
    else add_row(w[3], {{r - 1, 1.0}, {r, -2.0}, {r + 1, 1.0}});
  }
}

// In-place Cholesky A = R R^T (lower R); returns false if not positive definite.
bool cholesky(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    const double rjj = std::sqrt(d);
    A[(size_t)j * n + j] = rjj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = s / rjj;
    }
  }
  return true;
}

}  // namespace

bool build_factor(int H, double rho, const double* w, std::vector<double>& K, std::vector<double>& k) {
  const double ones[4] = {1.0, 1.0, 1.0, 1.0};
  std::vector<double> P;
  gram(H, w ? w : ones, P);
  for (auto& v : P) v *= rho;
  for (int i = 0; i < H; ++i) P[(size_t)i * H + i] += 1.0;
  std::vector<double> R = P;
  if (!cholesky(H, R)) return false;
  // Pi = P^-1 column by column: solve R y = e_c, R^T x = y.
  std::vector<double> Pi((size_t)H * H, 0.0), y(H), x(H);
  for (int c = 0; c < H; ++c) {
    for (int i = 0; i < H; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int t = 0; t < i; ++t) s -= R[(size_t)i * H + t] * y[t];
      y[i] = s / R[(size_t)i * H + i];
    }
    for (int i = H - 1; i >= 0; --i) {
      double s = y[i];
      for (int t = i + 1; t < H; ++t) s -= R[(size_t)t * H + i] * x[t];
      x[i] = s / R[(size_t)i * H + i];
    }
    for (int i = 0; i < H; ++i) Pi[(size_t)i * H + c] = x[i];
  }
  // symmetrize (the two triangular solves leave rounding asymmetry)
  for (int i = 0; i < H; ++i)
    for (int j = i + 1; j < H; ++j) {
      const double m = 0.5 * (Pi[(size_t)i * H + j] + Pi[(size_t)j * H + i]);
      Pi[(size_t)i * H + j] = Pi[(size_t)j * H + i] = m;
    }
  const double p11 = Pi[0];
  K.assign((size_t)H * H, 0.0);
  k.assign(H, 0.0);
  for (int i = 0; i < H; ++i) k[i] = Pi[(size_t)i * H] / p11;
  for (int i = 1; i < H; ++i)
    for (int j = 1; j < H; ++j)
      K[(size_t)i * H + j] = Pi[(size_t)i * H + j] - Pi[(size_t)i * H] * Pi[(size_t)j * H] / p11;
  // row and column 0 are exactly zero: the first step is pinned to v0
  return true;
}

namespace {

// Physical step held by A-operand row m of output block b (see the kernel's
// register layout): lane group m/4 of the output, chunk register 4b + m%4.
inline int out_row(int b, int m, int HQ, int H) {
  const int reg = 4 * b + (m & 3);
  const int row = (m >> 2) * HQ + reg;
  return (reg < HQ && row < H) ? row : -1;
}

// The same for the FP64 accumulator (row m of a block is lane group m%4, item m/4).
inline int out_row_f64(int b, int m, int HQ, int H) {
  const int reg = 4 * b + (m >> 2);
  const int row = (m & 3) * HQ + reg;
  return (reg < HQ && row < H) ? row : -1;
}

inline int in_row(int gk, int j, int HQ, int H) {
  const int row = gk * HQ + j;
  return (j < HQ && row < H) ? row : -1;
}

}  // namespace

void layout_f32(const std::vector<double>& K, int H, int HQ, std::vector<float>& out) {
  const int nb = (HQ + 3) / 4, nj4 = (HQ + 3) / 4;
  out.assign((size_t)nb * nj4 * 64 * 4, 0.0f);
  for (int b = 0; b < nb; ++b)
    for (int jj = 0; jj < nj4; ++jj)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 4; ++e) {
          const int r = out_row(b, lane & 15, HQ, H);
          const int c = in_row(lane >> 4, 4 * jj + e, HQ, H);
          const float v = (r >= 0 && c >= 0) ? (float)K[(size_t)r * H + c] : 0.0f;
          out[(((size_t)b * nj4 + jj) * 64 + lane) * 4 + e] = v;
        }
}

uint16_t float_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

uint16_t float_to_f16_rne(float f) {
  _Float16 h = (_Float16)f;   // IEEE round-to-nearest-even conversion
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

void layout_16(const std::vector<double>& K, int H, int HQ, bool bf16, std::vector<uint16_t>& out) {
  const int nb = (HQ + 3) / 4, nj8 = (HQ + 7) / 8;
  out.assign((size_t)nb * nj8 * 64 * 8, 0);
  for (int b = 0; b < nb; ++b)
    for (int jj = 0; jj < nj8; ++jj)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
          const int r = out_row(b, lane & 15, HQ, H);
          const int c = in_row(lane >> 4, 8 * jj + e, HQ, H);
          const float v = (r >= 0 && c >= 0) ? (float)K[(size_t)r * H + c] : 0.0f;
          out[(((size_t)b * nj8 + jj) * 64 + lane) * 8 + e] =
              bf16 ? float_to_bf16_rne(v) : float_to_f16_rne(v);
        }
}

namespace {

// Step of MFMA row `row` of member m's output block b (lane group row / 4 of the
// member, chunk register 4b + row % 4), or -1 past the chunk or past H.
inline int pair_out_row(int m, int b, int row, int HP, int H) {
  const int reg = 4 * b + (row & 3);
  const int step = (4 * m + (row >> 2)) * HP + reg;
  return (reg < HP && step < H) ? step : -1;
}

// Step of k-index (lane group gk, register j) of source member ms.
inline int pair_in_row(int ms, int gk, int j, int HP, int H) {
  const int step = (4 * ms + gk) * HP + j;
  return (j < HP && step < H) ? step : -1;
}

}  // namespace

void layout_pair_f32(const std::vector<double>& K, int H, int HP, std::vector<float>& out) {
  const int nb = (HP + 3) / 4, nj4 = (HP + 3) / 4;
  const size_t per = pair_f32_frag_count(HP);
  out.assign(2 * per, 0.0f);
  for (int m = 0; m < 2; ++m)
    for (int b = 0; b < nb; ++b)
      for (int s = 0; s < 2; ++s)
        for (int jj = 0; jj < nj4; ++jj)
          for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 4; ++e) {
              const int r = pair_out_row(m, b, lane & 15, HP, H);
              const int c = pair_in_row(s == 0 ? m : 1 - m, lane >> 4, 4 * jj + e, HP, H);
              const float v = (r >= 0 && c >= 0) ? (float)K[(size_t)r * H + c] : 0.0f;
              out[m * per + ((((size_t)b * 2 + s) * nj4 + jj) * 64 + lane) * 4 + e] = v;
            }
}

void layout_pair_16(const std::vector<double>& K, int H, int HP, bool bf16,
                    std::vector<uint16_t>& out) {
  const int nb = (HP + 3) / 4, nj8 = (HP + 7) / 8;
  const size_t per = pair_16_frag_count(HP);
  out.assign(2 * per, 0);
  for (int m = 0; m < 2; ++m)
    for (int b = 0; b < nb; ++b)
      for (int s = 0; s < 2; ++s)
        for (int jj = 0; jj < nj8; ++jj)
          for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
              const int r = pair_out_row(m, b, lane & 15, HP, H);
              const int c = pair_in_row(s == 0 ? m : 1 - m, lane >> 4, 8 * jj + e, HP, H);
              const float v = (r >= 0 && c >= 0) ? (float)K[(size_t)r * H + c] : 0.0f;
              out[m * per + ((((size_t)b * 2 + s) * nj8 + jj) * 64 + lane) * 8 + e] =
                  bf16 ? float_to_bf16_rne(v) : float_to_f16_rne(v);
            }
}

void layout_f64(const std::vector<double>& K, const std::vector<double>& k, int H, int HQ,
                std::vector<double>& out) {
  const int nb = (HQ + 3) / 4, nj2 = (HQ + 1) / 2;
  out.assign(f64_frag_count(HQ), 0.0);
  for (int b = 0; b < nb; ++b)
    for (int jp = 0; jp < nj2; ++jp)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 2; ++e) {
          const int r = out_row_f64(b, lane & 15, HQ, H);
          const int c = in_row(lane >> 4, 2 * jp + e, HQ, H);
          // column 0 of K is zero (step 1 is pinned); it carries k instead, so
          // x = K' r with r_1 := v0
          const double v = c == 0 ? k[r] : K[(size_t)r * H + c];
          out[(((size_t)b * nj2 + jp) * 64 + lane) * 2 + e] = (r >= 0 && c >= 0) ? v : 0.0;
        }
}

}  // namespace prism

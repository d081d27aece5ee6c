// A native consumer of the C ABI (include/prism_proj.h), with no Python or
// PyTorch involved: reads one projection problem from a binary file, allocates
// device buffers with the HIP runtime, calls the library, and writes the results.
// Mode 0: prism_proj_create_ex, prism_proj_solve_ex, prism_proj_feasibility.
// Mode 1 (the plain signatures): prism_proj_create (weights ignored),
// prism_proj_set_options, prism_proj_solve, prism_proj_feasibility; the
// iteration counts are then not reported (written as -1).
//
// Input (little-endian): int32 H, nj, N, iters, precision, mode; float64 dt, rho,
// weights[4]; float32 alpha, tol; float64 bounds[8][nj] (q_min, q_max, v_min,
// v_max, a_min, a_max, j_min, j_max), q0[nj], v0[nj]; float32 samples[N][H][nj].
// Output: float32 x[N][H][nj], r_primal[N][nj], r_dual[N][nj]; int32
// iters[N][nj]; float64 violations[N][nj][5].
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "prism_proj.h"

#define CHECK_HIP(x)                                                          \
  do {                                                                        \
    if ((x) != hipSuccess) {                                                  \
      std::fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__);       \
      return 3;                                                               \
    }                                                                         \
  } while (0)
#define CHECK_PRISM(x)                                                        \
  do {                                                                        \
    const prism_status_t s_ = (x);                                            \
    if (s_ != PRISM_OK) {                                                     \
      std::fprintf(stderr, "prism error %d (%s) at line %d\n", (int)s_,       \
                   prism_status_str(s_), __LINE__);                           \
      return 4;                                                               \
    }                                                                         \
  } while (0)

template <class T>
static bool rd(std::FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
    return 1;
  }
  std::FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 1;
  int32_t hdr[6];
  double dtrho[2], w[4];
  float at[2];
  if (!rd(f, hdr, 6) || !rd(f, dtrho, 2) || !rd(f, w, 4) || !rd(f, at, 2)) return 2;
  const int H = hdr[0], nj = hdr[1], N = hdr[2], iters = hdr[3], precision = hdr[4];
  const int mode = hdr[5];
  if (H < 2 || nj < 1 || N < 1 || (mode != 0 && mode != 1)) return 2;
  std::vector<double> b(8 * (size_t)nj), q0(nj), v0(nj);
  const size_t nx = (size_t)N * H * nj, nc = (size_t)N * nj;
  std::vector<float> xs(nx);
  if (!rd(f, b.data(), b.size()) || !rd(f, q0.data(), nj) || !rd(f, v0.data(), nj) ||
      !rd(f, xs.data(), nx))
    return 2;
  std::fclose(f);

  prism_bounds_t bounds = {&b[0 * nj], &b[1 * nj], &b[2 * nj], &b[3 * nj],
                           &b[4 * nj], &b[5 * nj], &b[6 * nj], &b[7 * nj]};
  prism_proj_t p = nullptr;
  if (mode == 0)
    CHECK_PRISM(prism_proj_create_ex(H, nj, dtrho[0], &bounds, dtrho[1], w, &p));
  else
    CHECK_PRISM(prism_proj_create(H, nj, dtrho[0], &bounds, dtrho[1], &p));
  prism_options_t o;
  prism_options_default(&o);
  o.precision = precision;
  o.alpha = at[0];
  o.tol = at[1];
  o.fp32_tail = precision == PRISM_PREC_FP32 ? 0 : 10;

  float *d_x = nullptr, *d_out = nullptr, *d_rp = nullptr, *d_rd = nullptr;
  int32_t* d_it = nullptr;
  double* d_v = nullptr;
  CHECK_HIP(hipMalloc(&d_x, nx * sizeof(float)));
  CHECK_HIP(hipMalloc(&d_out, nx * sizeof(float)));
  CHECK_HIP(hipMalloc(&d_rp, nc * sizeof(float)));
  CHECK_HIP(hipMalloc(&d_rd, nc * sizeof(float)));
  CHECK_HIP(hipMalloc(&d_it, nc * sizeof(int32_t)));
  CHECK_HIP(hipMalloc(&d_v, nc * 5 * sizeof(double)));
  CHECK_HIP(hipMemcpy(d_x, xs.data(), nx * sizeof(float), hipMemcpyHostToDevice));
  hipStream_t st;
  CHECK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));

  if (mode == 0) {
    prism_solve_args_t a = {};
    a.v_samples = d_x;
    a.N = N;
    a.iters = iters;
    a.q0 = q0.data();
    a.v0 = v0.data();
    a.v_out = d_out;
    a.r_primal = d_rp;
    a.r_dual = d_rd;
    a.iters_out = d_it;
    a.opts = &o;
    CHECK_PRISM(prism_proj_solve_ex(p, &a, st));
  } else {
    CHECK_HIP(hipMemset(d_it, 0xff, nc * sizeof(int32_t)));
    CHECK_PRISM(prism_proj_set_options(p, &o));
    CHECK_PRISM(prism_proj_solve(p, d_x, N, q0.data(), v0.data(), iters, d_out, d_rp, d_rd, st));
  }
  CHECK_PRISM(prism_proj_feasibility(p, d_out, N, q0.data(), v0.data(), d_v, st));
  CHECK_HIP(hipStreamSynchronize(st));

  std::vector<float> xo(nx), rpo(nc), rdo(nc);
  std::vector<int32_t> ito(nc);
  std::vector<double> vo(nc * 5);
  CHECK_HIP(hipMemcpy(xo.data(), d_out, nx * sizeof(float), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(rpo.data(), d_rp, nc * sizeof(float), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(rdo.data(), d_rd, nc * sizeof(float), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(ito.data(), d_it, nc * sizeof(int32_t), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(vo.data(), d_v, nc * 5 * sizeof(double), hipMemcpyDeviceToHost));
  std::FILE* g = std::fopen(argv[2], "wb");
  if (!g) return 1;
  std::fwrite(xo.data(), sizeof(float), nx, g);
  std::fwrite(rpo.data(), sizeof(float), nc, g);
  std::fwrite(rdo.data(), sizeof(float), nc, g);
  std::fwrite(ito.data(), sizeof(int32_t), nc, g);
  std::fwrite(vo.data(), sizeof(double), nc * 5, g);
  std::fclose(g);

  (void)hipStreamDestroy(st);
  (void)hipFree(d_x);
  (void)hipFree(d_out);
  (void)hipFree(d_rp);
  (void)hipFree(d_rd);
  (void)hipFree(d_it);
  (void)hipFree(d_v);
  prism_proj_destroy(p);
  std::printf("abi_solve: N=%d H=%d joints=%d done\n", N, H, nj);
  return 0;
}

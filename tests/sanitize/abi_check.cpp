// Driver of the C ABI for the host AddressSanitizer / UndefinedBehaviorSanitizer
// build (paper_2404_07293_amd/build.py --sanitize). Every host source of the
// library is compiled with -fsanitize=address,undefined on the host side
// only; this program links those objects and walks the ABI:
//
//   abi_check cpu   argument validation and error reporting of every entry
//                   point that can be reached without a device (null
//                   arguments, bad sizes, no device), then exits 0;
//   abi_check gpu   the same, then a context, FP64 host setups of a small
//                   layered sample on both boundary routes and of a batch
//                   with the device eigensolver, syntheses in FP64 and FP32
//                   (plain, tiled, no-allocation), the exterior coefficients,
//                   a batched sweep, the surrogate's forward pass in both
//                   arithmetics, and the error paths of a solved problem.
//
// Any sanitizer report aborts the program with a non-zero status; the test
// (tests/test_sanitize_abi.py) also looks for the reports' banners.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "scw.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, scw_last_error());
    ++failures;
  }
}

// a two-layer sample of 8 x 6 voxels with a lossy inclusion
std::vector<double> sample_index(int nx, int ny, int nz) {
  std::vector<double> n(2 * (size_t)nx * ny * nz);
  for (int l = 0; l < nz; ++l)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t k = ((size_t)l * ny + j) * nx + i;
        const bool in = (i - nx / 2) * (i - nx / 2) + (j - ny / 2) * (j - ny / 2) < 5;
        n[2 * k] = in ? 1.6 : 1.3 + 0.02 * l;
        n[2 * k + 1] = in ? 0.03 : 0.0;
      }
  return n;
}

scw_problem problem(const std::vector<double>& n, int nx, int ny, int nz, int U, int V) {
  scw_problem p;
  std::memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.px = 0.31;
  p.py = 0.27;
  p.pz = 0.19;
  p.n = n.data();
  p.lambda = 1.0;
  p.n_top = 1.0;
  p.n_bot_re = 1.45;
  p.n_bot_im = 0.01;
  p.U = U;
  p.V = V;
  p.pw_ex[0] = 0.8;
  p.pw_ey[0] = 0.3;
  p.pw_ey[1] = -0.2;
  return p;
}

void validation_paths() {
  // null and out-of-range arguments are reported, never dereferenced
  expect(scw_create(nullptr, 0, 0) != SCW_OK, "scw_create(null)");
  scw_ctx* none = nullptr;
  expect(scw_create(&none, -1, 0) != SCW_OK && none == nullptr, "scw_create(device -1)");
  expect(std::strlen(scw_last_error()) > 0, "error message set");
  scw_solution* sol = nullptr;
  expect(scw_solve(nullptr, nullptr, &sol) != SCW_OK, "scw_solve(null)");
  expect(scw_solve_batch(nullptr, nullptr, 0, nullptr) != SCW_OK, "scw_solve_batch(null)");
  scw_grid g{4, 4, 4, 0.0, 1.0};
  expect(scw_synthesize(nullptr, nullptr, &g, SCW_FP32, nullptr, nullptr) != SCW_OK,
         "scw_synthesize(null)");
  expect(scw_synthesize_noalloc(nullptr, nullptr, &g, SCW_FP32, nullptr, nullptr) != SCW_OK,
         "scw_synthesize_noalloc(null)");
  expect(scw_solution_exterior(nullptr, nullptr, nullptr, nullptr) != SCW_OK,
         "scw_solution_exterior(null)");
  scw_solution_info info;
  expect(scw_solution_info_get(nullptr, &info) != SCW_OK, "scw_solution_info_get(null)");
  expect(scw_sur_param_count() > 0, "scw_sur_param_count");
  scw_sur* sur = nullptr;
  expect(scw_sur_create(nullptr, 8, 0, &sur) != SCW_OK, "scw_sur_create(null ctx)");
  expect(scw_stage_name(0) != nullptr, "scw_stage_name");
  scw_solution_free(nullptr);
  scw_destroy(nullptr);
}

double rel(const std::vector<std::complex<double>>& a, const std::vector<std::complex<double>>& b) {
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += std::norm(a[i] - b[i]);
    den += std::norm(b[i]);
  }
  return std::sqrt(num / den);
}

void device_paths() {
  scw_ctx* ctx = nullptr;
  expect(scw_create(&ctx, 0, 4) == SCW_OK, "scw_create(0)");
  if (!ctx) return;
  const int nx = 8, ny = 6, nz = 3, U = 5, V = 3;
  std::vector<double> n = sample_index(nx, ny, nz);
  scw_problem p = problem(n, nx, ny, nz, U, V);
  scw_solution* sol = nullptr;
  expect(scw_solve(ctx, &p, &sol) == SCW_OK, "scw_solve (stable route)");
  p.route = SCW_ROUTE_CONNECTION;
  scw_solution* sol_c = nullptr;
  expect(scw_solve(ctx, &p, &sol_c) == SCW_OK, "scw_solve (connection route)");
  p.route = SCW_ROUTE_STABLE;
  if (!sol || !sol_c) {
    scw_destroy(ctx);
    return;
  }
  scw_solution_info info;
  expect(scw_solution_info_get(sol, &info) == SCW_OK && info.M == U * V && info.L == nz,
         "scw_solution_info_get");
  // exterior coefficients of both routes agree
  const int M = U * V;
  std::vector<std::complex<double>> inc(3 * M), ref(3 * M), trn(3 * M), trn_c(3 * M);
  expect(scw_solution_exterior(sol, reinterpret_cast<double*>(inc.data()),
                               reinterpret_cast<double*>(ref.data()),
                               reinterpret_cast<double*>(trn.data())) == SCW_OK,
         "scw_solution_exterior");
  expect(scw_solution_exterior(sol_c, nullptr, nullptr,
                               reinterpret_cast<double*>(trn_c.data())) == SCW_OK,
         "scw_solution_exterior (connection)");
  expect(rel(trn_c, trn) < 1e-9, "routes agree on p_trn");
  // syntheses: FP64, FP32, and the no-allocation entry point against FP32
  scw_grid g{13, 7, 9, -0.3, 0.9};
  const size_t nvox = 3 * (size_t)g.fx * g.fy * g.fz;
  void *E64 = nullptr, *E32 = nullptr, *E32b = nullptr, *Et = nullptr;
  expect(hipMalloc(&E64, nvox * 16) == hipSuccess && hipMalloc(&E32, nvox * 8) == hipSuccess &&
             hipMalloc(&E32b, nvox * 8) == hipSuccess && hipMalloc(&Et, 6 * nvox * 8) == hipSuccess,
         "hipMalloc");
  expect(scw_synthesize(ctx, sol, &g, SCW_FP64, E64, nullptr) == SCW_OK, "synthesize FP64");
  expect(scw_synthesize(ctx, sol, &g, SCW_FP32, E32, nullptr) == SCW_OK, "synthesize FP32");
  expect(scw_synthesize_noalloc(ctx, sol, &g, SCW_FP32, E32b, nullptr) == SCW_OK,
         "synthesize without allocation");
  expect(scw_synthesize_tiled(ctx, sol, &g, 3, 2, SCW_FP32, Et, nullptr) == SCW_OK,
         "synthesize tiled");
  expect(hipDeviceSynchronize() == hipSuccess, "synchronize");
  std::vector<std::complex<double>> e64(nvox), e32(nvox);
  std::vector<std::complex<float>> f32(nvox), f32b(nvox);
  expect(hipMemcpy(e64.data(), E64, nvox * 16, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(f32.data(), E32, nvox * 8, hipMemcpyDeviceToHost) == hipSuccess &&
             hipMemcpy(f32b.data(), E32b, nvox * 8, hipMemcpyDeviceToHost) == hipSuccess,
         "copy back");
  std::vector<std::complex<double>> e32b(nvox);
  for (size_t i = 0; i < nvox; ++i) {
    e32[i] = std::complex<double>(f32[i]);
    e32b[i] = std::complex<double>(f32b[i]);
  }
  expect(rel(e32, e64) < 5e-6, "FP32 field against FP64");
  // the no-allocation path builds its tables on the device: FP32 agreement
  expect(rel(e32b, e32) < 1e-6, "no-allocation field agrees");
  // a batch of three problems with the device eigensolver
  std::vector<double> n2 = sample_index(nx, ny, 2);
  scw_problem batch[3] = {problem(n, nx, ny, nz, U, V), problem(n2, nx, ny, 2, 3, 3),
                          problem(n2, nx, ny, 2, 5, 5)};
  for (scw_problem& b : batch) b.eig = SCW_EIG_DEVICE;
  scw_solution* bs[3] = {nullptr, nullptr, nullptr};
  expect(scw_solve_batch(ctx, batch, 3, bs) == SCW_OK, "scw_solve_batch (device eigensolver)");
  if (bs[0]) {
    std::vector<std::complex<double>> trn_b(3 * M);
    expect(scw_solution_exterior(bs[0], nullptr, nullptr,
                                 reinterpret_cast<double*>(trn_b.data())) == SCW_OK,
           "batch exterior");
    expect(rel(trn_b, trn) < 1e-9, "batch member agrees with its single solve");
  }
  // a batched sweep over the three solutions (below the sample)
  scw_grid gb{16, 16, 2, 1.0, 1.2};
  scw_batch* batch_plan = nullptr;
  void* Eb = nullptr;
  expect(hipMalloc(&Eb, 3 * 3 * 16 * 16 * 2 * 8) == hipSuccess, "hipMalloc (batch)");
  if (bs[0] && bs[1] && bs[2]) {
    expect(scw_batch_plan(ctx, bs, 3, &gb, SCW_FP32, &batch_plan) == SCW_OK, "scw_batch_plan");
    if (batch_plan) {
      expect(scw_batch_launch(batch_plan, Eb, nullptr) == SCW_OK, "scw_batch_launch");
      scw_batch_free(batch_plan);
    }
  }
  // the surrogate, both arithmetics, on zero input
  scw_sur* sur = nullptr;
  expect(scw_sur_create(ctx, 8, 1, &sur) == SCW_OK, "scw_sur_create");
  if (sur) {
    void *x = nullptr, *out = nullptr;
    expect(hipMalloc(&x, 8 * 16 * 1024 * 4) == hipSuccess &&
               hipMalloc(&out, 8 * 3 * 225 * 8) == hipSuccess,
           "hipMalloc (surrogate)");
    expect(hipMemset(x, 0, 8 * 16 * 1024 * 4) == hipSuccess, "hipMemset");
    for (int bf16 = 0; bf16 < 2; ++bf16) {
      expect(scw_sur_set_compute(sur, bf16) == SCW_OK, "scw_sur_set_compute");
      expect(scw_sur_forward(sur, x, 8, out, nullptr) == SCW_OK, "scw_sur_forward");
    }
    expect(scw_sur_forward(sur, x, 9, out, nullptr) != SCW_OK, "surrogate batch bound");
    expect(hipDeviceSynchronize() == hipSuccess, "synchronize");
    (void)hipFree(x);
    (void)hipFree(out);
    scw_sur_free(sur);
  }
  // error paths of a solved problem and of bad problems
  scw_grid bad{0, 4, 4, 0.0, 1.0};
  expect(scw_synthesize(ctx, sol, &bad, SCW_FP32, E32, nullptr) != SCW_OK, "empty grid");
  scw_problem even = problem(n, nx, ny, nz, 4, 3);
  scw_solution* s_bad = nullptr;
  expect(scw_solve(ctx, &even, &s_bad) != SCW_OK && s_bad == nullptr, "even U rejected");
  for (scw_solution* b : bs) scw_solution_free(b);
  (void)hipFree(E64);
  (void)hipFree(E32);
  (void)hipFree(E32b);
  (void)hipFree(Et);
  (void)hipFree(Eb);
  scw_solution_free(sol);
  scw_solution_free(sol_c);
  scw_destroy(ctx);
}

}  // namespace

int main(int argc, char** argv) {
  const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
  validation_paths();
  if (gpu) device_paths();
  std::printf("abi_check %s: %d failure(s)\n", gpu ? "gpu" : "cpu", failures);
  return failures == 0 ? 0 : 1;
}

// Host driver of the batched device eigensolver (kernels_eig.hip) and its C
// ABI entry point scw_eig_batched: Hessenberg reduction, Schur form and the
// Schur factor's eigenvectors per matrix, then X = Z Y for the whole batch as
// one strided-batched complex GEMM and unit-norm columns.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <string>
#include <vector>

#include "scw_internal.h"

namespace scw {

int blas_handle(Context& ctx, hipStream_t st, void** out) {
  if (!ctx.blas) {
    rocblas_handle h = nullptr;
    const rocblas_status r = rocblas_create_handle(&h);
    if (r != rocblas_status_success)
      return fail(SCW_EHIP, std::string("rocblas_create_handle: ") + rocblas_status_to_string(r));
    ctx.blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(ctx.blas);
  const rocblas_status r = rocblas_set_stream(h, st);
  if (r != rocblas_status_success)
    return fail(SCW_EHIP, std::string("rocblas_set_stream: ") + rocblas_status_to_string(r));
  *out = h;
  return SCW_OK;
}

int device_eig_batched(Context& ctx, int n, int count, double* A, double* w, double* X,
                       hipStream_t st) {
  if (n < 1 || n > kEigMaxN || count < 1)
    return fail(SCW_EINVAL, "batched eigensolver: n must be in 1.." + std::to_string(kEigMaxN) +
                                " and count positive");
  if (!A || !w || !X) return fail(SCW_EINVAL, "batched eigensolver: null pointer");
  SCW_HIP(hipSetDevice(ctx.device));
  const size_t nn = (size_t)n * n;
  DevBuf dZ, dTt, dinfo;
  int rc;
  if ((rc = dZ.reserve(nn * 16 * count)) || (rc = dTt.reserve(nn * 16 * count)) ||
      (rc = dinfo.reserve(sizeof(int) * count)))
    return rc;
  SCW_HIP(launch_eig_hessenberg(n, count, A, dZ.as<double>(), st));
  SCW_HIP(launch_eig_schur(n, count, A, dZ.as<double>(), w, dinfo.as<int>(), st));
  // the Schur factor's eigenvectors overwrite A once it is copied row-major
  SCW_HIP(launch_eig_vectors(n, count, A, dTt.as<double>(), w, A, st));
  void* hv = nullptr;
  if ((rc = blas_handle(ctx, st, &hv))) return rc;
  rocblas_handle h = static_cast<rocblas_handle>(hv);
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  const rocblas_status bs = rocblas_zgemm_strided_batched(
      h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one,
      reinterpret_cast<const rocblas_double_complex*>(dZ.p), n, (rocblas_stride)nn,
      reinterpret_cast<const rocblas_double_complex*>(A), n, (rocblas_stride)nn, &zero,
      reinterpret_cast<rocblas_double_complex*>(X), n, (rocblas_stride)nn, count);
  if (bs != rocblas_status_success)
    return fail(SCW_EHIP, std::string("rocblas_zgemm_strided_batched: ") +
                              rocblas_status_to_string(bs));
  SCW_HIP(launch_eig_normalize(n, (long long)count * n, X, st));
  std::vector<int> info(count);
  SCW_HIP(hipMemcpyAsync(info.data(), dinfo.p, sizeof(int) * count, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < count; ++b)
    if (info[b])
      return fail(SCW_ELAPACK, "batched eigensolver: QR iteration of matrix " +
                                   std::to_string(b) + " did not converge at eigenvalue " +
                                   std::to_string(info[b] - 1));
  return SCW_OK;
}

}  // namespace scw

using namespace scw;

extern "C" int scw_eig_batched(scw_ctx* ctx, int n, int count, double* A_dev, double* w_dev,
                               double* X_dev, void* hip_stream) {
  if (!ctx) return fail(SCW_EINVAL, "null context");
  return device_eig_batched(ctx->c, n, count, A_dev, w_dev, X_dev,
                            reinterpret_cast<hipStream_t>(hip_stream));
}

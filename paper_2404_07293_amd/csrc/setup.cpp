// FP64 setup of one CWT problem (Sec. 3.1-3.4, Sec. 3.6): layer spectra and
// property-matrix blocks on the device, eigendecompositions and the boundary
// solve on the host (LAPACK), then the per-layer synthesis matrices on the
// device.
//
// Eigenproblem. D = [[0, A], [C, 0]] (Eq. 21) gives D^2 = diag(A C, C A), so
// the 4M eigenpairs of D come in pairs +-gamma_j with gamma_j^2 an eigenvalue
// of the 2M x 2M product A C. With A C x_j = gamma_j^2 x_j and y_j = C x_j /
// gamma_j, the forward eigenvector is [x_j; y_j] and the backward one
// [x_j; -y_j]. So Q = W = [[X, X], [Y, -Y]] with forward columns first.
//
// Boundary solve. Field at the top / bottom of layer l (Eqs. 24-26 in the
// top/bottom reading): W_l [a_l; E_l b_l] and W_l [E_l a_l; b_l], with
// E_l = diag(exp(i k gamma d)) (|E| <= 1), a_l forward amplitudes referenced at
// the top and b_l backward amplitudes referenced at the bottom.
//   SCW_ROUTE_STABLE: eliminate from the bottom up. Below layer l the field at
//   its bottom is F_{l+1} x_{l+1} (x = downward amplitudes of the region
//   below, F_{L+1} = transmitted plane waves). Solving W_l [E a_l; b_l] =
//   F_{l+1} x_{l+1} gives x_{l+1} = t_l E a_l and b_l = r_l E a_l, hence the
//   field at the top of layer l is F_l a_l with F_l = W_l [I; E r_l E]. At the
//   top surface, incident + reflected = F_1 a_1. Only E (never E^-1) appears.
//   SCW_ROUTE_CONNECTION: the paper's K = prod B_l T_l^-1 and the 6M x 6M
//   system C_t p_trn - K C_r p_ref = K C_i p_inc plus Gauss rows (Eq. 29).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <functional>
#include <mutex>
#include <thread>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "lapack.h"
#include "scw_internal.h"

namespace scw {

namespace {

using Mat = std::vector<zc>;  // column-major

// Limits of the connection route (Eqs. 27-29): reciprocal condition number of
// its 6M x 6M system and growth exponent of K.
constexpr double kConnectionMinRcond = 1e-13;
constexpr double kConnectionMaxGrowth = 25.0;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Runs fn(i) for i in [0, n) on up to `threads` host threads. Each worker
// pins MKL to one thread. Returns the first nonzero status.
int parallel_for(int n, int threads, const std::function<int(int)>& fn) {
  const Lapack& lp = lapack();
  std::atomic<int> next(0), status(0);
  std::mutex mu;
  std::string msg;
  auto worker = [&]() {
    if (lp.set_threads_local) lp.set_threads_local(1);
    for (;;) {
      int i = next.fetch_add(1);
      if (i >= n || status.load() != 0) break;
      int rc = fn(i);
      if (rc != 0) {
        int zero = 0;
        if (status.compare_exchange_strong(zero, rc)) {
          std::lock_guard<std::mutex> g(mu);
          msg = scw_last_error();
        }
      }
    }
    if (lp.set_threads_local) lp.set_threads_local(0);
  };
  int nt = std::max(1, std::min(threads, n));
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  // a worker's message lives in that worker's thread-local slot; copy it here
  if (status.load() != 0) set_error(status.load(), msg);
  return status.load();
}

struct Lin {
  const Lapack& lp;
  void gemm(char ta, char tb, int m, int n, int k, zc alpha, const zc* A, int lda,
            const zc* B, int ldb, zc beta, zc* C, int ldc) const {
    lp.zgemm(&ta, &tb, &m, &n, &k, &alpha, A, &lda, B, &ldb, &beta, C, &ldc);
  }
  int lu(int n, zc* A, std::vector<int>& piv) const {
    piv.resize(n);
    int info = 0;
    lp.zgetrf(&n, &n, A, &n, piv.data(), &info);
    return info;
  }
  int lu_solve(int n, int nrhs, const zc* LU, const std::vector<int>& piv, zc* B) const {
    int info = 0;
    char t = 'N';
    lp.zgetrs(&t, &n, &nrhs, LU, &n, piv.data(), B, &n, &info);
    return info;
  }
};

Mat identity(int n) {
  Mat I((size_t)n * n, zc(0));
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  return I;
}

// Transverse plane-wave field map for a half-space wave with s = (sx, sy, sigma):
// [px, py] -> [px, py, bx, by] with pz = -(sx px + sy py)/sigma (Eq. 14) and
// b = s x p. Returns the 2M x 2M H block (the E block is the identity).
Mat half_space_h(const Solution& s, const std::vector<zc>& sigma) {
  const int M = s.M, n2 = 2 * M;
  Mat H((size_t)n2 * n2, zc(0));
  for (int m = 0; m < M; ++m) {
    const zc sg = sigma[m];
    const double sx = s.sx[m], sy = s.sy[m];
    // bx = -(sx sy / sg) px - (sy^2/sg + sg) py ; by = (sg + sx^2/sg) px + (sx sy/sg) py
    H[(size_t)m * n2 + m] = -(sx * sy) / sg;
    H[(size_t)(M + m) * n2 + m] = -(sy * sy / sg + sg);
    H[(size_t)m * n2 + M + m] = sg + sx * sx / sg;
    H[(size_t)(M + m) * n2 + M + m] = (sx * sy) / sg;
  }
  return H;
}

// Full 4M x 3M map C(sigma) of Eq. 28 with the corrected sign of b_x:
// [px, py, pz] -> [px, py, sy pz - sigma py, sigma px - sx pz].
Mat c_map(const Solution& s, const std::vector<zc>& sigma) {
  const int M = s.M, n4 = 4 * M;
  Mat C((size_t)n4 * 3 * M, zc(0));
  auto at = [&](int r, int c) -> zc& { return C[(size_t)c * n4 + r]; };
  for (int m = 0; m < M; ++m) {
    at(m, m) = 1.0;
    at(M + m, M + m) = 1.0;
    at(2 * M + m, M + m) = -sigma[m];
    at(2 * M + m, 2 * M + m) = s.sy[m];
    at(3 * M + m, m) = sigma[m];
    at(3 * M + m, 2 * M + m) = -s.sx[m];
  }
  return C;
}

zc principal_sqrt_branch(zc lam, double tol_abs) {
  zc g = std::sqrt(lam);  // Re >= 0
  if (g.imag() < -tol_abs) g = -g;
  return g;
}

struct LayerHost {
  Mat A, C;           // property blocks (freed after use)
  Mat X, Y;           // E and H parts of the forward eigenvectors
  Mat Xlu, Ylu;       // LU factors (stable route)
  std::vector<int> Xpiv, Ypiv;
  std::vector<zc> gamma;   // forward branch, [2M]
  std::vector<zc> E;       // exp(i k gamma d)
};

// Forward branch gamma_j = sqrt(lam_j) of the eigenvalues lam of A C, the
// defectiveness check and E = exp(i k gamma d) of one layer.
int layer_gamma(const Solution& s, const zc* lam, LayerHost& h) {
  const int n2 = 2 * s.M;
  double gmax = 0;
  h.gamma.resize(n2);
  for (int j = 0; j < n2; ++j) gmax = std::max(gmax, std::sqrt(std::abs(lam[j])));
  // forward iff Im(gamma) > tol, or |Im| <= tol and Re > 0 (tol = 1e-12 max|gamma|)
  for (int j = 0; j < n2; ++j) h.gamma[j] = principal_sqrt_branch(lam[j], 1e-12 * gmax);
  double gmin = gmax;
  for (int j = 0; j < n2; ++j) gmin = std::min(gmin, std::abs(h.gamma[j]));
  if (gmin < 1e-9 * gmax)
    return fail(SCW_EDEFECTIVE, "near-defective property matrix: |gamma| ~ 0");
  h.E.resize(n2);
  for (int j = 0; j < n2; ++j)
    h.E[j] = std::exp(zc(0, 1) * s.k * h.gamma[j] * s.d);
  return SCW_OK;
}

int layer_eig(const Lin& lin, Solution& s, LayerHost& h) {
  const int n2 = 2 * s.M;
  Mat AC((size_t)n2 * n2);
  lin.gemm('N', 'N', n2, n2, n2, 1.0, h.A.data(), n2, h.C.data(), n2, 0.0, AC.data(), n2);
  std::vector<zc> lam(n2), work(1);
  std::vector<double> rwork(2 * n2);
  h.X.assign((size_t)n2 * n2, zc(0));
  int lwork = -1, info = 0, one = 1;
  zc dummy;
  char jl = 'N', jr = 'V';
  lin.lp.zgeev(&jl, &jr, &n2, AC.data(), &n2, lam.data(), &dummy, &one, h.X.data(), &n2,
               work.data(), &lwork, rwork.data(), &info);
  lwork = std::max(1, (int)work[0].real());
  work.resize(lwork);
  lin.lp.zgeev(&jl, &jr, &n2, AC.data(), &n2, lam.data(), &dummy, &one, h.X.data(), &n2,
               work.data(), &lwork, rwork.data(), &info);
  if (info != 0) return fail(SCW_ELAPACK, "zgeev info=" + std::to_string(info));
  int rc = layer_gamma(s, lam.data(), h);
  if (rc) return rc;
  // Y = C X diag(1/gamma)
  h.Y.assign((size_t)n2 * n2, zc(0));
  lin.gemm('N', 'N', n2, n2, n2, 1.0, h.C.data(), n2, h.X.data(), n2, 0.0, h.Y.data(), n2);
  for (int j = 0; j < n2; ++j) {
    const zc ig = 1.0 / h.gamma[j];
    zc* col = h.Y.data() + (size_t)j * n2;
    for (int r = 0; r < n2; ++r) col[r] *= ig;
  }
  Mat().swap(h.A);
  Mat().swap(h.C);
  return SCW_OK;
}

// ---------------------------------------------------------------- stable route
int top_surface(const Lin& lin, Solution& s, const Mat& Fe, const Mat& Fh, std::vector<zc>& a1);
void top_surface_finish(Solution& s, const std::vector<zc>& x, std::vector<zc>& a1);
std::vector<zc> top_surface_rhs(const Solution& s);
Mat reflected_h(const Solution& s);
std::vector<zc> incident_rhs(const Solution& s, const Mat& Ci);
void connection_finish(Solution& s, const std::vector<zc>& x, const std::vector<zc>& cip,
                       const Mat& Cr, std::vector<zc>& alpha1);
void transmitted(Solution& s, int kk, const zc* a);

int solve_stable(const Lin& lin, Solution& s, std::vector<LayerHost>& layers) {
  const int M = s.M, n2 = 2 * M, L = s.L;
  std::vector<Mat> t(L), r(L);
  // F_{L+1}: transmitted waves
  Mat Fe = identity(n2);
  Mat Fh = half_space_h(s, s.sz_bot);
  for (int l = L - 1; l >= 0; --l) {
    LayerHost& h = layers[l];
    Mat A1 = Fe, A2 = Fh;
    if (lin.lu_solve(n2, n2, h.Xlu.data(), h.Xpiv, A1.data()) != 0 ||
        lin.lu_solve(n2, n2, h.Ylu.data(), h.Ypiv, A2.data()) != 0)
      return fail(SCW_ELAPACK, "zgetrs failed in the stable route");
    Mat Gt((size_t)n2 * n2), Gb((size_t)n2 * n2);
    for (size_t i = 0; i < Gt.size(); ++i) {
      Gt[i] = 0.5 * (A1[i] + A2[i]);
      Gb[i] = 0.5 * (A1[i] - A2[i]);
    }
    std::vector<int> piv;
    if (lin.lu(n2, Gt.data(), piv) != 0)
      return fail(SCW_EILLCOND, "singular interface matrix in the stable route");
    t[l] = identity(n2);
    lin.lu_solve(n2, n2, Gt.data(), piv, t[l].data());
    r[l].assign((size_t)n2 * n2, zc(0));
    lin.gemm('N', 'N', n2, n2, n2, 1.0, Gb.data(), n2, t[l].data(), n2, 0.0, r[l].data(), n2);
    // F_l = [X (I + E r E); Y (I - E r E)]
    Mat P1((size_t)n2 * n2), P2((size_t)n2 * n2);
    for (int c = 0; c < n2; ++c)
      for (int rr = 0; rr < n2; ++rr) {
        const zc ere = h.E[rr] * r[l][(size_t)c * n2 + rr] * h.E[c];
        const zc id = (rr == c) ? zc(1) : zc(0);
        P1[(size_t)c * n2 + rr] = id + ere;
        P2[(size_t)c * n2 + rr] = id - ere;
      }
    Fe.assign((size_t)n2 * n2, zc(0));
    Fh.assign((size_t)n2 * n2, zc(0));
    lin.gemm('N', 'N', n2, n2, n2, 1.0, h.X.data(), n2, P1.data(), n2, 0.0, Fe.data(), n2);
    lin.gemm('N', 'N', n2, n2, n2, 1.0, h.Y.data(), n2, P2.data(), n2, 0.0, Fh.data(), n2);
  }
  std::vector<zc> a1;
  int rc = top_surface(lin, s, Fe, Fh, a1);
  if (rc) return rc;
  // back-substitution, one illumination at a time: b_l = r_l E a_l, a_{l+1} = t_l E a_l
  const int K = s.K;
  s.a.assign((size_t)K * L * n2, zc(0));
  s.b.assign((size_t)K * L * n2, zc(0));
  std::vector<zc> ea(n2), nxt(n2);
  for (int kk = 0; kk < K; ++kk) {
    std::vector<zc> a(a1.begin() + (size_t)kk * n2, a1.begin() + (size_t)(kk + 1) * n2);
    zc* ak = s.a.data() + (size_t)kk * L * n2;
    zc* bk = s.b.data() + (size_t)kk * L * n2;
    for (int l = 0; l < L; ++l) {
      std::copy(a.begin(), a.end(), ak + (size_t)l * n2);
      for (int j = 0; j < n2; ++j) ea[j] = layers[l].E[j] * a[j];
      lin.gemm('N', 'N', n2, 1, n2, 1.0, r[l].data(), n2, ea.data(), n2, 0.0,
               bk + (size_t)l * n2, n2);
      lin.gemm('N', 'N', n2, 1, n2, 1.0, t[l].data(), n2, ea.data(), n2, 0.0, nxt.data(), n2);
      a = nxt;
    }
    transmitted(s, kk, a.data());
  }
  return SCW_OK;
}

// p_trn of illumination kk from the downward amplitudes below the last layer.
void transmitted(Solution& s, int kk, const zc* a) {
  const int M = s.M;
  if (s.p_trn.size() != (size_t)s.K * 3 * M) s.p_trn.assign((size_t)s.K * 3 * M, zc(0));
  zc* ptrn = s.p_trn.data() + (size_t)kk * 3 * M;
  for (int m = 0; m < M; ++m) {
    const zc px = a[m], py = a[M + m];
    ptrn[m] = px;
    ptrn[M + m] = py;
    ptrn[2 * M + m] = -(s.sx[m] * px + s.sy[m] * py) / s.sz_bot[m];
  }
}

// Top surface of the stable route: F(-sz_top) rho - F_1 a_1 = -C_i p_inc for
// every illumination, with F_1 = [Fe; Fh]. Sets p_ref and returns a_1 as
// n2 x K (column-major).
// p_ref and the top-layer amplitudes a_1 of every illumination from the
// solution x = [p_ref,xy; a_1] (4M x K, column per illumination) of the
// top-surface system; p_ref,z from Gauss's law (Eq. 14).
void top_surface_finish(Solution& s, const std::vector<zc>& x, std::vector<zc>& a1) {
  const int M = s.M, n2 = 2 * M, n4 = 4 * M, K = s.K;
  s.p_ref.assign((size_t)K * 3 * M, zc(0));
  s.p_trn.assign((size_t)K * 3 * M, zc(0));
  a1.assign((size_t)K * n2, zc(0));
  for (int kk = 0; kk < K; ++kk) {
    const zc* rhs = x.data() + (size_t)kk * n4;
    zc* pref = s.p_ref.data() + (size_t)kk * 3 * M;
    for (int m = 0; m < M; ++m) {
      const zc px = rhs[m], py = rhs[M + m];
      pref[m] = px;
      pref[M + m] = py;
      pref[2 * M + m] = (s.sx[m] * px + s.sy[m] * py) / s.sz_top[m];
    }
    std::copy(rhs + n2, rhs + n4, a1.begin() + (size_t)kk * n2);
  }
}

// Right-hand sides -C_i p_inc of the top-surface system, 4M x K.
std::vector<zc> top_surface_rhs(const Solution& s) {
  const int M = s.M, n4 = 4 * M, K = s.K;
  Mat Ci = c_map(s, s.sz_top);
  std::vector<zc> rhs((size_t)n4 * K, zc(0));
  for (int kk = 0; kk < K; ++kk) {
    const zc* pin = s.p_inc.data() + (size_t)kk * 3 * M;
    zc* r = rhs.data() + (size_t)kk * n4;
    for (int c = 0; c < 3 * M; ++c)
      for (int rr = 0; rr < n4; ++rr) r[rr] -= Ci[(size_t)c * n4 + rr] * pin[c];
  }
  return rhs;
}

Mat reflected_h(const Solution& s) {
  std::vector<zc> msz(s.M);
  for (int m = 0; m < s.M; ++m) msz[m] = -s.sz_top[m];
  return half_space_h(s, msz);
}

int top_surface(const Lin& lin, Solution& s, const Mat& Fe, const Mat& Fh, std::vector<zc>& a1) {
  const int M = s.M, n2 = 2 * M, n4 = 4 * M;
  Mat Hr = reflected_h(s);
  Mat S((size_t)n4 * n4, zc(0));
  for (int c = 0; c < n2; ++c) {
    S[(size_t)c * n4 + c] = 1.0;
    for (int rr = 0; rr < n2; ++rr) S[(size_t)c * n4 + n2 + rr] = Hr[(size_t)c * n2 + rr];
    for (int rr = 0; rr < n2; ++rr) {
      S[(size_t)(n2 + c) * n4 + rr] = -Fe[(size_t)c * n2 + rr];
      S[(size_t)(n2 + c) * n4 + n2 + rr] = -Fh[(size_t)c * n2 + rr];
    }
  }
  std::vector<int> piv;
  if (lin.lu(n4, S.data(), piv) != 0)
    return fail(SCW_EILLCOND, "singular top-surface system in the stable route");
  // every illumination shares the factorisation
  std::vector<zc> x = top_surface_rhs(s);
  lin.lu_solve(n4, s.K, S.data(), piv, x.data());
  top_surface_finish(s, x, a1);
  return SCW_OK;
}

int connection_system(const Lin& lin, Solution& s, const Mat& K, std::vector<zc>& alpha1);

// ---------------------------------------------------------------- stable route on the device
// The same elimination in FP64 with rocSOLVER (LU with partial pivoting) and
// rocBLAS (complex GEMM) on the setup stream: per layer, from the bottom up,
// A1 = X^-1 Fe, A2 = Y^-1 Fh, G_t = (A1 + A2)/2, G_b = (A1 - A2)/2,
// t = G_t^-1, r = G_b t, Fe = X (I + E r E), Fh = Y (I - E r E). The LU
// factors of every layer's X and Y do not depend on the recursion and are
// computed first, in one batched call over the 2L matrices. The 4M x 4M
// top-surface system is solved on the host (top_surface); the
// back-substitution runs on the device for all illuminations at once.
namespace {
rocblas_double_complex* zp(const DevBuf& b, size_t off = 0) {
  return reinterpret_cast<rocblas_double_complex*>(b.as<zc>() + off);
}
}  // namespace

#define SCW_BLAS(call)                                                                   \
  do {                                                                                   \
    rocblas_status st_ = (call);                                                         \
    if (st_ != rocblas_status_success)                                                   \
      return fail(SCW_EHIP, std::string(#call) + ": " + rocblas_status_to_string(st_));  \
  } while (0)

// The stable route's 4M x 4M top-surface system on the device: assembled from
// the device F_1 (Fe, Fh), LU-factored by rocSOLVER, solved for every
// illumination; p_ref and a_1 as top_surface leaves them.
int top_surface_device(Context& ctx, Solution& s, const DevBuf& dFe, const DevBuf& dFh,
                       std::vector<zc>& a1) {
  const int M = s.M, n2 = 2 * M, n4 = 4 * M, K = s.K;
  hipStream_t st = ctx.setup_stream;
  void* hv = nullptr;
  int rc;
  if ((rc = blas_handle(ctx, st, &hv))) return rc;
  rocblas_handle h = static_cast<rocblas_handle>(hv);
  const Mat Hr = reflected_h(s);
  std::vector<zc> x = top_surface_rhs(s);
  DevBuf dHr, dS, drhs, dpiv, dinfo;
  if ((rc = dHr.reserve((size_t)n2 * n2 * 16)) || (rc = dS.reserve((size_t)n4 * n4 * 16)) ||
      (rc = drhs.reserve(x.size() * 16)) || (rc = dpiv.reserve((size_t)n4 * sizeof(rocblas_int))) ||
      (rc = dinfo.reserve(sizeof(rocblas_int))))
    return rc;
  SCW_HIP(hipMemcpyAsync(dHr.p, Hr.data(), Hr.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(drhs.p, x.data(), x.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(launch_top_system(dHr.as<double>(), dFe.as<double>(), dFh.as<double>(), n2,
                            dS.as<double>(), st));
  SCW_BLAS(rocsolver_zgetrf(h, n4, n4, zp(dS), n4, dpiv.as<rocblas_int>(), dinfo.as<rocblas_int>()));
  SCW_BLAS(rocsolver_zgetrs(h, rocblas_operation_none, n4, K, zp(dS), n4, dpiv.as<rocblas_int>(),
                            zp(drhs), n4));
  rocblas_int info = 0;
  SCW_HIP(hipMemcpyAsync(&info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost, st));
  SCW_HIP(hipMemcpyAsync(x.data(), drhs.p, x.size() * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  if (info != 0) return fail(SCW_EILLCOND, "singular top-surface system in the device elimination");
  top_surface_finish(s, x, a1);
  return SCW_OK;
}

// The connection route's 6M x 6M system (Eq. 29) on the device, from the
// device product K: assembled, LU-factored and solved by rocSOLVER. Its
// 1-norm condition number is computed exactly (the norm of the explicit
// inverse, from the same factors) where the host route estimates it
// (zgecon); the same 1e-13 limit on its reciprocal applies.
int connection_system_device(Context& ctx, Solution& s, const DevBuf& dK,
                             std::vector<zc>& alpha1) {
  const int M = s.M, n4 = 4 * M, n6 = 6 * M, nk = s.K;
  hipStream_t st = ctx.setup_stream;
  void* hv = nullptr;
  int rc;
  if ((rc = blas_handle(ctx, st, &hv))) return rc;
  rocblas_handle h = static_cast<rocblas_handle>(hv);
  std::vector<zc> msz(M);
  for (int m = 0; m < M; ++m) msz[m] = -s.sz_top[m];
  const Mat Ci = c_map(s, s.sz_top), Cr = c_map(s, msz), Ct = c_map(s, s.sz_bot);
  const std::vector<zc> cip = incident_rhs(s, Ci);
  const size_t n43 = (size_t)n4 * 3 * M, nn6 = (size_t)n6 * n6;
  DevBuf dCr, dCt, dKCr, dsx, dsy, dszt, dszb, dA, dInv, dnorm, dcip, drhs, dpiv, dinfo;
  if ((rc = dCr.reserve(n43 * 16)) || (rc = dCt.reserve(n43 * 16)) ||
      (rc = dKCr.reserve(n43 * 16)) || (rc = dsx.reserve((size_t)M * 8)) ||
      (rc = dsy.reserve((size_t)M * 8)) || (rc = dszt.reserve((size_t)M * 16)) ||
      (rc = dszb.reserve((size_t)M * 16)) || (rc = dA.reserve(nn6 * 16)) ||
      (rc = dInv.reserve(nn6 * 16)) || (rc = dnorm.reserve((size_t)n6 * 8 * 2)) ||
      (rc = dcip.reserve(cip.size() * 16)) || (rc = drhs.reserve((size_t)n6 * nk * 16)) ||
      (rc = dpiv.reserve((size_t)n6 * sizeof(rocblas_int))) ||
      (rc = dinfo.reserve(sizeof(rocblas_int))))
    return rc;
  SCW_HIP(hipMemcpyAsync(dCr.p, Cr.data(), n43 * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(dCt.p, Ct.data(), n43 * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(dsx.p, s.sx.data(), (size_t)M * 8, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(dsy.p, s.sy.data(), (size_t)M * 8, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(dszt.p, s.sz_top.data(), (size_t)M * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(dszb.p, s.sz_bot.data(), (size_t)M * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(dcip.p, cip.data(), cip.size() * 16, hipMemcpyHostToDevice, st));
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  const rocblas_operation N = rocblas_operation_none;
  SCW_BLAS(rocblas_zgemm(h, N, N, n4, 3 * M, n4, &one, zp(dK), n4, zp(dCr), n4, &zero, zp(dKCr),
                         n4));
  SCW_HIP(launch_connection_system(dKCr.as<double>(), dCt.as<double>(), dsx.as<double>(),
                                   dsy.as<double>(), dszt.as<double>(), dszb.as<double>(), M,
                                   dA.as<double>(), st));
  double* colsum = dnorm.as<double>();
  SCW_HIP(launch_col_abs_sum(dA.as<double>(), n6, colsum, st));
  SCW_BLAS(rocsolver_zgetrf(h, n6, n6, zp(dA), n6, dpiv.as<rocblas_int>(), dinfo.as<rocblas_int>()));
  SCW_HIP(launch_eye(dInv.as<double>(), n6, st));
  SCW_BLAS(rocsolver_zgetrs(h, N, n6, n6, zp(dA), n6, dpiv.as<rocblas_int>(), zp(dInv), n6));
  SCW_HIP(launch_col_abs_sum(dInv.as<double>(), n6, colsum + n6, st));
  // rhs = [K C_i p_inc; 0], every illumination
  SCW_HIP(hipMemsetAsync(drhs.p, 0, (size_t)n6 * nk * 16, st));
  SCW_BLAS(rocblas_zgemm(h, N, N, n4, nk, n4, &one, zp(dK), n4, zp(dcip), n4, &zero, zp(drhs),
                         n6));
  SCW_BLAS(rocsolver_zgetrs(h, N, n6, nk, zp(dA), n6, dpiv.as<rocblas_int>(), zp(drhs), n6));
  std::vector<double> sums(2 * (size_t)n6);
  std::vector<zc> x((size_t)n6 * nk);
  rocblas_int info = 0;
  SCW_HIP(hipMemcpyAsync(&info, dinfo.p, sizeof(info), hipMemcpyDeviceToHost, st));
  SCW_HIP(hipMemcpyAsync(sums.data(), dnorm.p, sums.size() * 8, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipMemcpyAsync(x.data(), drhs.p, x.size() * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  if (info != 0) return fail(SCW_EILLCOND, "singular 6M x 6M connection system");
  double anorm = 0, inorm = 0;
  for (int c = 0; c < n6; ++c) {
    anorm = std::max(anorm, sums[c]);
    inorm = std::max(inorm, sums[n6 + c]);
  }
  const double rcond = (anorm > 0 && inorm > 0 && std::isfinite(inorm)) ? 1.0 / (anorm * inorm)
                                                                          : 0.0;
  s.info.connection_rcond = rcond;
  if (!(rcond >= kConnectionMinRcond))
    return fail(SCW_EILLCOND, "connection system is ill-conditioned (rcond " +
                                  std::to_string(rcond) + " < 1e-13)");
  connection_finish(s, x, cip, Cr, alpha1);
  return SCW_OK;
}

int solve_stable_device(Context& ctx, const Lin& lin, Solution& s,
                        std::vector<LayerHost>& layers) {
  const int M = s.M, n2 = 2 * M, L = s.L, K = s.K;
  const size_t nn = (size_t)n2 * n2;
  hipStream_t st = ctx.setup_stream;
  if (!ctx.blas) {
    rocblas_handle h = nullptr;
    SCW_BLAS(rocblas_create_handle(&h));
    ctx.blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(ctx.blas);
  SCW_BLAS(rocblas_set_stream(h, st));
  // XY: X_l, Y_l of every layer at 2l, 2l + 1; XYlu: their LU factors
  DevBuf dXY, dXYlu, dFe, dFh, dA1, dA2, dP1, dP2, dT, dR, dE, dpiv, dxypiv, dinfo;
  int rc;
  if ((rc = dXY.reserve(nn * 16 * 2 * L)) || (rc = dXYlu.reserve(nn * 16 * 2 * L)) ||
      (rc = dFe.reserve(nn * 16)) || (rc = dFh.reserve(nn * 16)) ||
      (rc = dA1.reserve(nn * 16)) || (rc = dA2.reserve(nn * 16)) || (rc = dP1.reserve(nn * 16)) ||
      (rc = dP2.reserve(nn * 16)) || (rc = dT.reserve(nn * 16 * L)) ||
      (rc = dR.reserve(nn * 16 * L)) || (rc = dE.reserve((size_t)L * n2 * 16)) ||
      (rc = dpiv.reserve((size_t)n2 * sizeof(rocblas_int))) ||
      (rc = dxypiv.reserve((size_t)2 * L * n2 * sizeof(rocblas_int))) ||
      (rc = dinfo.reserve((size_t)3 * L * sizeof(rocblas_int))))
    return rc;
  for (int l = 0; l < L; ++l) {
    SCW_HIP(hipMemcpyAsync(dE.as<zc>() + (size_t)l * n2, layers[l].E.data(), n2 * 16,
                           hipMemcpyHostToDevice, st));
    SCW_HIP(hipMemcpyAsync(dXY.as<zc>() + (size_t)(2 * l) * nn, layers[l].X.data(), nn * 16,
                           hipMemcpyHostToDevice, st));
    SCW_HIP(hipMemcpyAsync(dXY.as<zc>() + (size_t)(2 * l + 1) * nn, layers[l].Y.data(), nn * 16,
                           hipMemcpyHostToDevice, st));
  }
  SCW_HIP(hipMemcpyAsync(dXYlu.p, dXY.p, nn * 16 * 2 * L, hipMemcpyDeviceToDevice, st));
  SCW_HIP(launch_eye(dFe.as<double>(), n2, st));
  const Mat Fh0 = half_space_h(s, s.sz_bot);
  SCW_HIP(hipMemcpyAsync(dFh.p, Fh0.data(), nn * 16, hipMemcpyHostToDevice, st));
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  rocblas_int* info = dinfo.as<rocblas_int>();  // [0, 2L): X, Y of each layer; [2L, 3L): G_t
  rocblas_int* piv = dpiv.as<rocblas_int>();
  rocblas_int* xypiv = dxypiv.as<rocblas_int>();
  const rocblas_operation N = rocblas_operation_none;
  SCW_BLAS(rocsolver_zgetrf_strided_batched(h, n2, n2, zp(dXYlu), n2, (rocblas_stride)nn, xypiv,
                                            (rocblas_stride)n2, info, 2 * L));
  for (int l = L - 1; l >= 0; --l) {
    rocblas_double_complex* Xl = zp(dXY, (size_t)(2 * l) * nn);
    rocblas_double_complex* Yl = zp(dXY, (size_t)(2 * l + 1) * nn);
    SCW_HIP(hipMemcpyAsync(dA1.p, dFe.p, nn * 16, hipMemcpyDeviceToDevice, st));
    SCW_HIP(hipMemcpyAsync(dA2.p, dFh.p, nn * 16, hipMemcpyDeviceToDevice, st));
    // A1 = X^-1 Fe, A2 = Y^-1 Fh with the factors of the batched call
    SCW_BLAS(rocsolver_zgetrs(h, N, n2, n2, zp(dXYlu, (size_t)(2 * l) * nn), n2,
                              xypiv + (size_t)(2 * l) * n2, zp(dA1), n2));
    SCW_BLAS(rocsolver_zgetrs(h, N, n2, n2, zp(dXYlu, (size_t)(2 * l + 1) * nn), n2,
                              xypiv + (size_t)(2 * l + 1) * n2, zp(dA2), n2));
    // G_t, G_b in place; t = G_t^-1; r = G_b t
    SCW_HIP(launch_half_sum_diff(dA1.as<double>(), dA2.as<double>(), (long long)nn, st));
    zc* tl = dT.as<zc>() + (size_t)l * nn;
    zc* rl = dR.as<zc>() + (size_t)l * nn;
    SCW_HIP(launch_eye(reinterpret_cast<double*>(tl), n2, st));
    SCW_BLAS(rocsolver_zgetrf(h, n2, n2, zp(dA1), n2, piv, info + 2 * L + l));
    SCW_BLAS(rocsolver_zgetrs(h, N, n2, n2, zp(dA1), n2, piv,
                              reinterpret_cast<rocblas_double_complex*>(tl), n2));
    SCW_BLAS(rocblas_zgemm(h, N, N, n2, n2, n2, &one, zp(dA2), n2,
                           reinterpret_cast<rocblas_double_complex*>(tl), n2, &zero,
                           reinterpret_cast<rocblas_double_complex*>(rl), n2));
    // F_l = [X (I + E r E); Y (I - E r E)]
    SCW_HIP(launch_i_pm_ere(reinterpret_cast<double*>(rl), dE.as<double>() + (size_t)l * n2 * 2,
                            n2, dP1.as<double>(), dP2.as<double>(), st));
    SCW_BLAS(rocblas_zgemm(h, N, N, n2, n2, n2, &one, Xl, n2, zp(dP1), n2, &zero, zp(dFe), n2));
    SCW_BLAS(rocblas_zgemm(h, N, N, n2, n2, n2, &one, Yl, n2, zp(dP2), n2, &zero, zp(dFh), n2));
  }
  std::vector<rocblas_int> hinfo(3 * L);
  SCW_HIP(hipMemcpyAsync(hinfo.data(), info, hinfo.size() * sizeof(rocblas_int),
                         hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < 3 * L; ++i)
    if (hinfo[i] != 0)
      return fail(i >= 2 * L ? SCW_EILLCOND : SCW_EDEFECTIVE,
                  i >= 2 * L ? "singular interface matrix in the device elimination (layer " +
                                   std::to_string(i - 2 * L) + ")"
                             : "eigenvector matrix is singular (layer " + std::to_string(i / 2) +
                                   ")");
  std::vector<zc> a1;
  if ((rc = top_surface_device(ctx, s, dFe, dFh, a1))) return rc;
  // back-substitution of all illuminations: columns of n2 x K blocks
  DevBuf dAc, dEA, dAs, dBs;
  const size_t nk = (size_t)n2 * K;
  if ((rc = dAc.reserve(nk * 16)) || (rc = dEA.reserve(nk * 16)) ||
      (rc = dAs.reserve(nk * 16 * L)) || (rc = dBs.reserve(nk * 16 * L)))
    return rc;
  SCW_HIP(hipMemcpyAsync(dAc.p, a1.data(), nk * 16, hipMemcpyHostToDevice, st));
  for (int l = 0; l < L; ++l) {
    SCW_HIP(hipMemcpyAsync(dAs.as<zc>() + (size_t)l * nk, dAc.p, nk * 16, hipMemcpyDeviceToDevice,
                           st));
    SCW_HIP(launch_scale_rows(dE.as<double>() + (size_t)l * n2 * 2, dAc.as<double>(), n2, K,
                              dEA.as<double>(), st));
    SCW_BLAS(rocblas_zgemm(h, N, N, n2, K, n2, &one,
                           reinterpret_cast<rocblas_double_complex*>(dR.as<zc>() + (size_t)l * nn),
                           n2, zp(dEA), n2, &zero, zp(dBs, (size_t)l * nk), n2));
    SCW_BLAS(rocblas_zgemm(h, N, N, n2, K, n2, &one,
                           reinterpret_cast<rocblas_double_complex*>(dT.as<zc>() + (size_t)l * nn),
                           n2, zp(dEA), n2, &zero, zp(dAc), n2));
  }
  std::vector<zc> As(nk * L), Bs(nk * L), last(nk);
  SCW_HIP(hipMemcpyAsync(As.data(), dAs.p, As.size() * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipMemcpyAsync(Bs.data(), dBs.p, Bs.size() * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipMemcpyAsync(last.data(), dAc.p, nk * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  // [L][K][n2] on the device -> [K][L][n2]
  s.a.assign((size_t)K * L * n2, zc(0));
  s.b.assign((size_t)K * L * n2, zc(0));
  for (int l = 0; l < L; ++l)
    for (int kk = 0; kk < K; ++kk) {
      std::copy(As.begin() + (size_t)l * nk + (size_t)kk * n2,
                As.begin() + (size_t)l * nk + (size_t)(kk + 1) * n2,
                s.a.begin() + ((size_t)kk * L + l) * n2);
      std::copy(Bs.begin() + (size_t)l * nk + (size_t)kk * n2,
                Bs.begin() + (size_t)l * nk + (size_t)(kk + 1) * n2,
                s.b.begin() + ((size_t)kk * L + l) * n2);
    }
  for (int kk = 0; kk < K; ++kk) transmitted(s, kk, last.data() + (size_t)kk * n2);
  return SCW_OK;
}
// The connection route with its per-layer work on the device: T_l and B_l
// from X, Y, E, T_l = LU (kept per layer with its pivots), M_l = B_l T_l^-1,
// K = M_L ... M_1; the 6M x 6M system on the host (connection_system); then
// alpha_l = T_l^-1 B_{l-1} alpha_{l-1} for all illuminations on the device.
int solve_connection_device(Context& ctx, const Lin& lin, Solution& s,
                            std::vector<LayerHost>& layers) {
  const int M = s.M, n2 = 2 * M, n4 = 4 * M, L = s.L, nk = s.K;
  const size_t nn = (size_t)n2 * n2, nn4 = (size_t)n4 * n4;
  hipStream_t st = ctx.setup_stream;
  if (!ctx.blas) {
    rocblas_handle h = nullptr;
    SCW_BLAS(rocblas_create_handle(&h));
    ctx.blas = h;
  }
  rocblas_handle h = static_cast<rocblas_handle>(ctx.blas);
  SCW_BLAS(rocblas_set_stream(h, st));
  DevBuf dX, dY, dE, dT, dB, dTi, dMk, dK, dK2, dpiv, dinfo;
  int rc;
  if ((rc = dX.reserve(nn * 16)) || (rc = dY.reserve(nn * 16)) ||
      (rc = dE.reserve((size_t)L * n2 * 16)) || (rc = dT.reserve(nn4 * 16 * L)) ||
      (rc = dB.reserve(nn4 * 16 * L)) || (rc = dTi.reserve(nn4 * 16)) ||
      (rc = dMk.reserve(nn4 * 16)) || (rc = dK.reserve(nn4 * 16)) || (rc = dK2.reserve(nn4 * 16)) ||
      (rc = dpiv.reserve((size_t)L * n4 * sizeof(rocblas_int))) ||
      (rc = dinfo.reserve((size_t)L * sizeof(rocblas_int))))
    return rc;
  for (int l = 0; l < L; ++l)
    SCW_HIP(hipMemcpyAsync(dE.as<zc>() + (size_t)l * n2, layers[l].E.data(), n2 * 16,
                           hipMemcpyHostToDevice, st));
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  const rocblas_operation N = rocblas_operation_none;
  rocblas_int* info = dinfo.as<rocblas_int>();
  auto piv = [&](int l) { return dpiv.as<rocblas_int>() + (size_t)l * n4; };
  auto Tl = [&](int l) { return zp(dT, (size_t)l * nn4); };
  auto Bl = [&](int l) { return zp(dB, (size_t)l * nn4); };
  SCW_HIP(launch_eye(dK.as<double>(), n4, st));
  for (int l = 0; l < L; ++l) {
    SCW_HIP(hipMemcpyAsync(dX.p, layers[l].X.data(), nn * 16, hipMemcpyHostToDevice, st));
    SCW_HIP(hipMemcpyAsync(dY.p, layers[l].Y.data(), nn * 16, hipMemcpyHostToDevice, st));
    SCW_HIP(launch_build_tb(dX.as<double>(), dY.as<double>(), dE.as<double>() + (size_t)l * n2 * 2,
                            n2, reinterpret_cast<double*>(Tl(l)),
                            reinterpret_cast<double*>(Bl(l)), st));
    SCW_BLAS(rocsolver_zgetrf(h, n4, n4, Tl(l), n4, piv(l), info + l));
    SCW_HIP(launch_eye(dTi.as<double>(), n4, st));
    SCW_BLAS(rocsolver_zgetrs(h, N, n4, n4, Tl(l), n4, piv(l), zp(dTi), n4));
    SCW_BLAS(rocblas_zgemm(h, N, N, n4, n4, n4, &one, Bl(l), n4, zp(dTi), n4, &zero, zp(dMk), n4));
    SCW_BLAS(rocblas_zgemm(h, N, N, n4, n4, n4, &one, zp(dMk), n4, zp(dK), n4, &zero, zp(dK2), n4));
    std::swap(dK.p, dK2.p);
  }
  std::vector<rocblas_int> hinfo(L);
  SCW_HIP(hipMemcpyAsync(hinfo.data(), info, L * sizeof(rocblas_int), hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  for (int l = 0; l < L; ++l)
    if (hinfo[l] != 0)
      return fail(SCW_EILLCOND, "singular layer matrix T in the connection route (layer " +
                                    std::to_string(l) + ")");
  std::vector<zc> alpha1;
  if ((rc = connection_system_device(ctx, s, dK, alpha1))) return rc;
  // alpha recursion of all illuminations: n4 x K blocks
  DevBuf dAl, dTmp, dAs;
  const size_t n4k = (size_t)n4 * nk;
  if ((rc = dAl.reserve(n4k * 16)) || (rc = dTmp.reserve(n4k * 16)) ||
      (rc = dAs.reserve(n4k * 16 * L)))
    return rc;
  SCW_HIP(hipMemcpyAsync(dAl.p, alpha1.data(), n4k * 16, hipMemcpyHostToDevice, st));
  for (int l = 0; l < L; ++l) {
    if (l > 0) {
      SCW_BLAS(rocblas_zgemm(h, N, N, n4, nk, n4, &one, Bl(l - 1), n4, zp(dAl), n4, &zero,
                             zp(dTmp), n4));
      std::swap(dAl.p, dTmp.p);
    }
    SCW_BLAS(rocsolver_zgetrs(h, N, n4, nk, Tl(l), n4, piv(l), zp(dAl), n4));
    SCW_HIP(hipMemcpyAsync(dAs.as<zc>() + (size_t)l * n4k, dAl.p, n4k * 16,
                           hipMemcpyDeviceToDevice, st));
  }
  std::vector<zc> As(n4k * L);
  SCW_HIP(hipMemcpyAsync(As.data(), dAs.p, As.size() * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  s.a.assign((size_t)nk * L * n2, zc(0));
  s.b.assign((size_t)nk * L * n2, zc(0));
  for (int l = 0; l < L; ++l)
    for (int kk = 0; kk < nk; ++kk) {
      const zc* col = As.data() + (size_t)l * n4k + (size_t)kk * n4;
      std::copy(col, col + n2, s.a.begin() + ((size_t)kk * L + l) * n2);
      std::copy(col + n2, col + n4, s.b.begin() + ((size_t)kk * L + l) * n2);
    }
  return SCW_OK;
}


// ---------------------------------------------------------------- connection route
int connection_system(const Lin& lin, Solution& s, const Mat& K, std::vector<zc>& alpha1);

int solve_connection(const Lin& lin, Solution& s, std::vector<LayerHost>& layers, int threads) {
  const int M = s.M, n2 = 2 * M, n4 = 4 * M, L = s.L;
  std::vector<Mat> Tlu(L), Bm(L), Mk(L);
  std::vector<std::vector<int>> Tpiv(L);
  // T_l = W diag(I, E), B_l = W diag(E, I), M_l = B_l T_l^-1 (Eq. 27)
  int rc = parallel_for(L, threads, [&](int l) -> int {
    LayerHost& h = layers[l];
    Mat T((size_t)n4 * n4), B((size_t)n4 * n4);
    for (int c = 0; c < n2; ++c)
      for (int rr = 0; rr < n2; ++rr) {
        const zc x = h.X[(size_t)c * n2 + rr], y = h.Y[(size_t)c * n2 + rr];
        const zc e = h.E[c];
        // forward column c, backward column n2 + c
        T[(size_t)c * n4 + rr] = x;
        T[(size_t)c * n4 + n2 + rr] = y;
        T[(size_t)(n2 + c) * n4 + rr] = x * e;
        T[(size_t)(n2 + c) * n4 + n2 + rr] = -y * e;
        B[(size_t)c * n4 + rr] = x * e;
        B[(size_t)c * n4 + n2 + rr] = y * e;
        B[(size_t)(n2 + c) * n4 + rr] = x;
        B[(size_t)(n2 + c) * n4 + n2 + rr] = -y;
      }
    if (lin.lu(n4, T.data(), Tpiv[l]) != 0)
      return fail(SCW_EILLCOND, "singular layer matrix T in the connection route");
    Mat Ti = identity(n4);
    lin.lu_solve(n4, n4, T.data(), Tpiv[l], Ti.data());
    Mk[l].assign((size_t)n4 * n4, zc(0));
    lin.gemm('N', 'N', n4, n4, n4, 1.0, B.data(), n4, Ti.data(), n4, 0.0, Mk[l].data(), n4);
    Tlu[l] = std::move(T);
    Bm[l] = std::move(B);
    return 0;
  });
  if (rc) return rc;
  Mat K = identity(n4), tmp((size_t)n4 * n4);
  for (int l = 0; l < L; ++l) {
    lin.gemm('N', 'N', n4, n4, n4, 1.0, Mk[l].data(), n4, K.data(), n4, 0.0, tmp.data(), n4);
    K.swap(tmp);
    Mat().swap(Mk[l]);
  }
  std::vector<zc> alpha1;
  if ((rc = connection_system(lin, s, K, alpha1))) return rc;
  // alpha_l = T_l^-1 B_{l-1} alpha_{l-1}, one illumination at a time
  const int nk = s.K;
  s.a.assign((size_t)nk * L * n2, zc(0));
  s.b.assign((size_t)nk * L * n2, zc(0));
  std::vector<zc> nxt(n4);
  for (int kk = 0; kk < nk; ++kk) {
    std::vector<zc> alpha(alpha1.begin() + (size_t)kk * n4, alpha1.begin() + (size_t)(kk + 1) * n4);
    zc* ak = s.a.data() + (size_t)kk * L * n2;
    zc* bk = s.b.data() + (size_t)kk * L * n2;
    for (int l = 0; l < L; ++l) {
      if (l > 0) {
        lin.gemm('N', 'N', n4, 1, n4, 1.0, Bm[l - 1].data(), n4, alpha.data(), n4, 0.0,
                 nxt.data(), n4);
        alpha = nxt;
      }
      lin.lu_solve(n4, 1, Tlu[l].data(), Tpiv[l], alpha.data());
      std::copy(alpha.begin(), alpha.begin() + n2, ak + (size_t)l * n2);
      std::copy(alpha.begin() + n2, alpha.end(), bk + (size_t)l * n2);
    }
  }
  return SCW_OK;
}

// The 6M x 6M system of the connection route, C_t p_trn - K C_r p_ref =
// K C_i p_inc plus the Gauss rows (Eq. 29), for every illumination. Sets
// p_ref, p_trn and the reciprocal condition number, and returns
// alpha_1 = C_i p_inc + C_r p_ref as n4 x K (column-major).
// C_i p_inc of every illumination (4M x K).
std::vector<zc> incident_rhs(const Solution& s, const Mat& Ci) {
  const int M = s.M, n4 = 4 * M, K = s.K;
  std::vector<zc> cip((size_t)n4 * K, zc(0));
  for (int kk = 0; kk < K; ++kk) {
    const zc* pin = s.p_inc.data() + (size_t)kk * 3 * M;
    zc* r = cip.data() + (size_t)kk * n4;
    for (int c = 0; c < 3 * M; ++c)
      for (int rr = 0; rr < n4; ++rr) r[rr] += Ci[(size_t)c * n4 + rr] * pin[c];
  }
  return cip;
}

// p_ref, p_trn and alpha_1 = C_i p_inc + C_r p_ref (Sec. 2.5.4) from the
// solution x = [p_ref; p_trn] (6M x K) of the connection system.
void connection_finish(Solution& s, const std::vector<zc>& x, const std::vector<zc>& cip,
                       const Mat& Cr, std::vector<zc>& alpha1) {
  const int M = s.M, n4 = 4 * M, n6 = 6 * M, nk = s.K;
  s.p_ref.assign((size_t)nk * 3 * M, zc(0));
  s.p_trn.assign((size_t)nk * 3 * M, zc(0));
  alpha1.assign((size_t)nk * n4, zc(0));
  for (int kk = 0; kk < nk; ++kk) {
    const zc* r = x.data() + (size_t)kk * n6;
    zc* pref = s.p_ref.data() + (size_t)kk * 3 * M;
    std::copy(r, r + 3 * M, pref);
    std::copy(r + 3 * M, r + n6, s.p_trn.begin() + (size_t)kk * 3 * M);
    zc* al = alpha1.data() + (size_t)kk * n4;
    std::copy(cip.begin() + (size_t)kk * n4, cip.begin() + (size_t)(kk + 1) * n4, al);
    for (int c = 0; c < 3 * M; ++c)
      for (int rr = 0; rr < n4; ++rr) al[rr] += Cr[(size_t)c * n4 + rr] * pref[c];
  }
}

int connection_system(const Lin& lin, Solution& s, const Mat& K, std::vector<zc>& alpha1) {
  const int M = s.M, n4 = 4 * M, n6 = 6 * M;
  std::vector<zc> msz(M);
  for (int m = 0; m < M; ++m) msz[m] = -s.sz_top[m];
  Mat Ci = c_map(s, s.sz_top), Cr = c_map(s, msz), Ct = c_map(s, s.sz_bot);
  Mat KCr((size_t)n4 * 3 * M);
  lin.gemm('N', 'N', n4, 3 * M, n4, 1.0, K.data(), n4, Cr.data(), n4, 0.0, KCr.data(), n4);
  Mat A((size_t)n6 * n6, zc(0));
  for (int c = 0; c < 3 * M; ++c)
    for (int rr = 0; rr < n4; ++rr) {
      A[(size_t)c * n6 + rr] = -KCr[(size_t)c * n4 + rr];
      A[(size_t)(3 * M + c) * n6 + rr] = Ct[(size_t)c * n4 + rr];
    }
  for (int m = 0; m < M; ++m) {  // Gauss rows (Eq. 14)
    A[(size_t)m * n6 + n4 + m] = s.sx[m];
    A[(size_t)(M + m) * n6 + n4 + m] = s.sy[m];
    A[(size_t)(2 * M + m) * n6 + n4 + m] = -s.sz_top[m];
    A[(size_t)(3 * M + m) * n6 + n4 + M + m] = s.sx[m];
    A[(size_t)(4 * M + m) * n6 + n4 + M + m] = s.sy[m];
    A[(size_t)(5 * M + m) * n6 + n4 + M + m] = s.sz_bot[m];
  }
  char one = '1';
  std::vector<double> rw(2 * n6);
  const double anorm = lin.lp.zlange(&one, &n6, &n6, A.data(), &n6, rw.data());
  std::vector<int> piv;
  if (lin.lu(n6, A.data(), piv) != 0)
    return fail(SCW_EILLCOND, "singular 6M x 6M connection system");
  double rcond = 0;
  int info = 0;
  std::vector<zc> cw(2 * n6);
  lin.lp.zgecon(&one, &n6, A.data(), &n6, &anorm, &rcond, cw.data(), rw.data(), &info);
  s.info.connection_rcond = rcond;
  // condition number above 1e13: FP64 keeps fewer than three digits of the
  // coefficients, so the forced route reports it instead of answering
  if (!(rcond >= kConnectionMinRcond))
    return fail(SCW_EILLCOND, "connection system is ill-conditioned (rcond " +
                                  std::to_string(rcond) + " < 1e-13)");
  // every illumination shares the factorisation of A: rhs = [K C_i p_inc; 0]
  const int nk = s.K;
  std::vector<zc> cip = incident_rhs(s, Ci), x((size_t)n6 * nk, zc(0));
  for (int kk = 0; kk < nk; ++kk)
    lin.gemm('N', 'N', n4, 1, n4, 1.0, K.data(), n4, cip.data() + (size_t)kk * n4, n4, 0.0,
             x.data() + (size_t)kk * n6, n6);
  lin.lu_solve(n6, nk, A.data(), piv, x.data());
  connection_finish(s, x, cip, Cr, alpha1);
  return SCW_OK;
}

}  // namespace

void release_blas(Context& ctx) {
  if (ctx.blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(ctx.blas));
  ctx.blas = nullptr;
}

// ---------------------------------------------------------------- phases of a solve
// What a solve keeps between its steps, so that the device eigendecompositions
// of many problems can share launches (solve_problems).
struct PendingSolve {
  double t_start = 0;
  bool dev_eig = false;
  double device_eig_seconds = 0;
  std::vector<LayerHost> layers;
  DevBuf d_A, d_C;  // property blocks of every layer (device eigensolver only)
  DevBuf d_psi, d_u, d_v, d_sx, d_sy;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  PendingSolve() = default;
  PendingSolve(const PendingSolve&) = delete;
  PendingSolve& operator=(const PendingSolve&) = delete;
  ~PendingSolve() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

// ---------------------------------------------------------------- device eigensolver
// The layers of n problems of one truncation (2M x 2M products): every A C
// by one strided-batched GEMM, all of them eigendecomposed by the batched
// device eigensolver at once, gamma on the host, Y = C X diag(1/gamma) on the
// device; X, Y, gamma and E of every layer end in each problem's `layers` as
// layer_eig leaves them.
static int device_eig_group(Context& ctx, Solution** sols, PendingSolve** ps, int n) {
  const int n2 = 2 * sols[0]->M;
  const size_t nn = (size_t)n2 * n2;
  int total = 0;
  for (int i = 0; i < n; ++i) total += sols[i]->L;
  hipStream_t st = ctx.setup_stream;
  const double t0 = now_s();
  DevBuf cat_A, cat_C, d_AC, d_X, d_w, d_f;
  int rc;
  const DevBuf* A = &ps[0]->d_A;
  const DevBuf* C = &ps[0]->d_C;
  if (n > 1) {  // one contiguous batch
    if ((rc = cat_A.reserve(nn * 16 * total)) || (rc = cat_C.reserve(nn * 16 * total))) return rc;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      const size_t b = nn * 16 * sols[i]->L;
      SCW_HIP(hipMemcpyAsync(cat_A.as<char>() + off, ps[i]->d_A.p, b, hipMemcpyDeviceToDevice, st));
      SCW_HIP(hipMemcpyAsync(cat_C.as<char>() + off, ps[i]->d_C.p, b, hipMemcpyDeviceToDevice, st));
      off += b;
    }
    A = &cat_A;
    C = &cat_C;
  }
  if ((rc = d_AC.reserve(nn * 16 * total)) || (rc = d_X.reserve(nn * 16 * total)) ||
      (rc = d_w.reserve((size_t)n2 * 16 * total)) || (rc = d_f.reserve((size_t)n2 * 16 * total)))
    return rc;
  void* hv = nullptr;
  if ((rc = blas_handle(ctx, st, &hv))) return rc;
  rocblas_handle h = static_cast<rocblas_handle>(hv);
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  const rocblas_operation N = rocblas_operation_none;
  SCW_BLAS(rocblas_zgemm_strided_batched(h, N, N, n2, n2, n2, &one, zp(*A), n2,
                                         (rocblas_stride)nn, zp(*C), n2, (rocblas_stride)nn,
                                         &zero, zp(d_AC), n2, (rocblas_stride)nn, total));
  if ((rc = device_eig_batched(ctx, n2, total, d_AC.as<double>(), d_w.as<double>(),
                               d_X.as<double>(), st)))
    return rc;
  std::vector<zc> lam((size_t)n2 * total), f((size_t)n2 * total);
  SCW_HIP(hipMemcpyAsync(lam.data(), d_w.p, lam.size() * 16, hipMemcpyDeviceToHost, st));
  SCW_HIP(hipStreamSynchronize(st));
  size_t g = 0;  // global layer index
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < sols[i]->L; ++l, ++g) {
      LayerHost& lh = ps[i]->layers[l];
      if ((rc = layer_gamma(*sols[i], lam.data() + g * n2, lh))) return rc;
      for (int j = 0; j < n2; ++j) f[g * n2 + j] = 1.0 / lh.gamma[j];
    }
  SCW_HIP(hipMemcpyAsync(d_f.p, f.data(), f.size() * 16, hipMemcpyHostToDevice, st));
  SCW_BLAS(rocblas_zgemm_strided_batched(h, N, N, n2, n2, n2, &one, zp(*C), n2,
                                         (rocblas_stride)nn, zp(d_X), n2, (rocblas_stride)nn,
                                         &zero, zp(d_AC), n2, (rocblas_stride)nn, total));
  SCW_HIP(launch_eig_scale_cols(n2, (long long)n2 * total, d_f.as<double>(), d_AC.as<double>(),
                                st));
  g = 0;
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < sols[i]->L; ++l, ++g) {
      LayerHost& lh = ps[i]->layers[l];
      lh.X.resize(nn);
      lh.Y.resize(nn);
      SCW_HIP(hipMemcpyAsync(lh.X.data(), d_X.as<zc>() + g * nn, nn * 16, hipMemcpyDeviceToHost,
                             st));
      SCW_HIP(hipMemcpyAsync(lh.Y.data(), d_AC.as<zc>() + g * nn, nn * 16, hipMemcpyDeviceToHost,
                             st));
    }
  SCW_HIP(hipStreamSynchronize(st));
  const double dt = now_s() - t0;
  for (int i = 0; i < n; ++i) {
    ps[i]->d_A.release();
    ps[i]->d_C.release();
    ps[i]->device_eig_seconds = dt;
  }
  return SCW_OK;
}

#undef SCW_BLAS

// ---------------------------------------------------------------- driver
// Steps of a solve up to the eigendecompositions: validation, mode table,
// band coefficients and property blocks on the device (kept there for the
// device eigensolver, copied to `layers` for the host one), incident
// coefficients. `ps` keeps what the later steps need.
int solve_begin(Context& ctx, const scw_problem& p, Solution& s, int n_waves,
                const scw_plane_wave* waves, PendingSolve& ps) {
  ps.t_start = now_s();
  if (n_waves < 0 || (n_waves > 0 && !waves) || n_waves > 4096)
    return fail(SCW_EINVAL, "illumination count must be 0..4096 with a non-null list");
  if (p.nx < 1 || p.ny < 1 || p.nz < 1 || !p.n)
    return fail(SCW_EINVAL, "sample shape must be positive and n non-null");
  if (p.U < 1 || p.V < 1 || p.U % 2 == 0 || p.V % 2 == 0)
    return fail(SCW_EINVAL, "U and V must be odd and positive");
  if (!(p.px > 0) || !(p.py > 0) || !(p.pz > 0) || !(p.lambda > 0))
    return fail(SCW_EINVAL, "pitches and wavelength must be positive");
  if (!(p.n_top > 0)) return fail(SCW_EINVAL, "n_top must be positive");
  if (p.route < SCW_ROUTE_STABLE || p.route > SCW_ROUTE_CONNECTION_DEVICE)
    return fail(SCW_EINVAL, "unknown route");
  if (p.eig != SCW_EIG_HOST && p.eig != SCW_EIG_DEVICE)
    return fail(SCW_EINVAL, "unknown eigensolver placement");
  if (p.eig == SCW_EIG_DEVICE && 2LL * p.U * p.V > kEigMaxN)
    return fail(SCW_EINVAL, "device eigensolver needs 2 U V <= " + std::to_string(kEigMaxN));
  const bool image = !waves && (p.inc_ex || p.inc_ey);
  if (image && (p.inc_nx < 1 || p.inc_ny < 1))
    return fail(SCW_EINVAL, "incident image shape must be positive");
  if ((long long)p.U * p.V > 8192) return fail(SCW_EINVAL, "U*V above 8192");
  const Lapack& lp = lapack();
  if (!lp.ok) return fail(SCW_ELAPACK, "LAPACK unavailable: " + lp.error);

  s.U = p.U;
  s.V = p.V;
  s.M = p.U * p.V;
  s.L = p.nz;
  s.lam = p.lambda;
  s.k = 2.0 * M_PI / p.lambda;
  s.X = p.nx * p.px;
  s.Y = p.ny * p.py;
  s.d = p.pz;
  const int M = s.M, n2 = 2 * M, L = s.L, U = s.U, V = s.V;
  // Sec. 2.2 mode table and Eq. 6 spatial frequencies
  s.u.resize(M);
  s.v.resize(M);
  s.sx.resize(M);
  s.sy.resize(M);
  s.sz_top.resize(M);
  s.sz_bot.resize(M);
  const zc nbot(p.n_bot_re, p.n_bot_im);
  double min_sz = 1e300;
  for (int m = 0; m < M; ++m) {
    const int vv = m / U - V / 2;
    const int uu = m - (vv + V / 2) * U - U / 2;
    s.u[m] = uu;
    s.v[m] = vv;
    s.sx[m] = p.lambda * uu / s.X;
    s.sy[m] = p.lambda * vv / s.Y;
    const double st2 = s.sx[m] * s.sx[m] + s.sy[m] * s.sy[m];
    // Eq. 2 with the branch Im >= 0
    zc a = std::sqrt(zc(p.n_top * p.n_top - st2, 0.0));
    zc b = std::sqrt(nbot * nbot - st2);
    if (a.imag() < 0) a = -a;
    if (b.imag() < 0 || (b.imag() == 0 && b.real() < 0)) b = -b;
    s.sz_top[m] = a;
    s.sz_bot[m] = b;
    min_sz = std::min(min_sz, std::min(std::abs(a), std::abs(b)));
  }
  s.info.M = M;
  s.info.L = L;
  s.info.min_abs_sz = min_sz;
  if (min_sz < 1e-9) return fail(SCW_EGRAZING, "grazing spatial frequency in a half-space");

  SCW_HIP(hipSetDevice(ctx.device));
  hipStream_t st = ctx.setup_stream;
  SCW_HIP(hipEventCreate(&ps.ev0));
  SCW_HIP(hipEventCreate(&ps.ev1));
  hipEvent_t ev0 = ps.ev0, ev1 = ps.ev1;

  // ---- device: band coefficients of n^2 and 1/n^2 (Eqs. 11-12)
  const int nbu = 2 * U - 1, nbv = 2 * V - 1;
  const size_t nvox = (size_t)p.nx * p.ny * p.nz;
  DevBuf d_n, d_row, d_phi;
  DevBuf &d_psi = ps.d_psi, &d_u = ps.d_u, &d_v = ps.d_v, &d_sx = ps.d_sx, &d_sy = ps.d_sy;
  int rc;
  if ((rc = d_n.reserve(nvox * 16))) return rc;
  if ((rc = d_row.reserve((size_t)2 * L * p.ny * nbu * 16))) return rc;
  if ((rc = d_phi.reserve((size_t)L * nbv * nbu * 16))) return rc;
  if ((rc = d_psi.reserve((size_t)L * nbv * nbu * 16))) return rc;
  if ((rc = d_u.reserve(M * sizeof(int))) || (rc = d_v.reserve(M * sizeof(int))) ||
      (rc = d_sx.reserve(M * 8)) || (rc = d_sy.reserve(M * 8)))
    return rc;
  SCW_HIP(hipMemcpyAsync(d_n.p, p.n, nvox * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(d_u.p, s.u.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(d_v.p, s.v.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(d_sx.p, s.sx.data(), M * 8, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(d_sy.p, s.sy.data(), M * 8, hipMemcpyHostToDevice, st));
  SCW_HIP(hipEventRecord(ev0, st));
  SCW_HIP(launch_band_dft(d_n.as<double>(), L, p.ny, p.nx, U - 1, V - 1, true, true,
                          d_row.as<double>(), d_phi.as<double>(), d_psi.as<double>(), st));

  // ---- device: property blocks A, C per layer chunk, copied to the host (or,
  // for the device eigensolver, every layer kept on the device)
  std::vector<LayerHost>& layers = ps.layers;
  layers.assign(L, LayerHost{});
  const size_t blk = (size_t)n2 * n2;
  const bool dev_eig = p.eig == SCW_EIG_DEVICE;
  const int chunk = dev_eig ? L
                            : (int)std::max<size_t>(
                                  1, std::min<size_t>(L, (size_t)(1u << 30) / (blk * 32)));
  ps.dev_eig = dev_eig;
  DevBuf &d_A = ps.d_A, &d_C = ps.d_C;
  if ((rc = d_A.reserve(blk * 16 * chunk)) || (rc = d_C.reserve(blk * 16 * chunk))) return rc;
  float asm_ms = 0;
  for (int l0 = 0; l0 < L; l0 += chunk) {
    const int nl = std::min(chunk, L - l0);
    SCW_HIP(launch_assemble_ac(d_phi.as<double>() + (size_t)l0 * nbv * nbu * 2,
                               d_psi.as<double>() + (size_t)l0 * nbv * nbu * 2, d_u.as<int>(),
                               d_v.as<int>(), d_sx.as<double>(), d_sy.as<double>(), U, V, nl,
                               d_A.as<double>(), d_C.as<double>(), st));
    if (l0 == 0) {
      SCW_HIP(hipEventRecord(ev1, st));
      SCW_HIP(hipEventSynchronize(ev1));
      SCW_HIP(hipEventElapsedTime(&asm_ms, ev0, ev1));
    }
    for (int l = l0; l < l0 + nl && !dev_eig; ++l) {
      layers[l].A.resize(blk);
      layers[l].C.resize(blk);
      SCW_HIP(hipMemcpyAsync(layers[l].A.data(), d_A.as<char>() + (size_t)(l - l0) * blk * 16,
                             blk * 16, hipMemcpyDeviceToHost, st));
      SCW_HIP(hipMemcpyAsync(layers[l].C.data(), d_C.as<char>() + (size_t)(l - l0) * blk * 16,
                             blk * 16, hipMemcpyDeviceToHost, st));
    }
    SCW_HIP(hipStreamSynchronize(st));
  }
  s.info.assembly_device_ms = asm_ms * ((double)L / std::min(chunk, L));
  if (!dev_eig) {
    d_A.release();
    d_C.release();
  }

  // ---- incident coefficients (Sec. 2.3): in-band DFT of the images / plane
  // wave, or one plane wave per illumination (illumination-major [K][3M])
  s.K = waves ? n_waves : 1;
  s.p_inc.assign((size_t)s.K * 3 * M, zc(0));
  if (waves) {
    for (int kk = 0; kk < s.K; ++kk) {
      int hit = -1;
      for (int m = 0; m < M; ++m)
        if (s.u[m] == waves[kk].u && s.v[m] == waves[kk].v) hit = m;
      if (hit < 0)
        return fail(SCW_EINVAL, "illumination " + std::to_string(kk) +
                                    ": plane-wave frequency outside the U x V band");
      s.p_inc[(size_t)kk * 3 * M + hit] = zc(waves[kk].ex[0], waves[kk].ex[1]);
      s.p_inc[(size_t)kk * 3 * M + M + hit] = zc(waves[kk].ey[0], waves[kk].ey[1]);
    }
  } else if (image) {
    const int hu = U / 2, hv = V / 2;
    const size_t npx = (size_t)p.inc_nx * p.inc_ny;
    DevBuf d_img, d_irow, d_ic;
    if ((rc = d_img.reserve(npx * 16)) || (rc = d_irow.reserve((size_t)p.inc_ny * U * 16)) ||
        (rc = d_ic.reserve((size_t)M * 16)))
      return rc;
    std::vector<zc> coef(M);
    for (int comp = 0; comp < 2; ++comp) {
      const double* img = comp == 0 ? p.inc_ex : p.inc_ey;
      if (!img) continue;
      SCW_HIP(hipMemcpyAsync(d_img.p, img, npx * 16, hipMemcpyHostToDevice, st));
      SCW_HIP(launch_band_dft(d_img.as<double>(), 1, p.inc_ny, p.inc_nx, hu, hv, false, false,
                              d_irow.as<double>(), d_ic.as<double>(), nullptr, st));
      SCW_HIP(hipMemcpyAsync(coef.data(), d_ic.p, (size_t)M * 16, hipMemcpyDeviceToHost, st));
      SCW_HIP(hipStreamSynchronize(st));
      // the band is laid out [v + hv][u + hu], which is the mode order m
      for (int m = 0; m < M; ++m) s.p_inc[comp * M + m] = coef[m];
    }
  } else {
    int hit = -1;
    for (int m = 0; m < M; ++m)
      if (s.u[m] == p.pw_u && s.v[m] == p.pw_v) hit = m;
    if (hit < 0) return fail(SCW_EINVAL, "plane-wave frequency outside the U x V band");
    s.p_inc[hit] = zc(p.pw_ex[0], p.pw_ex[1]);
    s.p_inc[M + hit] = zc(p.pw_ey[0], p.pw_ey[1]);
  }
  for (int kk = 0; kk < s.K; ++kk) {  // Gauss (Eq. 14)
    zc* pin = s.p_inc.data() + (size_t)kk * 3 * M;
    for (int m = 0; m < M; ++m)
      pin[2 * M + m] = -(s.sx[m] * pin[m] + s.sy[m] * pin[M + m]) / s.sz_top[m];
  }
  return SCW_OK;
}

// Steps after the eigendecompositions' device part: host eigendecompositions
// (SCW_EIG_HOST), LU of the eigenvector blocks for the host stable route,
// growth exponent, boundary solve, synthesis matrices and device uploads.
int solve_finish(Context& ctx, const scw_problem& p, Solution& s, PendingSolve& ps) {
  const Lapack& lp = lapack();
  const Lin lin{lp};
  const int M = s.M, n2 = 2 * M, L = s.L, U = s.U, V = s.V;
  const int nbu = 2 * U - 1, nbv = 2 * V - 1;
  const size_t blk = (size_t)n2 * n2;
  const bool dev_eig = ps.dev_eig;
  std::vector<LayerHost>& layers = ps.layers;
  DevBuf &d_psi = ps.d_psi, &d_u = ps.d_u, &d_v = ps.d_v, &d_sx = ps.d_sx, &d_sy = ps.d_sy;
  hipStream_t st = ctx.setup_stream;
  int rc;
  // ---- eigendecompositions (Sec. 3.2, Sec. 4.2): on the host, one layer per
  // worker, or every layer at once by the device eigensolver
  const double t_eig = now_s();
  const bool stable = p.route == SCW_ROUTE_STABLE;
  ps.d_A.release();
  ps.d_C.release();
  rc = parallel_for(L, ctx.host_threads, [&](int l) -> int {
    if (!dev_eig) {
      int r = layer_eig(lin, s, layers[l]);
      if (r) return r;
    }
    if (stable) {
      layers[l].Xlu = layers[l].X;
      layers[l].Ylu = layers[l].Y;
      if (lin.lu(n2, layers[l].Xlu.data(), layers[l].Xpiv) != 0 ||
          lin.lu(n2, layers[l].Ylu.data(), layers[l].Ypiv) != 0)
        return fail(SCW_EDEFECTIVE, "eigenvector matrix is singular");
    }
    return 0;
  });
  if (rc) return rc;
  s.info.eig_seconds = (now_s() - t_eig) + ps.device_eig_seconds;
  double gmin_rel = 1e300, growth = 0;
  s.gamma.resize((size_t)L * n2);
  for (int l = 0; l < L; ++l) {
    double gmax = 0, gmin = 1e300, imax = 0;
    for (int j = 0; j < n2; ++j) {
      const zc g = layers[l].gamma[j];
      s.gamma[(size_t)l * n2 + j] = g;
      gmax = std::max(gmax, std::abs(g));
      gmin = std::min(gmin, std::abs(g));
      imax = std::max(imax, g.imag());
    }
    gmin_rel = std::min(gmin_rel, gmin / gmax);
    growth += s.k * s.d * imax;
  }
  s.info.min_abs_gamma_rel = gmin_rel;
  s.info.growth_exponent = growth;

  // ---- host: boundary solve (Sec. 2.5.4, Sec. 3.3-3.4)
  // The connection product K holds exp(growth_exponent) next to O(1) terms;
  // past e^25 (about 7e10) its system keeps fewer digits than the field needs,
  // so a forced connection route fails instead of returning degraded values.
  if ((p.route == SCW_ROUTE_CONNECTION || p.route == SCW_ROUTE_CONNECTION_DEVICE) &&
      growth > kConnectionMaxGrowth)
    return fail(SCW_EILLCOND, "connection route: growth exponent " + std::to_string(growth) +
                                  " above 25 (use SCW_ROUTE_STABLE)");
  if (lp.set_threads) lp.set_threads(ctx.host_threads);
  const double t_bnd = now_s();
  switch (p.route) {
    case SCW_ROUTE_STABLE: rc = solve_stable(lin, s, layers); break;
    case SCW_ROUTE_STABLE_DEVICE: rc = solve_stable_device(ctx, lin, s, layers); break;
    case SCW_ROUTE_CONNECTION_DEVICE: rc = solve_connection_device(ctx, lin, s, layers); break;
    default: rc = solve_connection(lin, s, layers, ctx.host_threads); break;
  }
  if (rc) return rc;
  s.info.boundary_seconds = now_s() - t_bnd;

  // ---- device: synthesis matrices P_l = [X; Psi (S_y Y_x - S_x Y_y)] (Sec. 4.1)
  const size_t pl = (size_t)3 * M * n2;
  if ((rc = s.d_P64.reserve(pl * 16 * L))) return rc;
  DevBuf d_X, d_Y;
  const int pchunk = std::max(1, std::min(L, (int)((size_t)(1u << 30) / (blk * 32))));
  if ((rc = d_X.reserve(blk * 16 * pchunk)) || (rc = d_Y.reserve(blk * 16 * pchunk))) return rc;
  for (int l0 = 0; l0 < L; l0 += pchunk) {
    const int nl = std::min(pchunk, L - l0);
    for (int l = l0; l < l0 + nl; ++l) {
      SCW_HIP(hipMemcpyAsync(d_X.as<char>() + (size_t)(l - l0) * blk * 16, layers[l].X.data(),
                             blk * 16, hipMemcpyHostToDevice, st));
      SCW_HIP(hipMemcpyAsync(d_Y.as<char>() + (size_t)(l - l0) * blk * 16, layers[l].Y.data(),
                             blk * 16, hipMemcpyHostToDevice, st));
    }
    SCW_HIP(launch_build_p(d_X.as<double>(), d_Y.as<double>(),
                           d_psi.as<double>() + (size_t)l0 * nbv * nbu * 2, d_u.as<int>(),
                           d_v.as<int>(), d_sx.as<double>(), d_sy.as<double>(), U, V, nl,
                           s.d_P64.as<double>() + (size_t)l0 * pl * 2, st));
    SCW_HIP(hipStreamSynchronize(st));
  }
  // the complex64 copy every FP32 and split-precision synthesis streams
  // (made here, once, so that no synthesis call has to create or wait for it)
  if ((rc = s.d_P32.reserve(pl * 8 * L))) return rc;
  SCW_HIP(launch_p_to_fp32(s.d_P64.as<double>(), s.d_P32.as<float>(), pl * L, st));
  // per-layer k*gamma, a, b and the exterior coefficients
  // (a, b and the exterior coefficients illumination-major: [K][L][2M], [K][3][3M])
  std::vector<zc> kg((size_t)L * n2), ext(9 * (size_t)M * s.K), ksz(2 * (size_t)M);
  for (size_t i = 0; i < kg.size(); ++i) kg[i] = s.k * s.gamma[i];
  for (int kk = 0; kk < s.K; ++kk)
    for (int i = 0; i < 3 * M; ++i) {
      const size_t o = (size_t)kk * 3 * M + i;
      ext[(size_t)kk * 9 * M + i] = s.p_inc[o];
      ext[(size_t)kk * 9 * M + 3 * M + i] = s.p_ref[o];
      ext[(size_t)kk * 9 * M + 6 * M + i] = s.p_trn[o];
    }
  for (int m = 0; m < M; ++m) {
    ksz[m] = s.k * s.sz_top[m];
    ksz[M + m] = s.k * s.sz_bot[m];
  }
  std::vector<float> kgab32(6 * kg.size());
  for (size_t i = 0; i < kg.size(); ++i) {
    kgab32[2 * i] = (float)kg[i].real();
    kgab32[2 * i + 1] = (float)kg[i].imag();
    kgab32[2 * (kg.size() + i)] = (float)s.a[i].real();
    kgab32[2 * (kg.size() + i) + 1] = (float)s.a[i].imag();
    kgab32[2 * (2 * kg.size() + i)] = (float)s.b[i].real();
    kgab32[2 * (2 * kg.size() + i) + 1] = (float)s.b[i].imag();
  }
  if ((rc = s.d_kgab32.reserve(kgab32.size() * 4))) return rc;
  SCW_HIP(hipMemcpyAsync(s.d_kgab32.p, kgab32.data(), kgab32.size() * 4, hipMemcpyHostToDevice, st));
  if (s.K > 1) {  // complex64 [K][2][L][2M]: a, b of every illumination
    std::vector<float> ab32(4 * s.a.size());
    for (int kk = 0; kk < s.K; ++kk)
      for (size_t i = 0; i < kg.size(); ++i) {
        const zc av = s.a[(size_t)kk * kg.size() + i], bv = s.b[(size_t)kk * kg.size() + i];
        float* o = ab32.data() + (size_t)kk * 4 * kg.size();
        o[2 * i] = (float)av.real();
        o[2 * i + 1] = (float)av.imag();
        o[2 * (kg.size() + i)] = (float)bv.real();
        o[2 * (kg.size() + i) + 1] = (float)bv.imag();
      }
    if ((rc = s.d_ab32.reserve(ab32.size() * 4))) return rc;
    SCW_HIP(hipMemcpyAsync(s.d_ab32.p, ab32.data(), ab32.size() * 4, hipMemcpyHostToDevice, st));
  }
  if ((rc = s.d_kg.reserve(kg.size() * 16)) || (rc = s.d_a.reserve(s.a.size() * 16)) ||
      (rc = s.d_b.reserve(s.b.size() * 16)) || (rc = s.d_ext.reserve(ext.size() * 16)) ||
      (rc = s.d_ksz.reserve(ksz.size() * 16)))
    return rc;
  SCW_HIP(hipMemcpyAsync(s.d_kg.p, kg.data(), kg.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(s.d_a.p, s.a.data(), s.a.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(s.d_b.p, s.b.data(), s.b.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(s.d_ext.p, ext.data(), ext.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipMemcpyAsync(s.d_ksz.p, ksz.data(), ksz.size() * 16, hipMemcpyHostToDevice, st));
  SCW_HIP(hipStreamSynchronize(st));
  s.device = ctx.device;
  s.info.setup_seconds = now_s() - ps.t_start;
  return SCW_OK;
}

int solve_problem(Context& ctx, const scw_problem& p, Solution& s, int n_waves,
                  const scw_plane_wave* waves) {
  PendingSolve ps;
  int rc = solve_begin(ctx, p, s, n_waves, waves, ps);
  if (rc) return rc;
  if (ps.dev_eig) {
    PendingSolve* one[1] = {&ps};
    Solution* sol[1] = {&s};
    if ((rc = device_eig_group(ctx, sol, one, 1))) return rc;
  }
  return solve_finish(ctx, p, s, ps);
}

int solve_problems(Context& ctx, const scw_problem* probs, int n, Solution** sols) {
  // in rounds of problems whose device eigendecompositions share launches:
  // problems of one round with the same matrix order form one batch
  const size_t kRoundBytes = (size_t)24 << 30;  // device A, C and eigensolver workspace
  int i0 = 0;
  while (i0 < n) {
    std::vector<std::unique_ptr<PendingSolve>> ps;
    size_t bytes = 0;
    int i1 = i0;
    while (i1 < n) {
      const size_t nn = 4 * (size_t)probs[i1].U * probs[i1].V * probs[i1].U * probs[i1].V;
      const size_t need = nn * 16 * 6 * (size_t)std::max(1, probs[i1].nz);
      if (i1 > i0 && bytes + need > kRoundBytes) break;
      bytes += need;
      ++i1;
    }
    for (int i = i0; i < i1; ++i) ps.emplace_back(new PendingSolve());
    int rc;
    for (int i = i0; i < i1; ++i)
      if ((rc = solve_begin(ctx, probs[i], *sols[i], 0, nullptr, *ps[i - i0]))) {
        set_error(rc, "problem " + std::to_string(i) + ": " + scw_last_error());
        return rc;
      }
    // device eigendecompositions: one batch per matrix order
    std::vector<char> done(i1 - i0, 0);
    for (int i = i0; i < i1; ++i) {
      if (done[i - i0] || !ps[i - i0]->dev_eig) continue;
      std::vector<PendingSolve*> grp;
      std::vector<Solution*> gs;
      for (int j = i; j < i1; ++j)
        if (!done[j - i0] && ps[j - i0]->dev_eig && sols[j]->M == sols[i]->M) {
          grp.push_back(ps[j - i0].get());
          gs.push_back(sols[j]);
          done[j - i0] = 1;
        }
      if ((rc = device_eig_group(ctx, gs.data(), grp.data(), (int)grp.size()))) {
        set_error(rc, "problems from " + std::to_string(i) + ": " + scw_last_error());
        return rc;
      }
    }
    for (int i = i0; i < i1; ++i)
      if ((rc = solve_finish(ctx, probs[i], *sols[i], *ps[i - i0]))) {
        set_error(rc, "problem " + std::to_string(i) + ": " + scw_last_error());
        return rc;
      }
    i0 = i1;
  }
  return SCW_OK;
}

}  // namespace scw

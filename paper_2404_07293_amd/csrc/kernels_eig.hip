// Batched FP64 complex non-symmetric eigensolver for the per-layer 2M x 2M
// products A C (Sec. 3.2, Sec. 4.2: the eigendecomposition step). Every
// matrix of a batch is independent, so each kernel gives one workgroup (or,
// for the eigenvectors, one wavefront) to one matrix or vector, and a batch of
// layers, wavelengths or patches fills the chip.
//
// Steps, each a published method restated for this layout:
//   1. Householder reduction to upper Hessenberg form H = Q^H A Q, with the
//      reflectors accumulated into Z = Q (Golub & Van Loan, Matrix
//      Computations, Alg. 7.4.2).
//   2. Complex Schur form T = Z^H A Z by the implicitly shifted single-shift
//      QR algorithm on H: Wilkinson shifts with exceptional shifts after 10
//      and 20 stalled iterations, deflation on negligible subdiagonals, every
//      Givens rotation applied to the whole rows and columns of H and to Z
//      (Golub & Van Loan, Sec. 7.5; the complex form of LAPACK's xLAHQR).
//   3. Eigenvectors of T by back-substitution, (T - t_jj I) y_j = 0 with
//      y_j(j) = 1, perturbing a vanishing pivot to eps |t_jj| as xTREVC does.
//      The eigenvectors of A are Z y_j (a batched matrix product done by the
//      caller), normalised to unit length.
// All matrices are column-major, complex128, n x n, stored one after another.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "scw_internal.h"

namespace scw {
namespace {

constexpr int kMaxSweepsPerEigenvalue = 300;
constexpr int kEigWindow = 16;  // rotations per window of the QR sweep

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ inline double2 cmulcj(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__device__ inline double cabs(double2 a) { return hypot(a.x, a.y); }

// a / b by Smith's method (no overflow for moderate ratios).
__device__ inline double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, den = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  const double r = b.x / b.y, den = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}

// Principal square root (Re >= 0).
__device__ inline double2 csqrt(double2 z) {
  const double m = cabs(z);
  if (m == 0.0) return make_double2(0.0, 0.0);
  const double re = sqrt(0.5 * (m + fabs(z.x)));
  const double im = z.y / (2.0 * re);
  if (z.x >= 0.0) return make_double2(re, im);
  return make_double2(fabs(im), copysign(re, z.y));
}

__device__ inline double2 shfl_xor2(double2 v, int mask) {
  return make_double2(__shfl_xor(v.x, mask, 64), __shfl_xor(v.y, mask, 64));
}
__device__ inline double2 wave_sum(double2 v) {
  for (int m = 32; m >= 1; m >>= 1) v = cadd(v, shfl_xor2(v, m));
  return v;
}

template <int TPB>
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TPB / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// M[:, k+1:n] -= tau (M[:, k+1:n] v) v^H on all n rows, one thread per row
// (NR rows per thread).
template <int TPB, int NR>
__device__ void reflect_right(double2* __restrict__ Mx, int n, int k, const double2* v,
                              double2 tau) {
  const int tid = threadIdx.x, m = n - k - 1;
  double2 acc[NR];
#pragma unroll
  for (int t = 0; t < NR; ++t) acc[t] = make_double2(0.0, 0.0);
  for (int i = 0; i < m; ++i) {
    const double2 vi = v[i];
    const double2* col = Mx + (size_t)(k + 1 + i) * n;
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      const int r = tid + t * TPB;
      if (r < n) acc[t] = cadd(acc[t], cmul(col[r], vi));
    }
  }
#pragma unroll
  for (int t = 0; t < NR; ++t) acc[t] = cmul(acc[t], tau);
  for (int i = 0; i < m; ++i) {
    const double2 vc = cconj(v[i]);
    double2* col = Mx + (size_t)(k + 1 + i) * n;
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      const int r = tid + t * TPB;
      if (r < n) col[r] = csub(col[r], cmul(acc[t], vc));
    }
  }
}

// Step 1. One workgroup of TPB threads per matrix; n <= NR * TPB and the
// reflector vector (n - 1 entries) in LDS.
template <int TPB, int NR>
__global__ void __launch_bounds__(TPB)
eig_hessenberg_kernel(int n, double2* __restrict__ A, double2* __restrict__ Z) {
  extern __shared__ double2 v[];
  __shared__ double red[TPB / 64];
  __shared__ double2 s_tau, s_scale;
  __shared__ int s_skip;
  const size_t nn = (size_t)n * n;
  double2* H = A + blockIdx.x * nn;
  double2* Q = Z + blockIdx.x * nn;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (size_t e = tid; e < nn; e += TPB)
    Q[e] = make_double2(e % (size_t)(n + 1) == 0 ? 1.0 : 0.0, 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // x = H[k+1 .. n-1, k]
    double2* x = H + (size_t)k * n + k + 1;
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += TPB) part += x[i].x * x[i].x + x[i].y * x[i].y;
    const double xnorm2 = block_sum<TPB>(part, red);
    if (tid == 0) {
      const double2 alpha = x[0];
      if (xnorm2 == 0.0 && alpha.y == 0.0) {
        s_skip = 1;
      } else {
        // beta = -sign(Re alpha) ||(alpha, x)||, tau = (beta - alpha) / beta,
        // v = [1; x / (alpha - beta)]: (I - tau v v^H)^H [alpha; x] = [beta; 0]
        const double beta =
            -copysign(sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2), alpha.x);
        s_tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        s_scale = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
        s_skip = 0;
        v[0] = make_double2(1.0, 0.0);
        x[0] = make_double2(beta, 0.0);
      }
    }
    __syncthreads();
    if (s_skip) continue;
    const double2 tau = s_tau, scale = s_scale;
    for (int i = 1 + tid; i < m; i += TPB) {
      v[i] = cmul(x[i], scale);
      x[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    reflect_right<TPB, NR>(H, n, k, v, tau);
    reflect_right<TPB, NR>(Q, n, k, v, tau);
    __syncthreads();
    // left: H[k+1:, c] -= conj(tau) v (v^H H[k+1:, c]) for c > k, a wave per column
    const double2 ctau = cconj(tau);
    for (int c = k + 1 + wave; c < n; c += TPB / 64) {
      double2* hc = H + (size_t)c * n + k + 1;
      double2 acc = make_double2(0.0, 0.0);
      for (int i = lane; i < m; i += 64) acc = cadd(acc, cmulcj(v[i], hc[i]));
      const double2 y = cmul(ctau, wave_sum(acc));
      for (int i = lane; i < m; i += 64) hc[i] = csub(hc[i], cmul(v[i], y));
    }
    __syncthreads();
  }
}

// Rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0], c real.
__device__ inline void givens(double2 x, double2 y, double& c, double2& s, double2& r) {
  const double ax = cabs(x), ay = cabs(y);
  if (ay == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
    r = x;
    return;
  }
  if (ax == 0.0) {
    c = 0.0;
    s = cscale(cconj(y), 1.0 / ay);
    r = make_double2(ay, 0.0);
    return;
  }
  const double nrm = hypot(ax, ay);
  const double2 ph = cscale(x, 1.0 / ax);  // x / |x|
  c = ax / nrm;
  s = cscale(cmul(ph, cconj(y)), 1.0 / nrm);
  r = cscale(ph, nrm);
}

__device__ inline double2& at(double2* M, int n, int i, int j) { return M[(size_t)j * n + i]; }

// Step 2. One workgroup of TPB threads per matrix: H (upper Hessenberg, from
// step 1) becomes the upper triangular Schur factor T, Z accumulates the
// rotations, w gets the eigenvalues t_jj. info[b] = 0, or j + 1 when
// eigenvalue j did not converge in kMaxSweepsPerEigenvalue sweeps.
//
// Each sweep runs in windows of W rotations (delayed updates): the diagonal
// block the window's rotations touch (rows and columns b0 .. be, at most
// W + 3) is chased in LDS, the rotations are kept, and then applied in one
// pass to the three regions outside the block that they change: rows
// k0 .. k1 right of the block (row rotations), columns k0 .. k1 above it and
// in Z (column rotations). A thread takes one column or row of a region and
// applies the whole window's rotations to its W + 1 values in registers, so a
// window costs one read and one write of those regions and no barrier per
// rotation outside the small block. Within a window the column entries a
// rotation produces (its r and the zeroed bulge) are written by thread 0 one
// rotation later, once every thread has read them.
template <int TPB, int W>
__global__ void __launch_bounds__(TPB)
eig_schur_kernel(int n, double2* __restrict__ Hall, double2* __restrict__ Zall,
                 double2* __restrict__ wall, int* __restrict__ info) {
  constexpr int LB = W + 3;  // leading dimension of the LDS block (column-major)
  __shared__ double2 blk[LB * LB];
  __shared__ double s_c[W];
  __shared__ double2 s_s[W];
  __shared__ int s_l;
  const size_t nn = (size_t)n * n;
  double2* H = Hall + blockIdx.x * nn;
  double2* Z = Zall + blockIdx.x * nn;
  double2* w = wall + (size_t)blockIdx.x * n;
  const int tid = threadIdx.x;
  const double ulp = DBL_EPSILON, smlnum = DBL_MIN * ((double)n / DBL_EPSILON);
  int ihi = n - 1, its = 0, status = 0;
  while (ihi >= 0) {
    // largest k in [1, ihi] with a negligible subdiagonal: the active block is [l, ihi]
    if (tid == 0) s_l = 0;
    __syncthreads();
    for (int k = 1 + tid; k <= ihi; k += TPB) {
      const double sub = cabs1(at(H, n, k, k - 1));
      double tst = cabs1(at(H, n, k - 1, k - 1)) + cabs1(at(H, n, k, k));
      if (tst == 0.0) {
        if (k >= 2) tst += fabs(at(H, n, k - 1, k - 2).x);
        if (k + 1 <= ihi) tst += fabs(at(H, n, k + 1, k).x);
      }
      if (sub <= fmax(smlnum, ulp * tst)) atomicMax(&s_l, k);
    }
    __syncthreads();
    const int l = s_l;
    __syncthreads();  // every thread has read s_l before it is reset
    if (l > 0 && tid == 0) at(H, n, l, l - 1) = make_double2(0.0, 0.0);
    if (l == ihi) {  // a 1 x 1 block: eigenvalue ihi has converged
      if (tid == 0) w[ihi] = at(H, n, ihi, ihi);
      --ihi;
      its = 0;
      __syncthreads();
      continue;
    }
    if (++its > kMaxSweepsPerEigenvalue) {
      status = ihi + 1;
      break;
    }
    // shift
    double2 mu;
    if (its % 20 == 10) {
      mu = cadd(at(H, n, l, l), make_double2(0.75 * fabs(at(H, n, l + 1, l).x), 0.0));
    } else if (its % 20 == 0) {
      mu = cadd(at(H, n, ihi, ihi), make_double2(0.75 * fabs(at(H, n, ihi, ihi - 1).x), 0.0));
    } else {
      // eigenvalue of the trailing 2 x 2 block closer to its last diagonal entry
      const double2 a = at(H, n, ihi - 1, ihi - 1), b = at(H, n, ihi - 1, ihi);
      const double2 c = at(H, n, ihi, ihi - 1), d = at(H, n, ihi, ihi);
      const double2 bc = cmul(b, c);
      const double2 x = cscale(csub(a, d), 0.5);
      double2 y = csqrt(cadd(cmul(x, x), bc));
      if (x.x * y.x + x.y * y.y < 0.0) y = make_double2(-y.x, -y.y);
      const double2 den = cadd(x, y);
      mu = (den.x == 0.0 && den.y == 0.0) ? d : csub(d, cdiv(bc, den));
    }
    // one implicit single-shift QR sweep over [l, ihi], W rotations per window
    for (int k0 = l; k0 < ihi; k0 += W) {
      const int k1 = min(k0 + W, ihi);        // rotations k0 .. k1 - 1
      const int b0 = k0 == l ? l : k0 - 1;    // block rows and columns b0 .. be
      const int be = min(k1 + 1, ihi);
      const int bn = be - b0 + 1;
      for (int e = tid; e < bn * bn; e += TPB) {
        const int r = e % bn, c = e / bn;
        blk[c * LB + r] = at(H, n, b0 + r, b0 + c);
      }
      __syncthreads();
      double2 r_prev = make_double2(0.0, 0.0);
      for (int k = k0; k < k1; ++k) {
        const int kk = k - b0;
        double2 x, y;
        if (k == l) {
          x = csub(blk[kk * LB + kk], mu);
          y = blk[kk * LB + kk + 1];
        } else {
          x = blk[(kk - 1) * LB + kk];
          y = blk[(kk - 1) * LB + kk + 1];
        }
        double c;
        double2 s, r;
        givens(x, y, c, s, r);
        const double2 ms = make_double2(-s.x, s.y);  // -conj(s)
        const double2 cs = cconj(s);
        if (tid == 0) {
          if (k > k0 && k - 1 > l) {  // the previous rotation's column entries
            blk[(kk - 2) * LB + kk - 1] = r_prev;
            blk[(kk - 2) * LB + kk] = make_double2(0.0, 0.0);
          }
          s_c[k - k0] = c;
          s_s[k - k0] = s;
        }
        r_prev = r;
        for (int j = kk + tid; j < bn; j += TPB) {  // rows k, k+1: columns k .. be
          const double2 t1 = blk[j * LB + kk], t2 = blk[j * LB + kk + 1];
          blk[j * LB + kk] = cadd(cscale(t1, c), cmul(s, t2));
          blk[j * LB + kk + 1] = cadd(cmul(ms, t1), cscale(t2, c));
        }
        __syncthreads();
        const int iend = min(k + 2, be) - b0;
        for (int i = tid; i <= iend; i += TPB) {  // columns k, k+1: rows b0 .. min(k+2, be)
          const double2 t1 = blk[kk * LB + i], t2 = blk[(kk + 1) * LB + i];
          blk[kk * LB + i] = cadd(cscale(t1, c), cmul(cs, t2));
          blk[(kk + 1) * LB + i] = csub(cscale(t2, c), cmul(s, t1));
        }
        __syncthreads();
      }
      if (tid == 0 && k1 - 1 > l) {  // the window's last pending entries
        const int kk = k1 - 1 - b0;
        blk[(kk - 1) * LB + kk] = r_prev;
        blk[(kk - 1) * LB + kk + 1] = make_double2(0.0, 0.0);
      }
      __syncthreads();
      for (int e = tid; e < bn * bn; e += TPB) {
        const int r = e % bn, c = e / bn;
        at(H, n, b0 + r, b0 + c) = blk[c * LB + r];
      }
      const int nq = k1 - k0;
      // rows k0 .. k1 of the columns right of the block
      for (int j = be + 1 + tid; j < n; j += TPB) {
        double2 v[W + 1];
#pragma unroll
        for (int q = 0; q <= W; ++q)
          if (q <= nq) v[q] = at(H, n, k0 + q, j);
#pragma unroll
        for (int q = 0; q < W; ++q) {
          if (q < nq) {
            const double c = s_c[q];
            const double2 sq = s_s[q], msq = make_double2(-sq.x, sq.y);
            const double2 t1 = v[q], t2 = v[q + 1];
            v[q] = cadd(cscale(t1, c), cmul(sq, t2));
            v[q + 1] = cadd(cmul(msq, t1), cscale(t2, c));
          }
        }
#pragma unroll
        for (int q = 0; q <= W; ++q)
          if (q <= nq) at(H, n, k0 + q, j) = v[q];
      }
      // columns k0 .. k1 of the rows above the block, then of every row of Z
      for (int i = tid; i < b0 + n; i += TPB) {
        double2* Mx = i < b0 ? H : Z;
        const int row = i < b0 ? i : i - b0;
        double2 v[W + 1];
#pragma unroll
        for (int q = 0; q <= W; ++q)
          if (q <= nq) v[q] = at(Mx, n, row, k0 + q);
#pragma unroll
        for (int q = 0; q < W; ++q) {
          if (q < nq) {
            const double c = s_c[q];
            const double2 sq = s_s[q];
            const double2 t1 = v[q], t2 = v[q + 1];
            v[q] = cadd(cscale(t1, c), cmul(cconj(sq), t2));
            v[q + 1] = csub(cscale(t2, c), cmul(sq, t1));
          }
        }
#pragma unroll
        for (int q = 0; q <= W; ++q)
          if (q <= nq) at(Mx, n, row, k0 + q) = v[q];
      }
      __syncthreads();
    }
  }
  if (tid == 0) info[blockIdx.x] = status;
}

// Column-major T -> row-major copy of its upper triangle (zeros below), in
// 32 x 32 tiles through LDS.
__global__ void __launch_bounds__(256)
eig_transpose_kernel(int n, const double2* __restrict__ T, double2* __restrict__ Tt) {
  __shared__ double2 tile[32][33];
  const size_t nn = (size_t)n * n;
  const double2* src = T + blockIdx.z * nn;
  double2* dst = Tt + blockIdx.z * nn;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + tx, c = c0 + j;
    tile[j][tx] = (r < n && c < n && r <= c) ? src[(size_t)c * n + r] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + j, c = c0 + tx;
    if (r < n && c < n) dst[(size_t)r * n + c] = tile[tx][j];
  }
}

// Step 3. One wavefront per eigenvector j of one matrix: lane l holds
// y(64 t + l) in slot t (n <= 64 NS). Row i of T (row-major Tt) against y,
// summed over the wave, gives y(i) = -(sum_{k>i} t_ik y(k)) / (t_ii - t_jj)
// for i = j-1 .. 0; the result goes to column j of Y (zeros below j).
template <int NS>
__global__ void __launch_bounds__(256)
eig_vectors_kernel(int n, int count, const double2* __restrict__ Tt,
                   const double2* __restrict__ wall, double2* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const long long gw = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gw >= (long long)count * n) return;
  const int b = (int)(gw / n), j = (int)(gw % n);
  const size_t nn = (size_t)n * n;
  const double2* T = Tt + b * nn;
  const double2 lam = wall[(size_t)b * n + j];
  const double smin = fmax(DBL_EPSILON * cabs1(lam), DBL_MIN * ((double)n / DBL_EPSILON));
  double2 y[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) y[t] = make_double2(64 * t + lane == j ? 1.0 : 0.0, 0.0);
  for (int i = j - 1; i >= 0; --i) {
    const double2* row = T + (size_t)i * n;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int k = 64 * t + lane;
      if (k > i && k <= j) acc = cadd(acc, cmul(row[k], y[t]));
    }
    acc = wave_sum(acc);
    double2 d = csub(row[i], lam);
    if (cabs1(d) < smin) d = make_double2(smin, 0.0);
    const double2 yi = cdiv(make_double2(-acc.x, -acc.y), d);
#pragma unroll
    for (int t = 0; t < NS; ++t)
      if (64 * t + lane == i) y[t] = yi;
  }
  double2* out = Y + b * nn + (size_t)j * n;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int k = 64 * t + lane;
    if (k < n) out[k] = k <= j ? y[t] : make_double2(0.0, 0.0);
  }
}

// Unit 2-norm columns, one wavefront per column.
__global__ void __launch_bounds__(256)
eig_normalize_kernel(int n, long long ncols, double2* __restrict__ X) {
  const int lane = threadIdx.x & 63;
  const long long col = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= ncols) return;
  double2* x = X + col * n;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) s += x[i].x * x[i].x + x[i].y * x[i].y;
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int i = lane; i < n; i += 64) x[i] = cscale(x[i], inv);
}

// Columns scaled by one complex factor each: X[:, j] *= f[j], [count][n] factors.
__global__ void __launch_bounds__(256)
eig_scale_cols_kernel(int n, long long ncols, const double2* __restrict__ f,
                      double2* __restrict__ X) {
  const int lane = threadIdx.x & 63;
  const long long col = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= ncols) return;
  const double2 g = f[col];
  double2* x = X + col * n;
  for (int i = lane; i < n; i += 64) x[i] = cmul(x[i], g);
}

}  // namespace

hipError_t launch_eig_hessenberg(int n, int count, double* A, double* Z, hipStream_t s) {
  if (n < 1 || n > kEigMaxN || count < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)n * sizeof(double2);
  double2* a = reinterpret_cast<double2*>(A);
  double2* z = reinterpret_cast<double2*>(Z);
  const int nr = (n + 255) / 256;
  if (nr <= 1) eig_hessenberg_kernel<256, 1><<<count, 256, lds, s>>>(n, a, z);
  else if (nr <= 2) eig_hessenberg_kernel<256, 2><<<count, 256, lds, s>>>(n, a, z);
  else if (nr <= 4) eig_hessenberg_kernel<256, 4><<<count, 256, lds, s>>>(n, a, z);
  else eig_hessenberg_kernel<256, 8><<<count, 256, lds, s>>>(n, a, z);
  return hipGetLastError();
}

hipError_t launch_eig_schur(int n, int count, double* H, double* Z, double* w, int* info,
                            hipStream_t s) {
  if (n < 1 || n > kEigMaxN || count < 1) return hipErrorInvalidValue;
  eig_schur_kernel<256, kEigWindow><<<count, 256, 0, s>>>(
      n, reinterpret_cast<double2*>(H), reinterpret_cast<double2*>(Z),
      reinterpret_cast<double2*>(w), info);
  return hipGetLastError();
}

hipError_t launch_eig_vectors(int n, int count, const double* T, double* Tt, const double* w,
                              double* Y, hipStream_t s) {
  if (n < 1 || n > kEigMaxN || count < 1) return hipErrorInvalidValue;
  const unsigned tiles = (unsigned)((n + 31) / 32);
  eig_transpose_kernel<<<dim3(tiles, tiles, count), 256, 0, s>>>(
      n, reinterpret_cast<const double2*>(T), reinterpret_cast<double2*>(Tt));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long waves = (long long)count * n;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  const double2* tt = reinterpret_cast<const double2*>(Tt);
  const double2* ww = reinterpret_cast<const double2*>(w);
  double2* y = reinterpret_cast<double2*>(Y);
  const int ns = (n + 63) / 64;
  if (ns <= 2) eig_vectors_kernel<2><<<blocks, 256, 0, s>>>(n, count, tt, ww, y);
  else if (ns <= 4) eig_vectors_kernel<4><<<blocks, 256, 0, s>>>(n, count, tt, ww, y);
  else if (ns <= 8) eig_vectors_kernel<8><<<blocks, 256, 0, s>>>(n, count, tt, ww, y);
  else if (ns <= 16) eig_vectors_kernel<16><<<blocks, 256, 0, s>>>(n, count, tt, ww, y);
  else eig_vectors_kernel<32><<<blocks, 256, 0, s>>>(n, count, tt, ww, y);
  return hipGetLastError();
}

hipError_t launch_eig_normalize(int n, long long ncols, double* X, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  eig_normalize_kernel<<<(unsigned)((ncols + 3) / 4), 256, 0, s>>>(
      n, ncols, reinterpret_cast<double2*>(X));
  return hipGetLastError();
}

hipError_t launch_eig_scale_cols(int n, long long ncols, const double* f, double* X,
                                 hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  eig_scale_cols_kernel<<<(unsigned)((ncols + 3) / 4), 256, 0, s>>>(
      n, ncols, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(X));
  return hipGetLastError();
}

}  // namespace scw

// FP64 device kernels of the setup: layer spectra (Sec. 2.4), property-matrix
// blocks (Sec. 2.5.2) and the per-layer synthesis matrix P (Sec. 4.1).
#include <hip/hip_runtime.h>

#include "scw_internal.h"

namespace scw {
namespace {

struct z2 {
  double x, y;
};
__device__ __forceinline__ z2 zmul(z2 a, z2 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ z2 zdiv_one(z2 a) {  // 1 / a
  double d = a.x * a.x + a.y * a.y;
  return {a.x / d, -a.y / d};
}
__device__ __forceinline__ void zfma(z2& acc, z2 a, z2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// exp(-2 pi i * idx / n) with idx reduced modulo n first, so the angle is
// exact to rounding of idx/n.
__device__ __forceinline__ z2 twiddle_fwd(long long idx, int n) {
  long long r = idx % n;
  if (r < 0) r += n;
  double s, c;
  sincospi(-2.0 * (double)r / (double)n, &s, &c);
  return {c, s};
}

// Pass 1 of the band DFT: for each layer, row j and du in [-hu, hu],
//   row[w][l][j][du] = sum_i f_w(l, j, i) exp(-2 pi i du i / nx),
// with f_0 = n^2 (or n when !square) and f_1 = 1/n^2.
__global__ void band_dft_rows(const z2* __restrict__ n, int L, int ny, int nx, int hu,
                              int nw, bool square, z2* __restrict__ row) {
  const int nu = 2 * hu + 1;
  const long long total = (long long)nw * L * ny * nu;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int du = (int)(t % nu) - hu;
  long long q = t / nu;
  const int j = (int)(q % ny);
  q /= ny;
  const int l = (int)(q % L);
  const int w = (int)(q / L);
  const z2* src = n + ((long long)l * ny + j) * nx;
  z2 acc = {0.0, 0.0};
  for (int i = 0; i < nx; ++i) {
    z2 v = src[i];
    if (square) v = zmul(v, v);
    if (w == 1) v = zdiv_one(v);
    zfma(acc, v, twiddle_fwd((long long)du * i, nx));
  }
  row[t] = acc;
}

// Pass 2: out[w][l][dv][du] = (1/(nx ny)) sum_j row[w][l][j][du] exp(-2 pi i dv j / ny).
__global__ void band_dft_cols(const z2* __restrict__ row, int L, int ny, int nx, int hu,
                              int hv, int nw, z2* __restrict__ out0,
                              z2* __restrict__ out1) {
  const int nu = 2 * hu + 1, nv = 2 * hv + 1;
  const long long total = (long long)nw * L * nv * nu;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int iu = (int)(t % nu);
  long long q = t / nu;
  const int iv = (int)(q % nv);
  q /= nv;
  const int l = (int)(q % L);
  const int w = (int)(q / L);
  const int dv = iv - hv;
  const z2* src = row + (((long long)w * L + l) * ny) * nu + iu;
  z2 acc = {0.0, 0.0};
  for (int j = 0; j < ny; ++j) zfma(acc, src[(long long)j * nu], twiddle_fwd((long long)dv * j, ny));
  const double s = 1.0 / ((double)nx * (double)ny);
  z2* dst = (w == 0) ? out0 : out1;
  dst[((long long)l * nv + iv) * nu + iu] = {acc.x * s, acc.y * s};
}

// Blocks of D = [[0, A], [C, 0]] (Eq. 21; lower blocks from Eqs. 15-16) in
// column-major 2M x 2M storage per layer:
//   A = [[Sx Psi Sy, I - Sx Psi Sx], [Sy Psi Sy - I, -Sy Psi Sx]]
//   C = [[-Sx Sy, Sx^2 - Phi], [Phi - Sy^2, Sy Sx]]
__global__ void assemble_ac(const z2* __restrict__ phi, const z2* __restrict__ psi,
                            const int* __restrict__ u, const int* __restrict__ v,
                            const double* __restrict__ sx, const double* __restrict__ sy,
                            int U, int V, int L, z2* __restrict__ A, z2* __restrict__ C) {
  const int M = U * V, n2 = 2 * M;
  const long long total = (long long)L * n2 * n2;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int r = (int)(t % n2);
  long long q = t / n2;
  const int c = (int)(q % n2);
  const int l = (int)(q / n2);
  const int br = r / M, bc = c / M, m = r % M, mp = c % M;
  const int nu = 2 * U - 1;
  const long long bidx = (long long)l * (2 * V - 1) * nu +
                         (long long)(v[m] - v[mp] + V - 1) * nu + (u[m] - u[mp] + U - 1);
  const z2 ps = psi[bidx];
  const z2 ph = phi[bidx];
  const double d = (m == mp) ? 1.0 : 0.0;
  const double sxm = sx[m], sym = sy[m], sxp = sx[mp], syp = sy[mp];
  z2 a, cc;
  if (br == 0 && bc == 0) {
    a = {sxm * syp * ps.x, sxm * syp * ps.y};
    cc = {-sxm * sym * d, 0.0};
  } else if (br == 0 && bc == 1) {
    a = {d - sxm * sxp * ps.x, -sxm * sxp * ps.y};
    cc = {sxm * sxm * d - ph.x, -ph.y};
  } else if (br == 1 && bc == 0) {
    a = {sym * syp * ps.x - d, sym * syp * ps.y};
    cc = {ph.x - sym * sym * d, ph.y};
  } else {
    a = {-sym * sxp * ps.x, -sym * sxp * ps.y};
    cc = {sym * sxm * d, 0.0};
  }
  A[t] = a;
  C[t] = cc;
}

// Rows 0..2M-1 of P: the E-part of the forward eigenvectors, transposed from
// LAPACK column-major X into row-major P[r][j].
__global__ void p_xy_rows(const z2* __restrict__ X, int M, int nlayers,
                          z2* __restrict__ P) {
  const int n2 = 2 * M, n3 = 3 * M;
  __shared__ z2 tile[16][17];
  const int l = blockIdx.z;
  const int r0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const z2* Xl = X + (long long)l * n2 * n2;
  // read column-major: X[j][r] contiguous in r
  {
    int r = r0 + tx, j = j0 + ty;
    if (r < n2 && j < n2) tile[ty][tx] = Xl[(long long)j * n2 + r];
  }
  __syncthreads();
  {
    int r = r0 + ty, j = j0 + tx;
    if (r < n2 && j < n2) P[((long long)l * n3 + r) * n2 + j] = tile[tx][ty];
  }
}

// Rows 2M..3M-1 of P: Z = Psi (S_y Y_x - S_x Y_y), the z component of the
// field from the H-part (Sec. 2.6.2, Eqs. 32-33; Sec. 4.1), with Psi gathered
// from the psi band, never stored. Tiled as a GEMM over m'.
__global__ void p_z_rows(const z2* __restrict__ Y, const z2* __restrict__ psi,
                         const int* __restrict__ u, const int* __restrict__ v,
                         const double* __restrict__ sx, const double* __restrict__ sy,
                         int U, int V, int nlayers, z2* __restrict__ P) {
  const int M = U * V, n2 = 2 * M, n3 = 3 * M;
  const int l = blockIdx.z;
  const int m0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int tx = threadIdx.x, ty = threadIdx.y;  // tx -> j, ty -> m
  __shared__ z2 sH[16][17];    // [m'][j]
  __shared__ z2 sPs[16][17];   // [m][m']
  const z2* Yl = Y + (long long)l * n2 * n2;
  const z2* psil = psi + (long long)l * (2 * V - 1) * (2 * U - 1);
  const int nu = 2 * U - 1;
  z2 acc = {0.0, 0.0};
  const int m = m0 + ty, j = j0 + tx;
  for (int k0 = 0; k0 < M; k0 += 16) {
    {  // H[m'][j] = sy[m'] Y[m'][j] - sx[m'] Y[M+m'][j]; thread (ty -> m', tx -> j)
      int mp = k0 + ty, jj = j0 + tx;
      z2 h = {0.0, 0.0};
      if (mp < M && jj < n2) {
        z2 yx = Yl[(long long)jj * n2 + mp];
        z2 yy = Yl[(long long)jj * n2 + M + mp];
        h = {sy[mp] * yx.x - sx[mp] * yy.x, sy[mp] * yx.y - sx[mp] * yy.y};
      }
      sH[ty][tx] = h;
    }
    {  // Psi[m][m'] = psi(u_m - u_m', v_m - v_m'); thread (ty -> m, tx -> m')
      int mm = m0 + ty, mp = k0 + tx;
      z2 p = {0.0, 0.0};
      if (mm < M && mp < M)
        p = psil[(long long)(v[mm] - v[mp] + V - 1) * nu + (u[mm] - u[mp] + U - 1)];
      sPs[ty][tx] = p;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) zfma(acc, sPs[ty][kk], sH[kk][tx]);
    __syncthreads();
  }
  if (m < M && j < n2) P[((long long)l * n3 + n2 + m) * n2 + j] = acc;
}

__global__ void to_fp32(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Elementwise steps of the device elimination (column-major n x n blocks).
__global__ void eye_kernel(z2* __restrict__ A, int n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n) return;
  A[i] = z2{i / n == i % n ? 1.0 : 0.0, 0.0};
}

// A1 <- (A1 + A2) / 2, A2 <- (A1 - A2) / 2
__global__ void half_sum_diff(z2* __restrict__ A1, z2* __restrict__ A2, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const z2 a = A1[i], b = A2[i];
  A1[i] = z2{0.5 * (a.x + b.x), 0.5 * (a.y + b.y)};
  A2[i] = z2{0.5 * (a.x - b.x), 0.5 * (a.y - b.y)};
}

// P1 = I + E r E, P2 = I - E r E (E diagonal)
__global__ void i_pm_ere(const z2* __restrict__ r, const z2* __restrict__ E, int n,
                         z2* __restrict__ P1, z2* __restrict__ P2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n) return;
  const int c = (int)(i / n), row = (int)(i % n);
  const z2 x = zmul(zmul(E[row], r[i]), E[c]);
  const double d = row == c ? 1.0 : 0.0;
  P1[i] = z2{d + x.x, x.y};
  P2[i] = z2{d - x.x, -x.y};
}

// out[c][j] = E[j] A[c][j] for n rows and k columns
__global__ void scale_rows(const z2* __restrict__ E, const z2* __restrict__ A, int n, int k,
                           z2* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * k) return;
  out[i] = zmul(E[i % n], A[i]);
}

// T_l = W diag(I, E) and B_l = W diag(E, I) of the connection route, with
// W = [[X, X], [Y, -Y]] (forward columns first), column-major 4M x 4M.
__global__ void build_tb(const z2* __restrict__ X, const z2* __restrict__ Y,
                         const z2* __restrict__ E, int n2, z2* __restrict__ T,
                         z2* __restrict__ B) {
  const int n4 = 2 * n2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n4 * n4) return;
  const int col = (int)(i / n4), row = (int)(i % n4);
  const int c = col % n2, rr = row % n2;
  const bool back = col >= n2, top = row < n2;
  const z2 v = top ? X[(long long)c * n2 + rr] : Y[(long long)c * n2 + rr];
  const z2 ve = zmul(v, E[c]);
  const double sg = (back && !top) ? -1.0 : 1.0;  // the backward H part changes sign
  T[i] = back ? z2{sg * ve.x, sg * ve.y} : v;
  B[i] = back ? z2{sg * v.x, sg * v.y} : ve;
}

}  // namespace

hipError_t launch_build_tb(const double* X, const double* Y, const double* E, int n2, double* T,
                           double* B, hipStream_t s) {
  build_tb<<<blocks_for(4LL * n2 * n2, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(X), reinterpret_cast<const z2*>(Y),
      reinterpret_cast<const z2*>(E), n2, reinterpret_cast<z2*>(T), reinterpret_cast<z2*>(B));
  return hipGetLastError();
}

// Top-surface system of the stable route, column-major n4 x n4 (n4 = 2 n2):
// S = [[I, -Fe], [Hr, -Fh]] (incident + reflected = field at the top of layer 1).
__global__ void top_system(const z2* __restrict__ Hr, const z2* __restrict__ Fe,
                           const z2* __restrict__ Fh, int n2, z2* __restrict__ S) {
  const int n4 = 2 * n2;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n4 * n4) return;
  const int col = (int)(i / n4), row = (int)(i % n4);
  z2 v;
  if (col < n2)
    v = row < n2 ? z2{row == col ? 1.0 : 0.0, 0.0} : Hr[(long long)col * n2 + row - n2];
  else {
    const z2 f = row < n2 ? Fe[(long long)(col - n2) * n2 + row]
                          : Fh[(long long)(col - n2) * n2 + row - n2];
    v = z2{-f.x, -f.y};
  }
  S[i] = v;
}

// Connection system of Eq. 29, column-major n6 x n6 (n6 = 6M): rows 0 .. 4M-1
// are [-K C_r | C_t], rows 4M .. 6M-1 the Gauss rows of the reflected and the
// transmitted waves (Eq. 14). KCr, Ct: 4M x 3M column-major; szt, szb: s_z of
// the two half-spaces.
__global__ void connection_system_kernel(const z2* __restrict__ KCr, const z2* __restrict__ Ct,
                                         const double* __restrict__ sx,
                                         const double* __restrict__ sy,
                                         const z2* __restrict__ szt, const z2* __restrict__ szb,
                                         int M, z2* __restrict__ A) {
  const int n4 = 4 * M, n6 = 6 * M;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n6 * n6) return;
  const int col = (int)(i / n6), row = (int)(i % n6);
  z2 v{0.0, 0.0};
  if (row < n4) {
    if (col < 3 * M) {
      const z2 k = KCr[(long long)col * n4 + row];
      v = z2{-k.x, -k.y};
    } else {
      v = Ct[(long long)(col - 3 * M) * n4 + row];
    }
  } else if (row < n4 + M) {  // reflected wave: s_x p_x + s_y p_y - s_z p_z = 0
    const int m = row - n4;
    if (col == m) v = z2{sx[m], 0.0};
    else if (col == M + m) v = z2{sy[m], 0.0};
    else if (col == 2 * M + m) v = z2{-szt[m].x, -szt[m].y};
  } else {  // transmitted wave: s_x p_x + s_y p_y + s_z p_z = 0
    const int m = row - n4 - M;
    if (col == 3 * M + m) v = z2{sx[m], 0.0};
    else if (col == 4 * M + m) v = z2{sy[m], 0.0};
    else if (col == 5 * M + m) v = szb[m];
  }
  A[i] = v;
}

// out[c] = sum_r |A[r][c]| over the n columns of a column-major n x n matrix
// (one wave per column).
__global__ void col_abs_sum(const z2* __restrict__ A, int n, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const long long c = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const z2* col = A + c * n;
  double acc = 0.0;
  for (int r = lane; r < n; r += 64) acc += hypot(col[r].x, col[r].y);
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) out[c] = acc;
}

hipError_t launch_top_system(const double* Hr, const double* Fe, const double* Fh, int n2,
                             double* S, hipStream_t s) {
  top_system<<<blocks_for(4LL * n2 * n2, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(Hr), reinterpret_cast<const z2*>(Fe),
      reinterpret_cast<const z2*>(Fh), n2, reinterpret_cast<z2*>(S));
  return hipGetLastError();
}

hipError_t launch_connection_system(const double* KCr, const double* Ct, const double* sx,
                                    const double* sy, const double* szt, const double* szb,
                                    int M, double* A, hipStream_t s) {
  connection_system_kernel<<<blocks_for(36LL * M * M, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(KCr), reinterpret_cast<const z2*>(Ct), sx, sy,
      reinterpret_cast<const z2*>(szt), reinterpret_cast<const z2*>(szb), M,
      reinterpret_cast<z2*>(A));
  return hipGetLastError();
}

hipError_t launch_col_abs_sum(const double* A, int n, double* out, hipStream_t s) {
  col_abs_sum<<<blocks_for(n, 4), 256, 0, s>>>(reinterpret_cast<const z2*>(A), n, out);
  return hipGetLastError();
}

hipError_t launch_eye(double* A, int n, hipStream_t s) {
  eye_kernel<<<blocks_for((long long)n * n, 256), 256, 0, s>>>(reinterpret_cast<z2*>(A), n);
  return hipGetLastError();
}

hipError_t launch_half_sum_diff(double* A1, double* A2, long long n, hipStream_t s) {
  half_sum_diff<<<blocks_for(n, 256), 256, 0, s>>>(reinterpret_cast<z2*>(A1),
                                                   reinterpret_cast<z2*>(A2), n);
  return hipGetLastError();
}

hipError_t launch_i_pm_ere(const double* r, const double* E, int n, double* P1, double* P2,
                           hipStream_t s) {
  i_pm_ere<<<blocks_for((long long)n * n, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(r), reinterpret_cast<const z2*>(E), n,
      reinterpret_cast<z2*>(P1), reinterpret_cast<z2*>(P2));
  return hipGetLastError();
}

hipError_t launch_scale_rows(const double* E, const double* A, int n, int k, double* out,
                             hipStream_t s) {
  scale_rows<<<blocks_for((long long)n * k, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(E), reinterpret_cast<const z2*>(A), n, k,
      reinterpret_cast<z2*>(out));
  return hipGetLastError();
}

hipError_t launch_band_dft(const double* n, int L, int ny, int nx, int hu, int hv,
                           bool inverse_eps_too, bool square, double* rowbuf,
                           double* out_eps, double* out_inv, hipStream_t s) {
  const int nw = inverse_eps_too ? 2 : 1;
  const long long n1 = (long long)nw * L * ny * (2 * hu + 1);
  band_dft_rows<<<blocks_for(n1, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(n), L, ny, nx, hu, nw, square,
      reinterpret_cast<z2*>(rowbuf));
  const long long n2 = (long long)nw * L * (2 * hv + 1) * (2 * hu + 1);
  band_dft_cols<<<blocks_for(n2, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(rowbuf), L, ny, nx, hu, hv, nw,
      reinterpret_cast<z2*>(out_eps), reinterpret_cast<z2*>(out_inv));
  return hipGetLastError();
}

hipError_t launch_assemble_ac(const double* phi, const double* psi, const int* u,
                              const int* v, const double* sx, const double* sy, int U,
                              int V, int L, double* A, double* C, hipStream_t s) {
  const long long n = (long long)L * 4 * (long long)U * V * U * V;
  assemble_ac<<<blocks_for(n, 256), 256, 0, s>>>(
      reinterpret_cast<const z2*>(phi), reinterpret_cast<const z2*>(psi), u, v, sx, sy,
      U, V, L, reinterpret_cast<z2*>(A), reinterpret_cast<z2*>(C));
  return hipGetLastError();
}

hipError_t launch_build_p(const double* X, const double* Y, const double* psi, const int* u,
                          const int* v, const double* sx, const double* sy, int U, int V,
                          int nlayers, double* P, hipStream_t s) {
  const int M = U * V, n2 = 2 * M;
  dim3 bs(16, 16);
  dim3 g1((n2 + 15) / 16, (n2 + 15) / 16, nlayers);
  p_xy_rows<<<g1, bs, 0, s>>>(reinterpret_cast<const z2*>(X), M, nlayers,
                              reinterpret_cast<z2*>(P));
  dim3 g2((n2 + 15) / 16, (M + 15) / 16, nlayers);
  p_z_rows<<<g2, bs, 0, s>>>(reinterpret_cast<const z2*>(Y),
                             reinterpret_cast<const z2*>(psi), u, v, sx, sy, U, V,
                             nlayers, reinterpret_cast<z2*>(P));
  return hipGetLastError();
}

hipError_t launch_p_to_fp32(const double* P64, float* P32, size_t n_complex, hipStream_t s) {
  const size_t n = 2 * n_complex;
  to_fp32<<<blocks_for((long long)n, 256), 256, 0, s>>>(P64, P32, n);
  return hipGetLastError();
}

}  // namespace scw

// Field synthesis kernels, the hot path (Sec. 2.6, Sec. 4.1, Eqs. 9, 10, 30-34):
//
//   phase     W±[task][p][j] = a_j exp(i k g_j dz_top) ± b_j exp(-i k g_j dz_bot)
//   modal     spec[plane][r] = sum_j P_l[r][j] W(sign(r))[task][p][j]
//             (rows r < 2M are p_x, p_y and take W+, rows >= 2M are p_z and
//              take W-, because a forward/backward eigenvector pair shares
//              its E part and has opposite H parts)
//   exterior  spec of planes above / below the sample from the plane-wave
//             coefficients (Eq. 9)
//   idft      E[c][plane][g][f] = sum_{v,u} spec[plane][c][v][u]
//             exp(2 pi i (u f / fx + v g / fy)), as two passes (x, then y).
#include <hip/hip_runtime.h>

#include "scw_internal.h"

namespace scw {
namespace {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

struct zd {
  double x, y;
};
__device__ __forceinline__ zd zexp_i(zd arg) {  // exp(i * arg)
  double s, c;
  sincos(arg.x, &s, &c);
  double m = exp(-arg.y);
  return {m * c, m * s};
}
__device__ __forceinline__ zd zmul(zd a, zd b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---------------------------------------------------------------- phase
template <typename T>
__global__ void phase_kernel(const Task* __restrict__ tasks, const double* __restrict__ dz,
                             const zd* __restrict__ kg, const zd* __restrict__ a,
                             const zd* __restrict__ b, int n2, int zt, int ntasks,
                             cx<T>* __restrict__ w) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)ntasks * n2) return;
  const int j = (int)(t % n2);
  const int task = (int)(t / n2);
  const Task tk = tasks[task];
  const long long lj = (long long)tk.layer * n2 + j;
  const zd g = kg[lj], aj = a[lj], bj = b[lj];
  for (int p = 0; p < zt; ++p) {
    cx<T> wp = {0, 0}, wm = {0, 0};
    if (p < tk.count) {
      const double dt = dz[((long long)task * zt + p) * 2 + 0];
      const double db = dz[((long long)task * zt + p) * 2 + 1];
      const zd gf = zexp_i({g.x * dt, g.y * dt});
      const zd gb = zexp_i({-g.x * db, -g.y * db});
      const zd f = zmul(aj, gf), bk = zmul(bj, gb);
      wp = {(T)(f.x + bk.x), (T)(f.y + bk.y)};
      wm = {(T)(f.x - bk.x), (T)(f.y - bk.y)};
    }
    w[(((long long)task * 2 + 0) * zt + p) * n2 + j] = wp;
    w[(((long long)task * 2 + 1) * zt + p) * n2 + j] = wm;
  }
}

// ---------------------------------------------------------------- modal sum
// One block = 4 waves; each wave owns RW consecutive rows of one category
// (x/y rows or z rows) of one task. The task's W table for that category is
// staged in LDS in chunks of jc columns; lanes stride over j, every lane keeps
// RW x ZT partial sums, and a butterfly reduction finishes each row.
template <typename T, int ZT, int RW>
__global__ void __launch_bounds__(256) modal_kernel(
    const cx<T>* __restrict__ P, const cx<T>* __restrict__ w, const Task* __restrict__ tasks,
    int M, int nb_xy, int nb_z, int jc, cx<T>* __restrict__ spec) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* sw = reinterpret_cast<cx<T>*>(smem_raw);  // [ZT][jc]
  const int n2 = 2 * M, n3 = 3 * M;
  const int nb = nb_xy + nb_z;
  const int task = blockIdx.x / nb;
  const int rb = blockIdx.x % nb;
  const Task tk = tasks[task];
  const int sign = rb < nb_xy ? 0 : 1;
  const int rows_per_block = 4 * RW;
  const int row_begin = sign == 0 ? rb * rows_per_block : n2 + (rb - nb_xy) * rows_per_block;
  const int row_end = sign == 0 ? n2 : n3;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = row_begin + wave * RW;
  const cx<T>* Pl = P + (long long)tk.layer * n3 * n2;
  const cx<T>* wt = w + ((long long)task * 2 + sign) * ZT * n2;

  cx<T> acc[RW][ZT];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int p = 0; p < ZT; ++p) acc[r][p] = {0, 0};

  for (int j0 = 0; j0 < n2; j0 += jc) {
    const int jn = min(jc, n2 - j0);
    __syncthreads();
    for (int i = threadIdx.x; i < ZT * jn; i += blockDim.x) {
      const int p = i / jn, jj = i % jn;
      sw[p * jc + jj] = wt[(long long)p * n2 + j0 + jj];
    }
    __syncthreads();
    for (int jj = lane; jj < jn; jj += 64) {
      cx<T> wv[ZT];
#pragma unroll
      for (int p = 0; p < ZT; ++p) wv[p] = sw[p * jc + jj];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int row = r0 + r;
        if (row < row_end) {
          const cx<T> pv = Pl[(long long)row * n2 + j0 + jj];
#pragma unroll
          for (int p = 0; p < ZT; ++p) cfma(acc[r][p], pv, wv[p]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int p = 0; p < ZT; ++p) {
      T x = acc[r][p].x, y = acc[r][p].y;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off, 64);
        y += __shfl_xor(y, off, 64);
      }
      acc[r][p] = {x, y};
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = r0 + r;
      if (row >= row_end) continue;
#pragma unroll
      for (int p = 0; p < ZT; ++p)
        if (p < tk.count) spec[(long long)(tk.plane0 + p) * n3 + row] = acc[r][p];
    }
  }
}

// ---------------------------------------------------------------- exterior
template <typename T>
__global__ void exterior_kernel(const ExtPlane* __restrict__ ext, int n_ext, int M,
                                const zd* __restrict__ coef, const zd* __restrict__ ksz,
                                cx<T>* __restrict__ spec) {
  const int n3 = 3 * M;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n_ext * n3) return;
  const int r = (int)(t % n3);
  const ExtPlane e = ext[t / n3];
  const int m = r % M;
  zd val;
  if (e.kind == 0) {
    const zd kz = ksz[m];
    const zd gi = zexp_i({kz.x * e.dz, kz.y * e.dz});
    const zd gr = zexp_i({-kz.x * e.dz, -kz.y * e.dz});
    const zd pi = zmul(coef[r], gi), pr = zmul(coef[n3 + r], gr);
    val = {pi.x + pr.x, pi.y + pr.y};
  } else {
    const zd kz = ksz[M + m];
    val = zmul(coef[2 * n3 + r], zexp_i({kz.x * e.dz, kz.y * e.dz}));
  }
  spec[(long long)e.plane * n3 + r] = {(T)val.x, (T)val.y};
}

// ---------------------------------------------------------------- inverse DFT
// Pass 1: t1[plane][c][v][f] = sum_u spec[plane][c][v][u] twx[u][f].
template <typename T>
__global__ void idft_x_kernel(const cx<T>* __restrict__ spec, const cx<T>* __restrict__ twx,
                              int U, int V, int fx, int fz, cx<T>* __restrict__ t1) {
  const int M = U * V;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)fz * 3 * V * fx) return;
  const int f = (int)(t % fx);
  long long q = t / fx;
  const int vi = (int)(q % V);
  q /= V;  // plane * 3 + c
  const cx<T>* s = spec + q * M + (long long)vi * U;  // spec[plane][c*M + vi*U + u]
  cx<T> acc = {0, 0};
  for (int u = 0; u < U; ++u) cfma(acc, s[u], twx[(long long)u * fx + f]);
  t1[t] = acc;
}

// Pass 2: E[c][plane][g][f] = sum_v twy[v][g] t1[plane][c][v][f]; each thread
// computes GT consecutive g for one f.
template <typename T, int GT>
__global__ void idft_y_kernel(const cx<T>* __restrict__ t1, const cx<T>* __restrict__ twy,
                              int V, int fx, int fy, int fz, cx<T>* __restrict__ E) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  const int g0 = blockIdx.y * GT;
  const int pc = blockIdx.z;  // plane * 3 + c
  if (f >= fx) return;
  const int plane = pc / 3, c = pc % 3;
  const cx<T>* src = t1 + (long long)pc * V * fx + f;
  cx<T> acc[GT];
#pragma unroll
  for (int i = 0; i < GT; ++i) acc[i] = {0, 0};
  for (int vi = 0; vi < V; ++vi) {
    const cx<T> tv = src[(long long)vi * fx];
    const cx<T>* wy = twy + (long long)vi * fy + g0;
#pragma unroll
    for (int i = 0; i < GT; ++i)
      if (g0 + i < fy) cfma(acc[i], wy[i], tv);
  }
  cx<T>* dst = E + (((long long)c * fz + plane) * fy + g0) * fx + f;
#pragma unroll
  for (int i = 0; i < GT; ++i)
    if (g0 + i < fy) dst[(long long)i * fx] = acc[i];
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, int ZT>
hipError_t launch_modal(const SynthArgs& a, hipStream_t s) {
  constexpr int RW = (sizeof(T) == 4) ? (ZT <= 4 ? 8 : 4) : (ZT <= 2 ? 4 : 2);
  const int n2 = 2 * a.M;
  const int rows_per_block = 4 * RW;
  const int nb_xy = (n2 + rows_per_block - 1) / rows_per_block;
  const int nb_z = (a.M + rows_per_block - 1) / rows_per_block;
  const size_t max_lds = 64 * 1024;
  int jc = (int)(max_lds / (ZT * sizeof(cx<T>)));
  jc = jc >= n2 ? n2 : (jc / 64) * 64;
  const size_t lds = (size_t)ZT * jc * sizeof(cx<T>);
  const long long nblocks = (long long)a.ntasks * (nb_xy + nb_z);
  if (nblocks == 0) return hipSuccess;
  modal_kernel<T, ZT, RW><<<(unsigned)nblocks, 256, lds, s>>>(
      reinterpret_cast<const cx<T>*>(a.P), reinterpret_cast<const cx<T>*>(a.w), a.tasks, a.M,
      nb_xy, nb_z, jc, reinterpret_cast<cx<T>*>(a.spec));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_synthesis(const SynthArgs& a, hipStream_t s, hipEvent_t* ev) {
  hipError_t e;
  const int n2 = 2 * a.M;
  auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev[i], s) : hipSuccess; };
  if ((e = mark(0)) != hipSuccess) return e;
  if (a.ntasks > 0) {
    phase_kernel<T><<<blocks_for((long long)a.ntasks * n2, 256), 256, 0, s>>>(
        a.tasks, a.task_dz, reinterpret_cast<const zd*>(a.kg),
        reinterpret_cast<const zd*>(a.a), reinterpret_cast<const zd*>(a.b), n2, a.zt,
        a.ntasks, reinterpret_cast<cx<T>*>(a.w));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = mark(1)) != hipSuccess) return e;
    switch (a.zt) {
      case 1: e = launch_modal<T, 1>(a, s); break;
      case 2: e = launch_modal<T, 2>(a, s); break;
      case 4: e = launch_modal<T, 4>(a, s); break;
      case 8: e = launch_modal<T, 8>(a, s); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  } else if ((e = mark(1)) != hipSuccess) {
    return e;
  }
  if ((e = mark(2)) != hipSuccess) return e;
  if (a.n_ext > 0) {
    exterior_kernel<T><<<blocks_for((long long)a.n_ext * 3 * a.M, 256), 256, 0, s>>>(
        reinterpret_cast<const ExtPlane*>(a.ext_planes), a.n_ext, a.M,
        reinterpret_cast<const zd*>(a.ext), reinterpret_cast<const zd*>(a.ksz),
        reinterpret_cast<cx<T>*>(a.spec));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = mark(3)) != hipSuccess) return e;
  idft_x_kernel<T><<<blocks_for((long long)a.fz * 3 * a.V * a.fx, 256), 256, 0, s>>>(
      reinterpret_cast<const cx<T>*>(a.spec), reinterpret_cast<const cx<T>*>(a.twx), a.U,
      a.V, a.fx, a.fz, reinterpret_cast<cx<T>*>(a.t1));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = mark(4)) != hipSuccess) return e;
  constexpr int GT = 8;
  const int bx = a.fx >= 256 ? 256 : ((a.fx + 63) / 64) * 64;
  dim3 grid((a.fx + bx - 1) / bx, (a.fy + GT - 1) / GT, a.fz * 3);
  idft_y_kernel<T, GT><<<grid, bx, 0, s>>>(reinterpret_cast<const cx<T>*>(a.t1),
                                          reinterpret_cast<const cx<T>*>(a.twy), a.V, a.fx,
                                          a.fy, a.fz, reinterpret_cast<cx<T>*>(a.E));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return mark(5);
}

}  // namespace

hipError_t launch_synthesis_fp64(const SynthArgs& a, hipStream_t s, hipEvent_t* ev) {
  return launch_synthesis<double>(a, s, ev);
}
hipError_t launch_synthesis_fp32(const SynthArgs& a, hipStream_t s, hipEvent_t* ev) {
  return launch_synthesis<float>(a, s, ev);
}

}  // namespace scw

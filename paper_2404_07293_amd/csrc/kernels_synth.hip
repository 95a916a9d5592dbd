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

#include <type_traits>

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

// ---------------------------------------------------------------- modal sum, FP32
// Phase factors are generated in the block: W(sign)[p][j] = a_j g_f(z_p) +-
// b_j g_b(z_p) for the block's rows' sign, written straight into LDS. Lanes
// read P two complex at a time (16-byte loads); every lane accumulates
// RW rows x ZT planes, and a recursive-halving butterfly leaves the complete
// sum of value index i in lane i (NV = 2 RW ZT values, NV - 1 shuffles).
template <int N>
__device__ __forceinline__ void halve(float* v, int lane) {
  if constexpr (N > 1) {
    constexpr int H = N / 2;
    const bool up = (lane & H) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float send = up ? v[i] : v[i + H];
      const float keep = up ? v[i + H] : v[i];
      v[i] = keep + __shfl_xor(send, H, 64);
    }
    halve<H>(v, lane);
  }
}

// exp(i (re + i im)) for the phase factors of the FP32 modal sum. The angle is
// first reduced to [-pi, pi] by Cody and Waite's two-constant subtraction of
// the nearest multiple of 2 pi, then passed to the hardware sine and cosine;
// the magnitude uses the hardware exponential. The absolute phase error stays
// near 1e-6 for the angles k gamma dz of a layer (up to a few hundred
// radians), well inside the FP32 path's budget, at a fraction of the cost of
// the correctly rounded functions (these factors are rebuilt by every block).
__device__ __forceinline__ float2 cexpi_f(float re, float im) {
  const float n = rintf(re * 0.159154943091895336f);  // re / (2 pi), nearest integer
  float r = fmaf(-n, 6.28318548202514648f, re);       // 2 pi rounded to float
  r = fmaf(n, 1.74845553e-7f, r);                     // minus its rounding error
  const float m = __expf(-im);
  return make_float2(m * __cosf(r), m * __sinf(r));
}

template <int ZT, int RW>
__global__ void __launch_bounds__(256) modal_f32_kernel(
    const float4* __restrict__ P, const float2* __restrict__ kgab, const Task* __restrict__ tasks,
    const float2* __restrict__ tdz, int M, int L, int nb_xy, int nb_z, int jc,
    float2* __restrict__ spec) {
  constexpr int NV = 2 * RW * ZT;
  static_assert(NV <= 64 && (NV & (NV - 1)) == 0, "value count must be a power of two <= 64");
  extern __shared__ float4 sw4[];  // [ZT][jc / 2]
  float2* sw = reinterpret_cast<float2*>(sw4);
  const int n2 = 2 * M, n3 = 3 * M, h2 = M;  // h2 = float4 per row
  const int nb = nb_xy + nb_z;
  const int task = blockIdx.x / nb;
  const int rb = blockIdx.x % nb;
  const Task tk = tasks[task];
  const bool zrows = rb >= nb_xy;
  const int rows_per_block = 4 * RW;
  const int row_begin = zrows ? n2 + (rb - nb_xy) * rows_per_block : rb * rows_per_block;
  const int row_end = zrows ? n3 : n2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = row_begin + wave * RW;
  const float4* Pl = P + (long long)tk.layer * n3 * h2;
  const float2* kg = kgab + (long long)tk.layer * n2;
  const float2* av = kgab + ((long long)L + tk.layer) * n2;
  const float2* bv = kgab + (2LL * L + tk.layer) * n2;
  const float sgn = zrows ? -1.f : 1.f;
  const float4* prow[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) prow[r] = Pl + (long long)min(r0 + r, row_end - 1) * h2;
  float2 dzp[ZT];
#pragma unroll
  for (int p = 0; p < ZT; ++p) dzp[p] = tdz[task * ZT + p];

  float acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.f;

  // The phase table holds jq float4 per plane, jq = jc / 2 rounded up to a
  // multiple of 64, with zeros past the chunk. Every lane then runs the same
  // ceil(qn / 64) steps: a lane past the chunk reads a valid element of its
  // row (the index clamped to the row) and adds its product with a zero
  // weight, which leaves its sums unchanged. Each step first issues its RW
  // loads for the next step unconditionally, into the other of two register
  // sets, so the wait before its products leaves those loads in flight.
  const int jq = (jc / 2 + 63) / 64 * 64;
  float4 pa[RW], pb[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) pa[r] = prow[r][min(lane, h2 - 1)];
  auto step = [&](const float4 (&cur)[RW], float4 (&nxt)[RW], int q, int qg) {
#pragma unroll
    for (int r = 0; r < RW; ++r) nxt[r] = prow[r][qg];
    // keep the loads ahead of this step's products (the scheduler would
    // otherwise sink them to the end of the step)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int p = 0; p < ZT; ++p) {
      const float4 w = sw4[p * jq + q];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        float& re = acc[(r * ZT + p) * 2];
        float& im = acc[(r * ZT + p) * 2 + 1];
        re = fmaf(cur[r].x, w.x, re);
        re = fmaf(-cur[r].y, w.y, re);
        im = fmaf(cur[r].x, w.y, im);
        im = fmaf(cur[r].y, w.x, im);
        re = fmaf(cur[r].z, w.z, re);
        re = fmaf(-cur[r].w, w.w, re);
        im = fmaf(cur[r].z, w.w, im);
        im = fmaf(cur[r].w, w.z, im);
      }
    }
  };
  for (int j0 = 0; j0 < n2; j0 += jc) {
    const int jn = min(jc, n2 - j0);
    __syncthreads();
    for (int jj = threadIdx.x; jj < 2 * jq; jj += 256) {
      if (jj < jn) {
        const float2 g = kg[j0 + jj], a = av[j0 + jj], b = bv[j0 + jj];
#pragma unroll
        for (int p = 0; p < ZT; ++p) {
          const float2 gf = cexpi_f(g.x * dzp[p].x, g.y * dzp[p].x);
          const float2 gb = cexpi_f(-g.x * dzp[p].y, -g.y * dzp[p].y);
          const float fx = a.x * gf.x - a.y * gf.y, fy = a.x * gf.y + a.y * gf.x;
          const float bx = b.x * gb.x - b.y * gb.y, by = b.x * gb.y + b.y * gb.x;
          sw[p * 2 * jq + jj] = make_float2(fx + sgn * bx, fy + sgn * by);
        }
      } else {
#pragma unroll
        for (int p = 0; p < ZT; ++p) sw[p * 2 * jq + jj] = make_float2(0.f, 0.f);
      }
    }
    __syncthreads();
    // step i covers q = lane + 64 i of the chunk and loads element q + 64 of
    // the rows: the next step's, or for the last step the first of the next
    // chunk (chunks before the last hold a multiple of 64 float4)
    const int q0 = j0 / 2, ns = (jn / 2 + 63) / 64;
    int i = 0;
    for (; i + 2 <= ns; i += 2) {
      const int q = lane + 64 * i;
      step(pa, pb, q, min(q0 + q + 64, h2 - 1));
      step(pb, pa, q + 64, min(q0 + q + 128, h2 - 1));
    }
    if (i < ns) {
      const int q = lane + 64 * i;
      step(pa, pb, q, min(q0 + q + 64, h2 - 1));
#pragma unroll
      for (int r = 0; r < RW; ++r) pa[r] = pb[r];
    }
  }
  halve<NV>(acc, lane);
#pragma unroll
  for (int off = NV; off < 64; off <<= 1) acc[0] += __shfl_xor(acc[0], off, 64);
  if (lane < NV) {
    const int comp = lane & 1, p = (lane >> 1) % ZT, r = (lane >> 1) / ZT;
    const int row = r0 + r;
    if (row < row_end && p < tk.count)
      reinterpret_cast<float*>(spec)[((long long)(tk.plane0 + p) * n3 + row) * 2 + comp] = acc[0];
  }
}

template <int ZT, int RW>
hipError_t launch_modal_f32_rw(const SynthArgs& a, hipStream_t s) {
  const int n2 = 2 * a.M;
  const int rows_per_block = 4 * RW;
  const int nb_xy = (n2 + rows_per_block - 1) / rows_per_block;
  const int nb_z = (a.M + rows_per_block - 1) / rows_per_block;
  const size_t max_lds = 64 * 1024;
  int jc = (int)(max_lds / (ZT * sizeof(float2)));
  jc = jc >= n2 ? n2 : (jc / 128) * 128;
  // per plane jc / 2 float4 of phases, padded with zeros to a multiple of 64
  const size_t lds = (size_t)ZT * ((jc / 2 + 63) / 64 * 64) * sizeof(float4);
  const long long nblocks = (long long)a.ntasks * (nb_xy + nb_z);
  if (nblocks == 0) return hipSuccess;
  modal_f32_kernel<ZT, RW><<<(unsigned)nblocks, 256, lds, s>>>(
      reinterpret_cast<const float4*>(a.P), reinterpret_cast<const float2*>(a.kgab32), a.tasks,
      reinterpret_cast<const float2*>(a.task_dz32), a.M, a.L, nb_xy, nb_z, jc,
      reinterpret_cast<float2*>(a.spec));
  return hipGetLastError();
}

// Rows per wave RW with 2 RW ZT <= 64 accumulated values per lane.
template <int ZT>
hipError_t launch_modal_f32(const SynthArgs& a, hipStream_t s) {
  switch (a.modal_rw) {
    case 2: return launch_modal_f32_rw<ZT, 2>(a, s);
    case 4: return launch_modal_f32_rw<ZT, 4>(a, s);
    case 8:
      if constexpr (ZT <= 4) return launch_modal_f32_rw<ZT, 8>(a, s);
      break;
    case 16:
      if constexpr (ZT <= 2) return launch_modal_f32_rw<ZT, 16>(a, s);
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- modal sum, many illuminations
// With several illuminations the columns of a task are (illumination, plane)
// pairs c = ki * zt + p, 32 per launch group, and the product P_l W becomes a
// real GEMM pair on the matrix cores: spec_re = P_re W_re - P_im W_im and
// spec_im = P_re W_im + P_im W_re, four v_mfma_f32_32x32x2f32 per pair of j.
//
// multi_phase_kernel writes the group's phase table once,
// W[task][sign][c][j] = a_kj g_f(z_p) +- b_kj g_b(z_p), zero for j >= 2M
// (rows padded to n2p, a multiple of 16) and for columns past the group.
// modal_multi_kernel: one block = four waves on the same 32 rows of one sign
// category of one task. P and W are staged through LDS in chunks of 64 j,
// read from memory in 512-byte runs per row (the operand layout read straight
// from memory would fetch 128-byte pieces of 32 rows 7 KB apart). Of a
// chunk's four 16-j steps wave w takes step w; the four tiles are added
// through LDS at the end. In the s-th product of a step, lane (i, h)
// (i = lane % 32, h = lane / 32) feeds j = step + 8 h + s: 8 consecutive
// complex of row i of each tile. The next chunk's loads are issued before the
// current chunk's products.
typedef float f32x16 __attribute__((ext_vector_type(16)));

__global__ void multi_phase_kernel(const float2* __restrict__ kg, const float2* __restrict__ ab,
                                   const Task* __restrict__ tasks,
                                   const float2* __restrict__ tdz, int zt, int M, int L, int n2p,
                                   int k0, int kcount, int ntasks, float2* __restrict__ W) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per_task = 32LL * n2p;
  if (t >= (long long)ntasks * per_task) return;
  const int task = (int)(t / per_task);
  const int rem = (int)(t % per_task);
  const int c = rem / n2p, j = rem % n2p;
  const int ki = c / zt, p = c % zt;
  const int n2 = 2 * M;
  float2 wp = make_float2(0.f, 0.f), wm = wp;
  if (j < n2 && ki < kcount) {
    const int layer = tasks[task].layer;
    const float2 g = kg[(long long)layer * n2 + j];
    const float2 dz = tdz[task * zt + p];
    const float2 gf = cexpi_f(g.x * dz.x, g.y * dz.x);
    const float2 gb = cexpi_f(-g.x * dz.y, -g.y * dz.y);
    const float2* abk = ab + (long long)(k0 + ki) * 2 * L * n2;
    const float2 a = abk[(long long)layer * n2 + j];
    const float2 b = abk[((long long)L + layer) * n2 + j];
    const float fx = a.x * gf.x - a.y * gf.y, fy = a.x * gf.y + a.y * gf.x;
    const float bx = b.x * gb.x - b.y * gb.y, by = b.x * gb.y + b.y * gb.x;
    wp = make_float2(fx + bx, fy + by);
    wm = make_float2(fx - bx, fy - by);
  }
  W[(((long long)task * 2 + 0) * 32 + c) * n2p + j] = wp;
  W[(((long long)task * 2 + 1) * 32 + c) * n2p + j] = wm;
}

constexpr int kMultiJ = 64;  // j per staged chunk: four 16-j steps, one per wave

// (up to three waves per SIMD: the staging and operand registers and the
// three accumulators need about 150 registers)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 3)))
modal_multi_kernel(
    const float4* __restrict__ P, const float4* __restrict__ W, const Task* __restrict__ tasks,
    int zt, int M, int fz, int n2p, int k0, int kcount, int ntasks, int nb_xy, int nb_z,
    float2* __restrict__ spec) {
  // the chunk's tiles: [0] 32 rows of P, [1] 32 columns of W, 64 j each,
  // padded by one float4 per row (bank spread); reused for the reduction
  __shared__ float4 tile[2][32][kMultiJ / 2 + 1];
  const int n2 = 2 * M, n3 = 3 * M;
  const int nb = nb_xy + nb_z;
  // Consecutive workgroups go to the eight XCDs in turn; numbering them so
  // that XCD x runs the logical blocks [x per, (x + 1) per) keeps a task's
  // blocks, which all read that task's W, on one XCD and its L2. The grid is
  // padded to 8 per blocks; the padding exits at once.
  const int per = gridDim.x / 8;
  const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (blk >= ntasks * nb) return;
  const int task = blk / nb;
  const int rb = blk % nb;
  const Task tk = tasks[task];
  const bool zrows = rb >= nb_xy;
  const int r0 = zrows ? n2 + (rb - nb_xy) * 32 : rb * 32;
  const int row_end = zrows ? n3 : n2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 31, lh = lane >> 5;
  // staging: thread t copies float4 8 q + t % 8 (q = 0..3) of row t / 8 of
  // both tiles, so that eight lanes read one 128-byte run per load and a
  // row's 512 bytes are read by eight lanes (rows past the end repeat the
  // last row; j past 2M meets zero entries of W, so P there only has to be
  // finite and its index is clamped to the row's last pair)
  const int srow = threadIdx.x >> 3, spart = threadIdx.x & 7;
  const float4* psrc =
      P + ((long long)tk.layer * n3 + min(r0 + srow, row_end - 1)) * (n2 / 2);
  const float4* wsrc = W + (((long long)task * 2 + (zrows ? 1 : 0)) * 32 + srow) * (n2p / 2);
  const int pmax = n2 / 2 - 1, wmax = n2p / 2 - 1;
  const int nsteps = n2p / 16;
  const int nchunks = (nsteps + 3) / 4;
  // three accumulators, so that no operand needs a sign flip:
  // spec_re = rr - ii, spec_im = im
  f32x16 rr, ii, im;
#pragma unroll
  for (int r = 0; r < 16; ++r) rr[r] = ii[r] = im[r] = 0.f;
  // staging registers of one chunk (named scalars, so that they stay in VGPRs)
  float4 p0, p1, p2, p3, w0, w1, w2, w3;
#define SCW_MULTI_LOAD(c)                                 \
  {                                                       \
    const int i0 = (c) * (kMultiJ / 2) + spart;           \
    p0 = psrc[min(i0, pmax)];                             \
    p1 = psrc[min(i0 + 8, pmax)];                         \
    p2 = psrc[min(i0 + 16, pmax)];                        \
    p3 = psrc[min(i0 + 24, pmax)];                        \
    w0 = wsrc[min(i0, wmax)];                             \
    w1 = wsrc[min(i0 + 8, wmax)];                         \
    w2 = wsrc[min(i0 + 16, wmax)];                        \
    w3 = wsrc[min(i0 + 24, wmax)];                        \
  }
  SCW_MULTI_LOAD(0);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();  // the previous tiles have been read
    tile[0][srow][spart] = p0;
    tile[0][srow][8 + spart] = p1;
    tile[0][srow][16 + spart] = p2;
    tile[0][srow][24 + spart] = p3;
    tile[1][srow][spart] = w0;
    tile[1][srow][8 + spart] = w1;
    tile[1][srow][16 + spart] = w2;
    tile[1][srow][24 + spart] = w3;
    __syncthreads();
    // the next chunk's loads are in flight during this chunk's products (the
    // last chunk loads itself again)
    SCW_MULTI_LOAD(min(c + 1, nchunks - 1));
    __builtin_amdgcn_sched_barrier(0);
    if (4 * c + wave < nsteps) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 a = tile[0][li][8 * wave + 4 * lh + q];
        const float4 b = tile[1][li][8 * wave + 4 * lh + q];
        rr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, rr, 0, 0, 0);
        ii = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, ii, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x, im, 0, 0, 0);
        rr = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, rr, 0, 0, 0);
        ii = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, ii, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.w, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.z, im, 0, 0, 0);
      }
    }
  }
#undef SCW_MULTI_LOAD
  // the four waves' tiles are added through LDS
  __syncthreads();
  float* red = reinterpret_cast<float*>(tile);  // [3][32][64]
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      red[((wave - 1) * 32 + r) * 64 + lane] = rr[r] - ii[r];
      red[((wave - 1) * 32 + 16 + r) * 64 + lane] = im[r];
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int ki = li / zt, p = li % zt;
    if (ki < kcount && p < tk.count) {
      float2* dst = spec + ((long long)(k0 + ki) * fz + tk.plane0 + p) * n3;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = r0 + 8 * (r / 4) + 4 * lh + (r % 4);
        float x = rr[r] - ii[r], y = im[r];
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          x += red[(w * 32 + r) * 64 + lane];
          y += red[(w * 32 + 16 + r) * 64 + lane];
        }
        if (row < row_end) dst[row] = make_float2(x, y);
      }
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
// One block per (plane, component, f tile, g tile). The spectrum S[v][u] of the
// plane/component is staged in LDS; each thread owns one output column f:
//   pass x:  T[v][f] = sum_u S[v][u] exp(2 pi i u f / fx)
//            = e^{-2 pi i (U/2) f/fx} * Horner_u(S[v][.], w_f),  w_f = e^{2 pi i f/fx}
//            kept in LDS as T[v][thread];
//   pass y:  E[g][f] = e^{-2 pi i (V/2) g/fy} * Horner_v(T[.][f], w_g)
//            for the block's rows g, four rows at a time sharing each LDS read.
// wx[0][f] = w_f, wx[1][f] = e^{-2 pi i (U/2) f/fx}; wy likewise for g.
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cmuladd(cx<T> a, cx<T> w, cx<T> c) {  // a*w + c
  cx<T> r;
  r.x = fma(a.x, w.x, fma(-a.y, w.y, c.x));
  r.y = fma(a.x, w.y, fma(a.y, w.x, c.y));
  return r;
}

template <typename T, int FT>
__global__ void __launch_bounds__(FT) idft_kernel(
    const cx<T>* __restrict__ spec, const cx<T>* __restrict__ wx, const cx<T>* __restrict__ wy,
    int U, int V, int fx, int fy, int fz, int grows, cx<T>* __restrict__ E) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* S = reinterpret_cast<cx<T>*>(smem_raw);  // [V*U]
  cx<T>* Tt = S + U * V;                          // [V][FT]
  const int M = U * V;
  const int pc = blockIdx.z;
  const int plane = pc / 3, comp = pc % 3;
  const int t = threadIdx.x;
  const int f = blockIdx.x * FT + t;
  const int g0 = blockIdx.y * grows;
  const int g1 = min(fy, g0 + grows);
  const cx<T>* src = spec + ((long long)plane * 3 + comp) * M;
  for (int i = t; i < M; i += FT) S[i] = src[i];
  __syncthreads();
  const bool live = f < fx;
  if (live) {
    const cx<T> w = wx[f], sh = wx[fx + f];
    for (int v = 0; v < V; ++v) {
      const cx<T>* row = S + v * U;
      cx<T> acc = row[U - 1];
      for (int u = U - 2; u >= 0; --u) acc = cmuladd(acc, w, row[u]);
      Tt[v * FT + t] = cmul(acc, sh);
    }
  }
  // each thread reads only its own column of Tt: no barrier needed
  if (!live) return;
  cx<T>* dst = E + (((long long)comp * fz + plane) * fy) * fx + f;
  int g = g0;
  for (; g + 4 <= g1; g += 4) {
    cx<T> w[4], acc[4];
    const cx<T> top = Tt[(V - 1) * FT + t];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[k] = wy[g + k];
      acc[k] = top;
    }
    for (int v = V - 2; v >= 0; --v) {
      const cx<T> c = Tt[v * FT + t];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = cmuladd(acc[k], w[k], c);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const cx<T> o = cmul(acc[k], wy[fy + g + k]);
      __builtin_nontemporal_store(o.x, &dst[(long long)(g + k) * fx].x);
      __builtin_nontemporal_store(o.y, &dst[(long long)(g + k) * fx].y);
    }
  }
  for (; g < g1; ++g) {
    const cx<T> w = wy[g];
    cx<T> acc = Tt[(V - 1) * FT + t];
    for (int v = V - 2; v >= 0; --v) acc = cmuladd(acc, w, Tt[v * FT + t]);
    const cx<T> o = cmul(acc, wy[fy + g]);
    __builtin_nontemporal_store(o.x, &dst[(long long)g * fx].x);
    __builtin_nontemporal_store(o.y, &dst[(long long)g * fx].y);
  }
}

// ---------------------------------------------------------------- inverse DFT, factored
// For fy = R * P with P in {2, 4, 8, 16, 32} and V <= 32. One block per
// (plane/component, 64 columns f); threads are 64 columns x 4 groups.
//   x pass: T[v][f] by Horner (as above) into 32 zero-padded slots s = v + 16.
//   y pass: write g = g1 + R g2. With w = exp(2 pi i / fy), w^R = exp(2 pi i / P):
//     E[g1 + R g2] = sum_r A[r] exp(2 pi i r g2 / P),
//     A[r] = sum_{v = r mod P} T[v] w^(v g1),
//   so each (column, g1) costs 32 twiddle MACs plus one P-point FFT held in
//   registers, and writes P outputs; each store writes 64 consecutive columns.
// cos(2 pi r / 32) for r = 0..8: the first quadrant of the twiddles of every
// radix P <= 32 (e^{2 pi i k / P} is entry k * 32 / P of the full circle).
__device__ __forceinline__ double quarter_cos(int r) {
  switch (r) {
    case 0: return 1.0;
    case 1: return 0.98078528040323044913;
    case 2: return 0.92387953251128675613;
    case 3: return 0.83146961230254523708;
    case 4: return 0.70710678118654752440;
    case 5: return 0.55557023301960222474;
    case 6: return 0.38268343236508977173;
    case 7: return 0.19509032201612826785;
    default: return 0.0;
  }
}

// v * e^{2 pi i k / P} for a k known at compile time once the caller's loops
// are unrolled: no multiply for k = 0, a swap for the quarter turn, and the
// constant folded in otherwise.
template <typename T, int P>
__device__ __forceinline__ cx<T> twiddle_mul(cx<T> v, int k) {
  const int k32 = (k * (32 / P)) & 31;
  if (k32 == 0) return v;
  if (k32 == 8) return {-v.y, v.x};
  if (k32 == 16) return {-v.x, -v.y};
  if (k32 == 24) return {v.y, -v.x};
  const int q = k32 >> 3, r = k32 & 7;
  const T c0 = (T)quarter_cos(r), s0 = (T)quarter_cos(8 - r);
  const T c = q == 0 ? c0 : (q == 1 ? -s0 : (q == 2 ? -c0 : s0));
  const T sn = q == 0 ? s0 : (q == 1 ? c0 : (q == 2 ? -s0 : -c0));
  return {v.x * c - v.y * sn, v.x * sn + v.y * c};
}

// In-register radix-2 FFT of length P with positive exponent:
// a[g2] <- sum_r a[r] e^{2 pi i r g2 / P}.
template <typename T, int P>
__device__ __forceinline__ void small_fft(cx<T>* a) {
  // bit-reversal permutation
#pragma unroll
  for (int i = 0; i < P; ++i) {
    int r = 0;
#pragma unroll
    for (int b = 1, x = i; b < P; b <<= 1, x >>= 1) r = (r << 1) | (x & 1);
    if (r > i) {
      const cx<T> tmp = a[i];
      a[i] = a[r];
      a[r] = tmp;
    }
  }
#pragma unroll
  for (int len = 2; len <= P; len <<= 1) {
#pragma unroll
    for (int i = 0; i < P; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const cx<T> u = a[i + j];
        const cx<T> t = twiddle_mul<T, P>(a[i + j + len / 2], j * (P / len));
        a[i + j] = {u.x + t.x, u.y + t.y};
        a[i + j + len / 2] = {u.x - t.x, u.y - t.y};
      }
    }
  }
}

// One non-temporal store of a whole complex value (the field is written once
// and not read back by the synthesis).
__device__ __forceinline__ void store_nt(cx<float>* d, cx<float> v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(f2v{v.x, v.y}, reinterpret_cast<f2v*>(d));
}
__device__ __forceinline__ void store_nt(cx<double>* d, cx<double> v) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(d2v{v.x, v.y}, reinterpret_cast<d2v*>(d));
}

// COLS columns per block (64 or 32); the 256 threads are COLS columns x
// 256 / COLS groups, each group taking every (256 / COLS)-th row in the x
// pass and g1 value in the y pass. The occupied frequency slots are lo..hi
// (slot = v + 16); the y pass runs over rounds of P slots that start at
// multiples of P, so that a slot's residue (slot - 16) mod P is fixed at
// compile time, and the slots of those rounds outside lo..hi hold zeros.
template <typename T, int P, int COLS>
__global__ void __launch_bounds__(256) idft_fft_kernel(
    const cx<T>* __restrict__ spec, const cx<T>* __restrict__ wx, const cx<T>* __restrict__ tw1g,
    int U, int V, int fx, int fy, int fz, cx<T>* __restrict__ E) {
  constexpr int NG = 256 / COLS;
  extern __shared__ unsigned char smem_raw[];
  const int R = fy / P;
  cx<T>* S = reinterpret_cast<cx<T>*>(smem_raw);  // [V*U]
  cx<T>* Ts = S + U * V;                          // [32][COLS]
  cx<T>* tw1 = Ts + 32 * COLS;                    // [R][32]: w^((s-16) g1)
  const int M = U * V;
  const int pc = blockIdx.y;
  const int plane = pc / 3, comp = pc % 3;
  const int t = threadIdx.x, col = t % COLS, q = t / COLS;
  const int f = blockIdx.x * COLS + col;
  const bool live = f < fx;
  const int lo = 16 - V / 2, hi = 16 + V / 2;
  const int s_begin = (lo / P) * P, s_end = (hi / P + 1) * P;
  const cx<T>* src = spec + (long long)pc * M;
  for (int i = t; i < M; i += 256) S[i] = src[i];
  for (int i = t; i < 32 * R; i += 256) tw1[i] = tw1g[i];
  {
    const int zl = lo - s_begin, zh = s_end - hi - 1;
    for (int i = t; i < (zl + zh) * COLS; i += 256) {
      const int rr = i / COLS, cc = i % COLS;
      const int sl = rr < zl ? s_begin + rr : hi + 1 + (rr - zl);
      Ts[sl * COLS + cc] = {0, 0};
    }
  }
  __syncthreads();
  if (live) {
    const cx<T> w = wx[f], sh = wx[fx + f];
    for (int vi = q; vi < V; vi += NG) {
      const cx<T>* row = S + vi * U;
      cx<T> acc = row[U - 1];
      for (int u = U - 2; u >= 0; --u) acc = cmuladd(acc, w, row[u]);
      Ts[(vi - V / 2 + 16) * COLS + col] = cmul(acc, sh);
    }
  }
  __syncthreads();
  if (!live) return;
  const cx<T>* tc = Ts + col;
  cx<T>* dst = E + (((long long)comp * fz + plane) * fy) * fx + f;
  const long long step = (long long)R * fx;
  for (int g1 = q; g1 < R; g1 += NG) {
    const cx<T>* tw = tw1 + g1 * 32;
    cx<T> a[P];
#pragma unroll
    for (int r = 0; r < P; ++r) a[r] = {0, 0};
    for (int s0 = s_begin; s0 < s_end; s0 += P) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int r = (i - 16) & (P - 1);
        const cx<T> tv = tc[(s0 + i) * COLS], w1 = tw[s0 + i];
        a[r].x = fma(tv.x, w1.x, fma(-tv.y, w1.y, a[r].x));
        a[r].y = fma(tv.x, w1.y, fma(tv.y, w1.x, a[r].y));
      }
    }
    small_fft<T, P>(a);
    cx<T>* d = dst + (long long)g1 * fx;  // row g1 + R g2
#pragma unroll
    for (int g2 = 0; g2 < P; ++g2) store_nt(d + g2 * step, a[g2]);
  }
}

// ---------------------------------------------------------------- lateral slice
// Eq. 10 on an x-z (axis 0) or y-z (axis 1) plane. One block per plane and
// component: the spectrum's other lateral index is summed first with the
// phase of the slice position, T[k] = sum_j S e^{2 pi i (j - J/2) frac}
// (in FP64; the J phases per block are few), then the kept index runs on the
// n samples by Horner's rule as in the volume's x pass.
template <typename T>
__global__ void __launch_bounds__(256) slice_kernel(const cx<T>* __restrict__ spec,
                                                    const cx<T>* __restrict__ tw, int U, int V,
                                                    int n, int fz, int axis, double frac,
                                                    cx<T>* __restrict__ E) {
  extern __shared__ unsigned char smem_raw[];
  cx<T>* S = reinterpret_cast<cx<T>*>(smem_raw);  // [V][U]
  cx<T>* Tk = S + U * V;                          // [K]
  const int M = U * V, pc = blockIdx.x;
  const cx<T>* src = spec + (long long)pc * M;
  for (int i = threadIdx.x; i < M; i += blockDim.x) S[i] = src[i];
  __syncthreads();
  const int K = axis == 0 ? U : V, J = axis == 0 ? V : U;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < J; ++j) {
      double sn, cs;
      sincospi(2.0 * (j - J / 2) * frac, &sn, &cs);
      const cx<T> v = axis == 0 ? S[j * U + k] : S[k * U + j];
      re += (double)v.x * cs - (double)v.y * sn;
      im += (double)v.x * sn + (double)v.y * cs;
    }
    Tk[k] = {(T)re, (T)im};
  }
  __syncthreads();
  const int plane = pc / 3, comp = pc % 3;
  cx<T>* dst = E + ((long long)comp * fz + plane) * n;
  for (int f = threadIdx.x; f < n; f += blockDim.x) {
    const cx<T> w = tw[f], sh = tw[n + f];
    cx<T> acc = Tk[K - 1];
    for (int k = K - 2; k >= 0; --k) acc = cmuladd(acc, w, Tk[k]);
    dst[f] = cmul(acc, sh);
  }
}

// ---------------------------------------------------------------- objective, intensity
// An ideal objective's coherent transfer function on the per-plane spectra:
// modes whose direction sine exceeds the numerical aperture are removed.
template <typename T>
__global__ void objective_kernel(cx<T>* __restrict__ spec, long long n, int M, int U, int V,
                                 double sx_step, double sy_step, double na2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = (int)(i % M);
  const double sx = (m % U - U / 2) * sx_step, sy = (m / U - V / 2) * sy_step;
  if (sx * sx + sy * sy > na2) spec[i] = {0, 0};
}

// A general transfer function on the per-plane spectra: every mode's
// coefficients times H[m] (complex128, applied in FP64).
template <typename T>
__global__ void transfer_kernel(cx<T>* __restrict__ spec, long long n, int M,
                                const double2* __restrict__ H) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 h = H[i % M];
  const cx<T> v = spec[i];
  spec[i] = {(T)((double)v.x * h.x - (double)v.y * h.y), (T)((double)v.x * h.y + (double)v.y * h.x)};
}

template <typename T>
__global__ void intensity_kernel(const cx<T>* __restrict__ E, T* __restrict__ I, long long npix) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  const cx<T> a = E[i], b = E[npix + i], c = E[2 * npix + i];
  I[i] = a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y + c.x * c.x + c.y * c.y;
}

template <typename T>
hipError_t launch_idft_fft(const SynthArgs& a, hipStream_t s) {
  const int P = a.fft_p, R = a.fy / P;
  const int cols = a.idft_gtiles == 32 ? 32 : 64;  // columns per block
  const size_t lds = ((size_t)a.U * a.V + 32 * (size_t)cols + 32 * (size_t)R) * sizeof(cx<T>);
  dim3 grid((a.fx + cols - 1) / cols, a.fz * 3);
  const cx<T>* tw1 = reinterpret_cast<const cx<T>*>(a.fft_tw);
  auto go = [&](auto kern) {
    kern<<<grid, 256, lds, s>>>(reinterpret_cast<const cx<T>*>(a.spec),
                                reinterpret_cast<const cx<T>*>(a.twx), tw1, a.U, a.V, a.fx,
                                a.fy, a.fz, reinterpret_cast<cx<T>*>(a.E));
  };
  auto radix = [&](auto cols_tag) -> hipError_t {
    constexpr int C = decltype(cols_tag)::value;
    switch (P) {
      case 2: go(idft_fft_kernel<T, 2, C>); break;
      case 4: go(idft_fft_kernel<T, 4, C>); break;
      case 8: go(idft_fft_kernel<T, 8, C>); break;
      case 16: go(idft_fft_kernel<T, 16, C>); break;
      case 32: go(idft_fft_kernel<T, 32, C>); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  return cols == 32 ? radix(std::integral_constant<int, 32>())
                    : radix(std::integral_constant<int, 64>());
}

template <typename T>
hipError_t launch_idft(const SynthArgs& a, hipStream_t s) {
  const int n_pc = a.fz * 3;
  auto go = [&](auto ft_tag) -> hipError_t {
    constexpr int FT = decltype(ft_tag)::value;
    const int nft = (a.fx + FT - 1) / FT;
    // enough g tiles for ~2 blocks per CU, but at least 64 rows per tile
    int ng = 1;
    while ((long long)n_pc * nft * ng < 512 && a.fy / (ng * 2) >= 64) ng *= 2;
    if (a.idft_gtiles > 0) ng = a.idft_gtiles;
    const int grows = (a.fy + ng - 1) / ng;
    const size_t lds = ((size_t)a.U * a.V + (size_t)a.V * FT) * sizeof(cx<T>);
    dim3 grid(nft, (a.fy + grows - 1) / grows, n_pc);
    idft_kernel<T, FT><<<grid, FT, lds, s>>>(
        reinterpret_cast<const cx<T>*>(a.spec), reinterpret_cast<const cx<T>*>(a.twx),
        reinterpret_cast<const cx<T>*>(a.twy), a.U, a.V, a.fx, a.fy, a.fz, grows,
        reinterpret_cast<cx<T>*>(a.E));
    return hipGetLastError();
  };
  if (a.fx <= 64) return go(std::integral_constant<int, 64>());
  if (a.fx <= 128) return go(std::integral_constant<int, 128>());
  return go(std::integral_constant<int, 256>());
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
  const bool modal = (a.stages & kStageModal) != 0;
  if (!modal) {
    if ((e = mark(1)) != hipSuccess) return e;
  } else if (a.ntasks > 0 && sizeof(T) == 8) {
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
  } else if (a.ntasks > 0) {
    if ((e = mark(1)) != hipSuccess) return e;
    switch (a.zt) {
      case 1: e = launch_modal_f32<1>(a, s); break;
      case 2: e = launch_modal_f32<2>(a, s); break;
      case 4: e = launch_modal_f32<4>(a, s); break;
      case 8: e = launch_modal_f32<8>(a, s); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  } else if ((e = mark(1)) != hipSuccess) {
    return e;
  }
  if ((e = mark(2)) != hipSuccess) return e;
  if (a.n_ext > 0 && (a.stages & kStageExterior)) {
    exterior_kernel<T><<<blocks_for((long long)a.n_ext * 3 * a.M, 256), 256, 0, s>>>(
        reinterpret_cast<const ExtPlane*>(a.ext_planes), a.n_ext, a.M,
        reinterpret_cast<const zd*>(a.ext), reinterpret_cast<const zd*>(a.ksz),
        reinterpret_cast<cx<T>*>(a.spec));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = mark(3)) != hipSuccess) return e;
  if (!(a.stages & kStageTransform)) {
    // transform not requested
  } else if (a.fft_p > 0) {
    if ((e = launch_idft_fft<T>(a, s)) != hipSuccess) return e;
  } else if (sizeof(T) == 4 && a.mfma) {
    MfmaArgs m{a.U, a.V, a.fx, a.fy, a.fz, a.kp, a.idft_gtiles, a.spec, a.twx, a.bmat, a.bscale, a.amat, a.E};
    if ((e = launch_idft_mfma(m, a.precision, s)) != hipSuccess) return e;
  } else if ((e = launch_idft<T>(a, s)) != hipSuccess) {
    return e;
  }
  return mark(4);
}

}  // namespace

hipError_t launch_modal_multi(const void* P, const void* kg, const void* ab, const Task* tasks,
                              const void* task_dz32, int ntasks, int zt, int M, int L, int fz,
                              int k0, int kcount, void* W, void* spec, hipStream_t s) {
  if (zt < 1 || zt > 8 || 32 % zt != 0 || kcount < 1 || kcount * zt > 32)
    return hipErrorInvalidValue;
  if (ntasks == 0) return hipSuccess;
  const int n2p = multi_row_pitch(M);
  multi_phase_kernel<<<blocks_for((long long)ntasks * 32 * n2p, 256), 256, 0, s>>>(
      reinterpret_cast<const float2*>(kg), reinterpret_cast<const float2*>(ab), tasks,
      reinterpret_cast<const float2*>(task_dz32), zt, M, L, n2p, k0, kcount, ntasks,
      reinterpret_cast<float2*>(W));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb_xy = (2 * M + 31) / 32, nb_z = (M + 31) / 32;
  const long long nblocks = (long long)ntasks * (nb_xy + nb_z);
  modal_multi_kernel<<<(unsigned)((nblocks + 7) / 8 * 8), 256, 0, s>>>(
      reinterpret_cast<const float4*>(P), reinterpret_cast<const float4*>(W), tasks, zt, M, fz,
      n2p, k0, kcount, ntasks, nb_xy, nb_z, reinterpret_cast<float2*>(spec));
  return hipGetLastError();
}

hipError_t launch_synthesis_fp64(const SynthArgs& a, hipStream_t s, hipEvent_t* ev) {
  return launch_synthesis<double>(a, s, ev);
}
hipError_t launch_objective(void* spec, long long n, int M, int U, int V, double sx_step,
                            double sy_step, double na, bool fp64, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = blocks_for(n, 256);
  if (fp64)
    objective_kernel<double><<<nb, 256, 0, s>>>(reinterpret_cast<cx<double>*>(spec), n, M, U, V,
                                                sx_step, sy_step, na * na);
  else
    objective_kernel<float><<<nb, 256, 0, s>>>(reinterpret_cast<cx<float>*>(spec), n, M, U, V,
                                               sx_step, sy_step, na * na);
  return hipGetLastError();
}

hipError_t launch_transfer(void* spec, long long n, int M, const void* H, bool fp64,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = blocks_for(n, 256);
  const double2* h = reinterpret_cast<const double2*>(H);
  if (fp64)
    transfer_kernel<double><<<nb, 256, 0, s>>>(reinterpret_cast<cx<double>*>(spec), n, M, h);
  else
    transfer_kernel<float><<<nb, 256, 0, s>>>(reinterpret_cast<cx<float>*>(spec), n, M, h);
  return hipGetLastError();
}

hipError_t launch_intensity(const void* E, void* I, long long npix, bool fp64, hipStream_t s) {
  if (npix <= 0) return hipSuccess;
  const unsigned nb = blocks_for(npix, 256);
  if (fp64)
    intensity_kernel<double><<<nb, 256, 0, s>>>(reinterpret_cast<const cx<double>*>(E),
                                                reinterpret_cast<double*>(I), npix);
  else
    intensity_kernel<float><<<nb, 256, 0, s>>>(reinterpret_cast<const cx<float>*>(E),
                                               reinterpret_cast<float*>(I), npix);
  return hipGetLastError();
}

hipError_t launch_slice(const SliceArgs& a, bool fp64, hipStream_t s) {
  const int K = a.axis == 0 ? a.U : a.V;
  if (a.fz * 3 < 1) return hipSuccess;
  auto go = [&](auto tag) -> hipError_t {
    using T = decltype(tag);
    const size_t lds = ((size_t)a.U * a.V + K) * sizeof(cx<T>);
    slice_kernel<T><<<a.fz * 3, 256, lds, s>>>(
        reinterpret_cast<const cx<T>*>(a.spec), reinterpret_cast<const cx<T>*>(a.tw), a.U, a.V,
        a.n, a.fz, a.axis, a.frac, reinterpret_cast<cx<T>*>(a.E));
    return hipGetLastError();
  };
  return fp64 ? go(double{}) : go(float{});
}

// Copies a field [np][fy][fx] (np = 3 fz plane-components) into the window
// at (ox, oy) of a wider field [np][dfy][dfx], rx x ry times side by side.
template <typename T>
__global__ void place_kernel(const cx<T>* __restrict__ src, int fx, int fy, long long total,
                             cx<T>* __restrict__ dst, int dfx, int dfy, int ox, int oy, int rx,
                             int ry) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int f = (int)(i % fx);
  const long long q = i / fx;
  const int g = (int)(q % fy);
  const long long pc = q / fy;
  const cx<T> v = src[i];
  for (int ty = 0; ty < ry; ++ty) {
    cx<T>* row = dst + (pc * dfy + oy + (long long)ty * fy + g) * dfx + ox + f;
    for (int tx = 0; tx < rx; ++tx) row[(long long)tx * fx] = v;
  }
}

hipError_t launch_place(const void* src, int fx, int fy, int fz, void* dst, int dfx, int dfy,
                        int ox, int oy, int rx, int ry, bool fp64, hipStream_t s) {
  const long long total = 3LL * fz * fy * fx;
  if (total <= 0) return hipSuccess;
  const unsigned nb = blocks_for(total, 256);
  if (fp64)
    place_kernel<double><<<nb, 256, 0, s>>>(reinterpret_cast<const cx<double>*>(src), fx, fy,
                                            total, reinterpret_cast<cx<double>*>(dst), dfx, dfy,
                                            ox, oy, rx, ry);
  else
    place_kernel<float><<<nb, 256, 0, s>>>(reinterpret_cast<const cx<float>*>(src), fx, fy,
                                           total, reinterpret_cast<cx<float>*>(dst), dfx, dfy,
                                           ox, oy, rx, ry);
  return hipGetLastError();
}

hipError_t launch_synthesis_fp32(const SynthArgs& a, hipStream_t s, hipEvent_t* ev) {
  return launch_synthesis<float>(a, s, ev);
}

}  // namespace scw

// Batched synthesis of many solved problems (wavelengths x patches of uneven
// truncation) in one persistent launch, for grids that lie outside the
// samples (Eq. 9 then Eq. 10): the transmitted field below each sample, or
// incident + reflected above it.
//
// Work item = (job, plane, 64-column tile), all three components. Items are
// sorted by cost (largest truncation first) and drained from an atomic
// counter by a persistent grid, `chunk` consecutive items per grab (items
// next to each other in the sorted order cost about the same, and fewer grabs
// mean less contention on the one counter); every block exits once the
// counter passes the item count. Per item, in one block:
//   spectra   S[c][v][u] = exterior coefficients of the job at the plane (LDS),
//             one set of phase factors for the three components
//   x pass    T[v][f] into 32 frequency slots: factored (one 8-point register
//             FFT per row and column group) when fx is a power of two up to
//             64, else by Horner over u per column
//   y pass    factored transform, fy = R * P (as in the single-problem path),
//             over the rounds of P slots that hold the V occupied ones
#include <hip/hip_runtime.h>

#include "scw_internal.h"

namespace scw {
namespace {

struct c32 {
  float x, y;
};
__device__ __forceinline__ c32 muladd(c32 a, c32 w, c32 c) {  // a*w + c
  return {fmaf(a.x, w.x, fmaf(-a.y, w.y, c.x)), fmaf(a.x, w.y, fmaf(a.y, w.x, c.y))};
}
__device__ __forceinline__ c32 mul(c32 a, c32 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// exp(i (re + i im)): the angle reduced to [-pi, pi] by Cody and Waite's
// two-constant subtraction of the nearest multiple of 2 pi, then the hardware
// sine, cosine and exponential (absolute error near 1e-6 for the angles
// k s_z dz of an exterior plane, a few tens of radians).
__device__ __forceinline__ c32 cexpi(float re, float im) {
  const float n = rintf(re * 0.159154943091895336f);
  float r = fmaf(-n, 6.28318548202514648f, re);
  r = fmaf(n, 1.74845553e-7f, r);
  const float m = __expf(-im);
  return {m * __cosf(r), m * __sinf(r)};
}

// cos(2 pi r / 32) for r = 0..8: the first quadrant of the twiddles of every
// radix P <= 32.
__device__ __forceinline__ float quarter_cos(int r) {
  switch (r) {
    case 0: return 1.0f;
    case 1: return 0.98078528040323044913f;
    case 2: return 0.92387953251128675613f;
    case 3: return 0.83146961230254523708f;
    case 4: return 0.70710678118654752440f;
    case 5: return 0.55557023301960222474f;
    case 6: return 0.38268343236508977173f;
    case 7: return 0.19509032201612826785f;
    default: return 0.0f;
  }
}

// v * e^{2 pi i k / P}, k known at compile time after unrolling.
template <int P>
__device__ __forceinline__ c32 twiddle_mul(c32 v, int k) {
  const int k32 = (k * (32 / P)) & 31;
  if (k32 == 0) return v;
  if (k32 == 8) return {-v.y, v.x};
  if (k32 == 16) return {-v.x, -v.y};
  if (k32 == 24) return {v.y, -v.x};
  const int q = k32 >> 3, r = k32 & 7;
  const float c0 = quarter_cos(r), s0 = quarter_cos(8 - r);
  const float c = q == 0 ? c0 : (q == 1 ? -s0 : (q == 2 ? -c0 : s0));
  const float sn = q == 0 ? s0 : (q == 1 ? c0 : (q == 2 ? -s0 : -c0));
  return {v.x * c - v.y * sn, v.x * sn + v.y * c};
}

// In-register radix-2 FFT of length P, positive exponent.
template <int P>
__device__ __forceinline__ void small_fft(c32* a) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    int r = 0;
#pragma unroll
    for (int b = 1, x = i; b < P; b <<= 1, x >>= 1) r = (r << 1) | (x & 1);
    if (r > i) {
      const c32 tmp = a[i];
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
        const c32 u = a[i + j];
        const c32 t = twiddle_mul<P>(a[i + j + len / 2], j * (P / len));
        a[i + j] = {u.x + t.x, u.y + t.y};
        a[i + j + len / 2] = {u.x - t.x, u.y - t.y};
      }
    }
  }
}

constexpr int COLS = 64;

__global__ void reset_counter(unsigned int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

// One work item by the whole block: the three field components of one (job,
// plane, 64-column tile). The exterior phase factors of the plane are formed
// once and applied to the three components' coefficients (Eq. 9), giving the
// spectra S[3][M] in LDS; each component then takes the x pass into Ts and
// the factored y pass. The caller synchronises before S and Ts are
// overwritten.
template <int P>
__device__ __forceinline__ void batch_item(
    const BatchItem item, const BatchJob* __restrict__ jobs,
    const BatchPlane* __restrict__ planes, const c32* __restrict__ coef,
    const c32* __restrict__ wfull, const c32* tw1, const c32* wl, int fx, int fy, int fz,
    c32* S, c32* Ts, c32* __restrict__ E) {
  const int R = fy / P;
  const int t = threadIdx.x, col = t % COLS, q = t / COLS;
  const BatchJob jb = jobs[item.job];
  const BatchPlane pl = planes[(long long)item.job * fz + item.plane];
  const int U = jb.U, V = jb.V, M = U * V;
  const c32* cf = coef + jb.coef_offset;  // [3][M] p_inc, [3][M] p_ref, [3][M] p_trn, [M] k sz_top, [M] k sz_bot
  for (int m = t; m < M; m += 256) {
    if (pl.kind == 0) {  // above the sample: incident + reflected
      const c32 kz = cf[9 * M + m];
      const c32 gi = cexpi(kz.x * pl.dz, kz.y * pl.dz);
      const c32 gr = cexpi(-kz.x * pl.dz, -kz.y * pl.dz);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const c32 x = mul(cf[c * M + m], gi), y = mul(cf[(3 + c) * M + m], gr);
        S[c * M + m] = {x.x + y.x, x.y + y.y};
      }
    } else {  // below: transmitted
      const c32 kz = cf[10 * M + m];
      const c32 g = cexpi(kz.x * pl.dz, kz.y * pl.dz);
#pragma unroll
      for (int c = 0; c < 3; ++c) S[c * M + m] = mul(cf[(6 + c) * M + m], g);
    }
  }
  const int f = item.ftile * COLS + col;
  const bool live = f < fx;
  c32 w = {0.f, 0.f}, sh = {0.f, 0.f};
  if (live) {
    w = wfull[f];
    int sidx = (int)(((long long)(-(U / 2)) * f) % fx);
    if (sidx < 0) sidx += fx;
    sh = wfull[sidx];
  }
  // Occupied frequency slots lo..hi (slot = v + 16). The y pass runs over
  // rounds of P slots that start at multiples of P, so that a slot's residue
  // (slot - 16) mod P is fixed at compile time; the slots of those rounds
  // outside lo..hi hold zeros, written once per item (the x pass writes only
  // lo..hi, and the rows are the same for the three components).
  const int lo = 16 - V / 2, hi = 16 + V / 2;
  const int s_begin = (lo / P) * P, s_end = (hi / P + 1) * P;
  {
    const int zl = lo - s_begin, zh = s_end - hi - 1;
    for (int i = t; i < (zl + zh) * COLS; i += 256) {
      const int rr = i / COLS, cc = i % COLS;
      const int sl = rr < zl ? s_begin + rr : hi + 1 + (rr - zl);
      Ts[sl * COLS + cc] = {0.f, 0.f};
    }
  }
  // x pass in factored form when the row is one tile of fx = 8 Rx columns:
  // T[v][g1 + Rx g2] = sum_r e^{2 pi i r g2 / 8} A[r],
  // A[r] = sum_{u = r mod 8} S[v][u] e^{2 pi i u g1 / fx}   (u from -U/2).
  // u runs in rounds of 8 from a multiple of 8, so u mod 8 is the position in
  // the round; terms outside [-U/2, U/2] are skipped by a predicate.
  const bool xfact = wl != nullptr;
  const int Rx = fx >> 3;
  const int h = U / 2, u0 = -((h + 7) & ~7), xmask = fx - 1;
  for (int comp = 0; comp < 3; ++comp) {
    __syncthreads();  // S complete (first component) / Ts consumed (later ones)
    const c32* Sc = S + comp * M;
    if (xfact) {
      if (t < V * Rx) {
        const int v = t / Rx, g1 = t % Rx;
        const c32* row = Sc + v * U + h;  // row[u] for u in [-h, h]
        c32 a[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r] = {0.f, 0.f};
        for (int ub = u0; ub <= h; ub += 8) {
          const int kb = ub * g1;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int u = ub + i;
            c32 sv = {0.f, 0.f};
            if ((unsigned)(u + h) <= (unsigned)(2 * h)) sv = row[u];
            a[i] = muladd(sv, wl[(kb + i * g1) & xmask], a[i]);
          }
        }
        small_fft<8>(a);
        c32* trow = Ts + (v - V / 2 + 16) * COLS + g1;
#pragma unroll
        for (int g2 = 0; g2 < 8; ++g2) trow[Rx * g2] = a[g2];
      }
    } else if (live) {
      for (int vi = q; vi < V; vi += 4) {
        const c32* row = Sc + vi * U;
        c32 acc = row[U - 1];
        for (int u = U - 2; u >= 0; --u) acc = muladd(acc, w, row[u]);
        Ts[(vi - V / 2 + 16) * COLS + col] = mul(acc, sh);
      }
    }
    __syncthreads();
    if (!live) continue;
    const c32* tc = Ts + col;
    c32* dst = E + ((((long long)item.job * 3 + comp) * fz + item.plane) * fy) * fx + f;
    for (int g1 = q; g1 < R; g1 += 4) {
      const c32* tw = tw1 + g1 * 32;  // e^{2 pi i (slot - 16) g1 / fy}
      c32 a[P];
#pragma unroll
      for (int r = 0; r < P; ++r) a[r] = {0.f, 0.f};
      for (int s0 = s_begin; s0 < s_end; s0 += P) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const int r = (i - 16) & (P - 1);
          a[r] = muladd(tc[(s0 + i) * COLS], tw[s0 + i], a[r]);
        }
      }
      small_fft<P>(a);
      typedef float f2v __attribute__((ext_vector_type(2)));
      f2v* d = reinterpret_cast<f2v*>(dst + (long long)g1 * fx);  // row g1 + R g2
      const long long step = (long long)R * fx;
#pragma unroll
      for (int g2 = 0; g2 < P; ++g2) __builtin_nontemporal_store(f2v{a[g2].x, a[g2].y}, d + g2 * step);
    }
  }
}

template <int P>
__global__ void __launch_bounds__(256) batch_kernel(
    const BatchJob* __restrict__ jobs, const BatchItem* __restrict__ items, int n_items,
    const BatchPlane* __restrict__ planes, const c32* __restrict__ coef,
    const c32* __restrict__ wfull, const c32* __restrict__ tw1g, int fx, int fy, int fz,
    int mmax, int chunk, unsigned int* __restrict__ counter, c32* __restrict__ E) {
  __shared__ c32 Ts[32 * COLS];
  __shared__ c32 wls[COLS];
  __shared__ int s_item;
  extern __shared__ unsigned char smem_raw[];
  const int R = fy / P;
  c32* tw1 = reinterpret_cast<c32*>(smem_raw);  // [R][32]
  c32* S = tw1 + 32 * R;                        // [3][mmax]
  const int t = threadIdx.x;
  for (int i = t; i < 32 * R; i += 256) tw1[i] = tw1g[i];
  // the factored x pass needs fx = 8 Rx <= 64 columns, a power of two
  const bool xfact = fx >= 8 && fx <= COLS && (fx & (fx - 1)) == 0;
  if (xfact && t < fx) wls[t] = wfull[t];
  for (;;) {
    __syncthreads();  // also: the previous grab's last item is consumed
    if (t == 0) s_item = (int)atomicAdd(counter, (unsigned)chunk);
    __syncthreads();
    const int first = s_item;
    if (first >= n_items) break;  // every block reaches this once the queue is drained
    const int last = min(first + chunk, n_items);
    for (int it = first; it < last; ++it) {
      if (it > first) __syncthreads();  // the previous item's S and Ts are consumed
      batch_item<P>(items[it], jobs, planes, coef, wfull, tw1, xfact ? wls : nullptr, fx, fy, fz,
                    S, Ts, E);
    }
  }
}

}  // namespace

hipError_t launch_batch(const BatchArgs& a, hipStream_t s) {
  reset_counter<<<1, 64, 0, s>>>(a.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int R = a.fy / a.P;
  const size_t lds = (32 * (size_t)R + 3 * (size_t)a.mmax) * sizeof(c32);
  auto go = [&](auto kern) {
    kern<<<a.grid, 256, lds, s>>>(a.jobs, a.items, a.n_items, a.planes,
                                  reinterpret_cast<const c32*>(a.coef),
                                  reinterpret_cast<const c32*>(a.wfull),
                                  reinterpret_cast<const c32*>(a.tw1), a.fx, a.fy, a.fz,
                                  a.mmax, a.chunk, a.counter, reinterpret_cast<c32*>(a.E));
  };
  switch (a.P) {
    case 2: go(batch_kernel<2>); break;
    case 4: go(batch_kernel<4>); break;
    case 8: go(batch_kernel<8>); break;
    case 16: go(batch_kernel<16>); break;
    case 32: go(batch_kernel<32>); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace scw

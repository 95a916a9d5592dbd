// Inference of the spectral-convolution surrogate in its matrix-core mode,
// with every activation and spectrum stored in bf16.
//
// In this mode both operands of every matrix product are rounded to bf16
// (nearest even) and the sums stay FP32. Each stored tensor is used only as
// an operand of such products: the activations h (forward transform and
// pointwise map of the next layer, the head), the spectra H (mixing) and the
// mixed spectra G (inverse transform). Storing them already rounded therefore
// gives the same operands, bit for bit, at half the memory traffic of FP32.
// The products run on v_mfma_f32_32x32x16_bf16. Only the order of the FP32
// sums differs from the vector-unit kernels that the training path uses.
//
// Storage: h[b][c][y][x] (bf16); spectra and mixed spectra as packed complex
// bf16 (one 32-bit word: real part in the low half), H[m][b][c] mode-major
// and G[b][m][o]. The layer modes are ky in [-8, 8] (17 rows of the table) x
// kx in [0, 8]; the head's are ky, kx in [-7, 7]; m = ky * KX + kx.
//
// MFMA lane layout (one wave, 32 x 32 x 16): lane l holds A[l % 32][8 (l / 32)
// + 0..7] and B[8 (l / 32) + 0..7][l % 32]; accumulator r of lane l is
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]. Within a K step the eight values
// of a lane may stand for any eight indices of the contraction, provided the A
// and B lanes of the same half agree; the kernels use that freedom to read
// packed complex values and to spread LDS accesses over the banks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scw_internal.h"

namespace scw {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf_t;

struct cf {
  float x, y;
};

constexpr int N = 32, C = 32;          // image side, channels
constexpr int LKY = 17, LKX = 9;       // a layer's modes
constexpr int LNM = LKY * LKX;         // 153
constexpr int HK = 15, HNM = HK * HK;  // the head's modes

// Rounding to bf16, nearest even: the hardware conversion (v_cvt_pk_bf16_f32
// on gfx950), two values per instruction; pk packs (lo, hi) into one word.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pk(float a, float b) {
  const bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ float lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi(unsigned w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ float rb(float x) { return (float)(__bf16)x; }

__device__ __forceinline__ floatx16 mma(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// GELU(z) = z (1 + erf(z / sqrt 2)) / 2 with erf from Abramowitz and Stegun
// 7.1.26 (absolute error at most 1.5e-7), the formula of the FP32 kernels
// rearranged for fewer operations: with x = |z| / sqrt 2, t = 1 / (1 + p x)
// and E = t P(t) exp(-x^2) / 2 (so erf x = 1 - 2 E), GELU(z) = max(z, 0) -
// |z| E for either sign of z. The halves and 1 / sqrt 2 are folded into the
// constants and exp(-x^2) = 2^(-z^2 log2(e) / 2): 11 vector operations and
// two transcendentals per value.
__device__ __forceinline__ float gelu(float z) {
  const float az = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.231641888f, az, 1.f));  // p / sqrt 2
  const float e = __builtin_amdgcn_exp2f(-(z * 0.72134752f) * z);       // log2(e) / 2
  float q = fmaf(0.5307027145f, t, -0.7265760135f);
  q = fmaf(q, t, 0.7107068705f);
  q = fmaf(q, t, -0.142248368f);
  q = fmaf(q, t, 0.127414796f);
  // max(z, 0) as an integer maximum of the bits: the float maximum would first
  // quiet a signalling NaN, one more operation
  const float zp = __int_as_float(max(__float_as_int(z), 0));
  return fmaf(-az, q * t * e, zp);
}

// ---------------------------------------------------------------------------
// Lift: h[b][o][p] = sum_c lw[c][o] x[b][c][p] + lb[o] (16 -> 32 channels),
// operands rounded, the sum in the order of the FP32 kernel, then stored
// rounded. One patch per block, 4 pixels per thread.
__global__ void __launch_bounds__(256) lift_bf16(const float* __restrict__ x,
                                                 const float* __restrict__ lw,
                                                 const float* __restrict__ lb,
                                                 bf_t* __restrict__ h) {
  constexpr int CI = 16;
  __shared__ float lws[CI * C], lbs[C];
  const int t = threadIdx.x, b = blockIdx.x;
  for (int i = t; i < CI * C; i += 256) lws[i] = rb(lw[i]);
  if (t < C) lbs[t] = lb[t];
  float xr[CI][4];
  const float* xb = x + (long long)b * CI * N * N;
#pragma unroll
  for (int c = 0; c < CI; ++c) {
    const float4 v = reinterpret_cast<const float4*>(xb + c * N * N)[t];
    xr[c][0] = rb(v.x);
    xr[c][1] = rb(v.y);
    xr[c][2] = rb(v.z);
    xr[c][3] = rb(v.w);
  }
  __syncthreads();
  bf_t* hb = h + (long long)b * C * N * N + 4 * t;
#pragma unroll 4
  for (int o = 0; o < C; ++o) {
    float a[4] = {lbs[o], lbs[o], lbs[o], lbs[o]};
#pragma unroll
    for (int c = 0; c < CI; ++c) {
      const float w = lws[c * C + o];
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = fmaf(w, xr[c][j], a[j]);
    }
    *reinterpret_cast<uint2*>(hb + o * N * N) = make_uint2(pk(a[0], a[1]), pk(a[2], a[3]));
  }
}

// ---------------------------------------------------------------------------
// Truncated forward DFT, 4 waves per block, the block's patches taken in turn
// (patch blockIdx.x, then every gridDim.x-th):
//   H[ky][kx][c] = sum_y fy[ky][y] sum_x h[c][y][x] fx[x][kx]
// Row transform, per channel: D[y][n] = sum_x h[c][y][x] T[x][n] with the
// twiddle columns n < KX the real parts of fx[.][n], KX <= n < 2 KX the
// imaginary parts (the input is real). A lane's K values are the 16
// consecutive pixels x = 16 (l / 32) .. + 15 of its row, read straight from
// memory; once a channel's registers are used they are refilled with the same
// rows of the next patch, so its loads are in flight during the rest of this
// one. The rounded results go to LDS as planes [n][c][y], the four 16-byte
// chunks of y of channel c placed at chunk ^ ((c / 2) % 4), so that 8 lanes
// reading one chunk each of 8 channels hit distinct banks.
// Column transform, per kx: D[ky][c] over K = 64 = (part, y): the real output
// takes (Re fy, -Im fy) against (Re, Im) of the row-transformed values, the
// imaginary output (Im fy, Re fy). Rows ky >= KY of the twiddle operand are
// zero. Output: packed complex, mode-major out[m][b][c]: 32 channels of one
// (mode, patch), one 128-byte line per half-wave.
constexpr int FW_PS = C * N + 8;  // bf16 per plane: 32 channels x 32 y + pad
__device__ __forceinline__ int fw_at(int c, int chunk) {
  return c * N + 8 * (chunk ^ ((c >> 1) & 3));
}
template <int KY, int KX>
__global__ void __launch_bounds__(256) fwd_bf16(const bf_t* __restrict__ h,
                                                const cf* __restrict__ fy,
                                                const cf* __restrict__ fx,
                                                unsigned* __restrict__ out, int B) {
  static_assert(2 * KX <= 32 && KY <= 32, "mode band exceeds one tile");
  __shared__ __attribute__((aligned(16))) bf_t hxl[2 * KX * FW_PS];
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63,
            li = l & 31, hh = l >> 5;
  int b = blockIdx.x;
  if (b >= B) return;  // uniform over the block, before any barrier
  // this wave's 8 channels: 32 rows of 32 pixels each, 2 x 16 bytes per lane
  const long long row_off = (long long)8 * w * N * N + li * N + 16 * hh;
  auto rows = [&](int bb, int c) {
    return reinterpret_cast<const u32x4*>(h + (long long)bb * C * N * N + row_off + c * N * N);
  };
  u32x4 a[8][2];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    a[c][0] = rows(b, c)[0];
    a[c][1] = rows(b, c)[1];
  }
  // row-transform twiddles: lane (n = li, hh), K step s, slot j: x = 16 hh + 8 s + j.
  // The table reads are unconditional (clamped index, the unwanted parts
  // multiplied by zero): a load under a lane condition becomes a branch that
  // waits for every load in flight, the first patch's rows included.
  const int tcol = li < KX ? li : (li < 2 * KX ? li - KX : 0);
  const int trow = li < KY ? li : 0;
  const float sx = li < KX ? 1.f : 0.f, sy = (li >= KX && li < 2 * KX) ? 1.f : 0.f;
  const float sr = li < KY ? 1.f : 0.f;
  u32x4 tb[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    unsigned v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float e[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int xx = 16 * hh + 8 * s + 2 * q + u;
        const cf f = fx[xx * KX + tcol];
        e[u] = fmaf(sx, f.x, sy * f.y);
      }
      v[q] = pk(e[0], e[1]);
    }
    tb[s] = u32x4{v[0], v[1], v[2], v[3]};
  }
  // column-transform twiddles: lane (ky = li, hh), K step s: part s / 2,
  // y = 16 (s % 2) + 8 hh + j
  u32x4 are[4], aim[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    unsigned vr[4], vi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float er[2], ei[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int yy = 16 * (s & 1) + 8 * hh + 2 * q + u;
        const cf f0 = fy[trow * N + yy];
        const cf f = {f0.x * sr, f0.y * sr};
        er[u] = s < 2 ? f.x : -f.y;
        ei[u] = s < 2 ? f.y : f.x;
      }
      vr[q] = pk(er[0], er[1]);
      vi[q] = pk(ei[0], ei[1]);
    }
    are[s] = u32x4{vr[0], vr[1], vr[2], vr[3]};
    aim[s] = u32x4{vi[0], vi[1], vi[2], vi[3]};
  }
  for (;;) {
    const int bn = b + gridDim.x;
    // every pass issues the next patch's loads (the last one, loads of the
    // first line of each of its own channel planes by every lane, with no
    // use), so that the count of loads in flight is the same on every path
    // and the waits before each channel's products stay exact
    const bool more = bn < B;
    const bf_t* nb = h + (long long)(more ? bn : b) * C * N * N + (more ? row_off : 8 * w * N * N);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      floatx16 d = {0};
      d = mma(a[c][0], tb[0], d);
      d = mma(a[c][1], tb[1], d);
      a[c][0] = reinterpret_cast<const u32x4*>(nb + c * N * N)[0];
      a[c][1] = reinterpret_cast<const u32x4*>(nb + c * N * N)[1];
      if (li < 2 * KX) {
        bf_t* dst = hxl + li * FW_PS + 4 * hh;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<uint2*>(dst + fw_at(8 * w + c, q)) =
              make_uint2(pk(d[4 * q], d[4 * q + 1]), pk(d[4 * q + 2], d[4 * q + 3]));
      }
    }
    __syncthreads();
    // column transform of kx; `mine` is the lane's share of the stores
    auto column = [&](int kx, bool mine) {
      floatx16 dr = {0}, di = {0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int plane = kx + (s >> 1) * KX;
        const u32x4 bv = *reinterpret_cast<const u32x4*>(hxl + plane * FW_PS +
                                                         fw_at(li, 2 * (s & 1) + hh));
        dr = mma(are[s], bv, dr);
        di = mma(aim[s], bv, di);
      }
      // the index as a part uniform over the wave (patch, ky block, kx) and
      // one 32-bit lane offset (channel, ky half), so that the stores share
      // one address register (the spectra hold fewer than 2^31 words)
      unsigned* ob = out + (long long)b * C;
      const unsigned bc = (unsigned)B * C;
      const unsigned lane_off = (unsigned)li + (unsigned)(4 * hh * KX) * bc;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ky = 8 * (r / 4) + 4 * hh + (r % 4);
        const unsigned uni = (unsigned)((8 * (r / 4) + (r % 4)) * KX + kx) * bc;
        if (ky < KY && mine) ob[uni + lane_off] = pk(dr[r], di[r]);
      }
    };
    // every wave issues the same stores on every path (the waits before the
    // next patch's products then count them exactly): wave w takes kx = w +
    // 4 i, and the KX % 4 last kx are transformed by all four waves, each
    // storing channels 8 w .. 8 w + 7
    // (loops kept rolled: unrolled, the columns' operands and accumulators
    // overlap and cost a wave per SIMD)
    constexpr int KS = KX / 4, KR = KX % 4;
#pragma unroll 1
    for (int i = 0; i < KS; ++i) column(w + 4 * i, true);
#pragma unroll 1
    for (int k = 0; k < KR; ++k) column(4 * KS + k, (li >> 3) == w);
    if (bn >= B) break;
    __syncthreads();  // the planes are read before the next patch overwrites them
    b = bn;
  }
}

// ---------------------------------------------------------------------------
// Mixing weights as B operands: Wb[k][m][part][s][hh][o] holds 8 bf16 for the
// lane (o, hh) of K step s: for j = 0..7, channel i = 8 s + 4 hh + j / 2 and
// (j even) Re W, -Im W for the real output (part 0), Im W, Re W for the
// imaginary output (part 1), W = W_k[i][o][m].
__global__ void mix_weights_bf16(const cf* __restrict__ W, long long layer_stride, int nmode,
                                 u32x4* __restrict__ Wb) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)nmode * 2 * 4 * 2 * C;
  if (q >= per) return;
  const int k = blockIdx.y;
  const int o = (int)(q % C), hh = (int)((q / C) % 2), s = (int)((q / (2 * C)) % 4);
  const int part = (int)((q / (8 * C)) % 2), m = (int)(q / (16 * C));
  unsigned v[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int i = 8 * s + 4 * hh + p;
    const cf wv = W[k * layer_stride + ((long long)i * C + o) * nmode + m];
    v[p] = part == 0 ? pk(wv.x, -wv.y) : pk(wv.y, wv.x);
  }
  Wb[(long long)k * per + q] = u32x4{v[0], v[1], v[2], v[3]};
}

// Per-mode mixing: G[b][m][o] = sum_i H[m][b][i] W[m][i][o] (complex, 32 x
// 32) as D[b][o] over K = 64: a lane's 8 values are 4 consecutive channels as
// (Re, Im) pairs, read as one 16-byte word of the packed spectra. One wave per
// mode keeps its 8 weight words and walks MIX_TT tiles of 32 patches.
constexpr int MIX_TT = 4;
__global__ void __launch_bounds__(256) mix_bf16(const unsigned* __restrict__ H,
                                                const u32x4* __restrict__ Wb, int nmode, int B,
                                                unsigned* __restrict__ G) {
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63,
            li = l & 31, hh = l >> 5;
  const int m = blockIdx.x * 4 + w;
  if (m >= nmode) return;  // no barrier in this kernel
  const u32x4* wm = Wb + (long long)m * 16 * C + hh * C + li;
  u32x4 wr[4], wi[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    wr[s] = wm[s * 2 * C];
    wi[s] = wm[8 * C + s * 2 * C];
  }
  const int b_first = blockIdx.y * MIX_TT * 32;
  for (int tt = 0; tt < MIX_TT; ++tt) {
    const int b0 = b_first + 32 * tt;
    if (b0 >= B) break;
    u32x4 av[4];
    const int ba = b0 + li;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      av[s] = ba < B ? *reinterpret_cast<const u32x4*>(H + ((long long)m * B + ba) * C + 8 * s +
                                                       4 * hh)
                     : u32x4{0u, 0u, 0u, 0u};
    floatx16 dr = {0}, di = {0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      dr = mma(av[s], wr[s], dr);
      di = mma(av[s], wi[s], di);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int bb = b0 + 8 * (r / 4) + 4 * hh + (r % 4);
      if (bb < B) G[((long long)bb * nmode + m) * C + li] = pk(dr[r], di[r]);
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse half of a Fourier layer, 4 waves per block, the block's patches
// taken in turn:
//   gy[o][y][kx] = sum_ky iy[y][ky] G[ky][kx][o]                  (column)
//   z[o][y][x]   = sum_i pw[i][o] h[i][y][x]
//                + sum_kx (Re gy Re ix[kx][x] - Im gy Im ix[kx][x]) + pb[o]
//   h'[o][y][x]  = GELU(z) (or z after the last layer: GELU false), stored rounded.
// Column transform on the matrix cores, per kx: D[y][o] over the 17 (up to
// 24) complex ky as (Re, Im) pairs: (Re iy, -Im iy) for the real part, (Im iy,
// Re iy) for the imaginary part, against G staged in LDS as rows [kx][ky] of
// 32 channels (40 words apart, so that the two halves of a wave, 4 rows apart,
// read distinct banks); the K slots of ky >= 17 take zeros from registers.
// Wave w transforms kx = w, w + 4 (and 8 for wave 0) for all 32 rows y; the
// packed results replace the staged G in LDS as gy[y][o][kx] (kx < 8, the two
// 16-byte halves of a record swapped for o / 8 odd so that 16 lanes reading
// one half each hit distinct banks) and gy8[y][o] (kx = 8).
// Output tile per row y: D[x][o] over K = 64: the pointwise part (K step s,
// slot j of half hh: channel 16 s + 2 j + hh, so that the two halves read
// neighbouring channel rows of the staged pixels, 64 bytes apart, on distinct
// LDS banks), the row transform (slots 2 kx, 2 kx + 1 = Re, Im; kx < 9, read
// from gy as one 16-byte word per half plus gy8) and the bias (slots 18 .. 20:
// its three bf16 terms against ones).
// Rows go in adjacent pairs (8 w + 2 jj, + 1): a channel's two rows are one
// 128-byte line of h and of h', loaded and stored whole in one iteration.
// Each wave stages its own pixel rows, so only wave-level ordering is needed
// there. Pixels are fetched one row pair ahead (the last pair fetches the
// next patch's first) and the next patch's G during the rows. Every load and
// store of h and h' moves whole 128-byte lines, eight lanes to a line: the
// pixels are regrouped for the products, and the outputs for the stores,
// through the wave's stage.
constexpr int IV_GR = 40;                   // words per staged G row: 32 channels + pad
constexpr int IV_GY8 = C * N * 8;           // offset of gy8 in the shared words
constexpr int IV_WORDS = C * N * 8 + C * N; // gy and gy8 (9216 words, 36 KB)
constexpr int IV_GQ = (LNM * C / 4 + 255) / 256;  // 16-byte chunks of G per thread
static_assert(LKX * LKY * IV_GR <= IV_WORDS, "staged G exceeds the shared words");
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
template <bool GELU>
__global__ void __launch_bounds__(256) inv_bf16(const unsigned* __restrict__ G,
                                                const bf_t* __restrict__ h,
                                                const cf* __restrict__ iy,
                                                const cf* __restrict__ ix,
                                                const float* __restrict__ pw,
                                                const float* __restrict__ pb,
                                                bf_t* __restrict__ h_out, int B) {
  // staged G, then (after every wave has read it) gy and gy8
  __shared__ __attribute__((aligned(16))) unsigned gsh[IV_WORDS];
  // per wave: a row pair as [i][row][x] (the 32 lines, in order), then the
  // outputs as [o][row][x] with the 16-byte chunks of line o at c ^ (o % 8)
  __shared__ __attribute__((aligned(16))) bf_t hst[4][2 * C * N];
  __shared__ u32x4 twl[2][3][64];  // column twiddles (Re, Im outputs) per K step and lane
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63,
            li = l & 31, hh = l >> 5;
  int b = blockIdx.x;
  if (b >= B) return;  // uniform over the block, before any barrier
  // a row pair of all channels is 32 lines of 128 bytes (channel i: rows y,
  // y + 1); load u takes lines 8 u .. 8 u + 7, eight lanes to a line (chunk
  // l % 8), so that every load reads whole lines
  const int lane_px = (l >> 3) * N * N + (l & 7) * 8 + 8 * w * N;
  auto load_rows = [&](int bb, int j, u32x4* pf) {
    const bf_t* hb = h + (long long)bb * C * N * N + lane_px + 2 * j * N;
#pragma unroll
    for (int u = 0; u < 4; ++u) pf[u] = *reinterpret_cast<const u32x4*>(hb + 8 * u * N * N);
  };
  auto load_g = [&](int bb, u32x4* gp) {
    const u32x4* gb = reinterpret_cast<const u32x4*>(G + (long long)bb * LNM * C);
#pragma unroll
    for (int u = 0; u < IV_GQ; ++u) {
      const int q = t + 256 * u;
      if (q < LNM * C / 4) gp[u] = gb[q];
    }
  };
  // pixel rows are fetched one row pair ahead
  u32x4 gpf[IV_GQ], pf[1][4];
  load_g(b, gpf);
  load_rows(b, 0, pf[0]);
  // row-transform twiddles (A operand, lane (x = li, hh)): K step 0 holds kx
  // 4 hh .. 4 hh + 3, step 1 kx 8 in the lower half; (Re ix, -Im ix) words
  u32x4 ta0, ta1;
  {
    unsigned v[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const cf f = ix[(4 * hh + p) * N + li];
      v[p] = pk(f.x, -f.y);
    }
    ta0 = u32x4{v[0], v[1], v[2], v[3]};
    // slots 2 .. 4 of the lower half multiply the bias terms of g1 by one
    const cf f8 = ix[8 * N + li];
    ta1 = hh == 0 ? u32x4{pk(f8.x, -f8.y), pk(1.f, 1.f), pk(1.f, 0.f), 0u} : u32x4{0u, 0u, 0u, 0u};
  }
  // pointwise weights (B operand, lane (o = li, hh)): channel 16 s + 2 p + hh
  u32x4 pwb[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    unsigned v[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
      v[p] = pk(pw[(16 * s + 4 * p + hh) * C + li], pw[(16 * s + 4 * p + 2 + hh) * C + li]);
    pwb[s] = u32x4{v[0], v[1], v[2], v[3]};
  }
  // the bias of output channel o = li as three bf16 terms whose sum is exactly
  // the FP32 value (each takes the next 8 significant bits of the remainder),
  // added by the row-transform product through K slots 2 .. 4 of the lower half
  unsigned bw1, bw2;
  {
    const float b0 = pb[li], bh = rb(b0), bm = rb(b0 - bh), bl = rb(b0 - bh - bm);
    bw1 = hh == 0 ? pk(bh, bm) : 0u;
    bw2 = hh == 0 ? pk(bl, 0.f) : 0u;
  }
  // column-transform twiddles (A operand, lane (y = li, hh), K step s: ky = 8 s
  // + 4 hh + p), built once per block into LDS by wave 0 with unconditional
  // table reads; read only after the first barrier of the patch loop
  if (w == 0) {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      unsigned vr[4], vi[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int ky = 8 * s + 4 * hh + p;
        const cf f0 = iy[li * LKY + min(ky, LKY - 1)];
        const float m = ky < LKY ? 1.f : 0.f;  // unconditional read, zero past the band
        const cf f = {f0.x * m, f0.y * m};
        vr[p] = pk(f.x, -f.y);
        vi[p] = pk(f.y, f.x);
      }
      twl[0][s][l] = u32x4{vr[0], vr[1], vr[2], vr[3]};
      twl[1][s][l] = u32x4{vi[0], vi[1], vi[2], vi[3]};
    }
  }
  bf_t* hs = &hst[w][0];
  const bf_t* hs_lane = hs + hh * 2 * N + li;
  // this lane's gy word: record (y, o = li), half hh of the 8 kx < 8
  const int gy_lane = li * 8 + 4 * (hh ^ ((li >> 3) & 1));
  for (;;) {
    // stage G[m][o] -> rows [kx][ky] of 32 channels
#pragma unroll
    for (int u = 0; u < IV_GQ; ++u) {
      const int q = t + 256 * u;
      if (q < LNM * C / 4) {
        const int m = q >> 3, o0 = (q & 7) * 4, ky = m / LKX, kx = m % LKX;
        *reinterpret_cast<u32x4*>(gsh + (kx * LKY + ky) * IV_GR + o0) = gpf[u];
      }
    }
    __syncthreads();  // G staged (and, before the first patch, the twiddle table)
    // column-transform twiddles from the block's LDS table (not held in
    // registers through the rows)
    u32x4 are[3], aim[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      are[s] = twl[0][s][l];
      aim[s] = twl[1][s][l];
    }
    // column transform of kx = w + 4 n (n = 0, 1) and, in wave 0, of kx = 8;
    // packed rows y = 8 (r / 4) + 4 hh + r % 4 of channel o = li
    auto column = [&](int kx, unsigned* res) {
      const unsigned* gk = gsh + kx * LKY * IV_GR + li + 4 * hh * IV_GR;
      floatx16 dr = {0}, di = {0};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        u32x4 bv;
        if (s < 2) {
#pragma unroll
          for (int p = 0; p < 4; ++p) bv[p] = gk[(8 * s + p) * IV_GR];
        } else {  // ky 16 in slot 0 of the lower half; ky 17 .. 23 are zero
          const unsigned v16 = gk[(LKY - 1 - 4 * hh) * IV_GR];
          bv = u32x4{hh ? 0u : v16, 0u, 0u, 0u};
        }
        dr = mma(are[s], bv, dr);
        di = mma(aim[s], bv, di);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) res[r] = pk(dr[r], di[r]);
    };
    // one column at a time: overlapping them would hold three accumulator pairs
    unsigned res0[16], res1[16], res8[16];
    column(w, res0);
    __builtin_amdgcn_sched_barrier(0);
    column(w + 4, res1);
    __builtin_amdgcn_sched_barrier(0);
    if (w == 0) column(8, res8);
    __syncthreads();  // every wave is done with the staged G
    {
      // row y = 8 (r / 4) + 4 hh + r % 4: lane base at row 4 hh
      const int sw = (li >> 3) & 1;
      unsigned* gq0 = gsh + (4 * hh * C + li) * 8 + w + 4 * sw;
      unsigned* gq1 = gsh + (4 * hh * C + li) * 8 + w + 4 * (sw ^ 1);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int y0 = 8 * (r / 4) + (r % 4);
        gq0[y0 * C * 8] = res0[r];
        gq1[y0 * C * 8] = res1[r];
      }
      if (w == 0) {
        unsigned* g8 = gsh + IV_GY8 + 4 * hh * C + li;
#pragma unroll
        for (int r = 0; r < 16; ++r) g8[(8 * (r / 4) + (r % 4)) * C] = res8[r];
      }
    }
    __syncthreads();  // gy complete
    const int bn = b + gridDim.x;
    if (bn < B) load_g(bn, gpf);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      // stage the pixels of rows 8 w + 2 jj and 8 w + 2 jj + 1 (each channel's
      // two rows are one 128-byte line, loaded and stored whole)
      // load u, lane l holds chunk l % 8 of line 8 u + l / 8: [i][row][x]
#pragma unroll
      for (int u = 0; u < 4; ++u)
        *reinterpret_cast<u32x4*>(hs + (64 * u + l) * 8) = pf[0][u];
      wave_sync();
      if (jj + 1 < 4) load_rows(b, jj + 1, pf[0]);
      else if (bn < B) load_rows(bn, 0, pf[0]);
      unsigned zw[2][8];  // packed outputs of both rows: x = 8 q + 4 hh + 2 e2, + 1
#pragma unroll
      for (int row = 0; row < 2; ++row) {
        const int y = 8 * w + 2 * jj + row;
        // pointwise A operand: pixels x = li of channels 16 s + 4 p + hh (+ 2)
        const bf_t* src = hs_lane + row * N;
        u32x4 pa[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          unsigned v[4];
#pragma unroll
          for (int p = 0; p < 4; ++p)
            v[p] = (unsigned)src[(16 * s + 4 * p) * 2 * N] |
                   ((unsigned)src[(16 * s + 4 * p + 2) * 2 * N] << 16);
          pa[s] = u32x4{v[0], v[1], v[2], v[3]};
        }
        const u32x4 g0 = *reinterpret_cast<const u32x4*>(gsh + y * C * 8 + gy_lane);
        const unsigned g8 = gsh[IV_GY8 + y * C + li];
        const u32x4 g1 = u32x4{hh ? 0u : g8, bw1, bw2, 0u};
        floatx16 d = {0};
        d = mma(pa[0], pwb[0], d);
        d = mma(pa[1], pwb[1], d);
        d = mma(ta0, g0, d);
        d = mma(ta1, g1, d);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float z[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            z[e] = GELU ? gelu(d[4 * q + e]) : d[4 * q + e];
          }
          zw[row][2 * q] = pk(z[0], z[1]);
          zw[row][2 * q + 1] = pk(z[2], z[3]);
        }
      }
      // outputs through the wave's stage: lane (o, hh) holds, per row, pixels
      // 8 q + 4 hh .. + 3 (8 bytes) of channel o; as [o][row][x] they form the
      // 32 output lines, whose 16-byte chunk c sits at c ^ (o % 8) to spread
      // the writes over the banks. The pixels are all read by now (the
      // products that used them are done), so the stage is free.
#pragma unroll
      for (int row = 0; row < 2; ++row)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          *reinterpret_cast<uint2*>(hs + li * 2 * N + (((4 * row + q) ^ (li & 7)) * 8) + 4 * hh) =
              make_uint2(zw[row][2 * q], zw[row][2 * q + 1]);
      wave_sync();
      // store u: lines 8 u .. 8 u + 7, eight lanes to a line, whole lines
      {
        bf_t* orow = h_out + (long long)b * C * N * N + (8 * w + 2 * jj) * N + (l & 7) * 8;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int o = 8 * u + (l >> 3);
          const u32x4 v =
              *reinterpret_cast<const u32x4*>(hs + o * 2 * N + (((l & 7) ^ (o & 7)) * 8));
          *reinterpret_cast<u32x4*>(orow + (long long)o * N * N) = v;
        }
      }
      wave_sync();  // this row pair's pixels are read before the next are staged
    }
    if (bn >= B) break;
    __syncthreads();  // every wave is done with gy before the next G is staged
    b = bn;
  }
}

// ---------------------------------------------------------------------------
// The head's mixing: out[b][o][m] = sum_i F[m][b][i] W[i][o][m] for the 3
// outputs, on the matrix cores. Per mode, D[b][n] over K = 64 = (channel,
// part) for 32 patches: a lane's 8 K values are 4 consecutive channels as
// (Re, Im), one 16-byte chunk of the patch's packed record; column n = 2 o
// takes (Re W, -Im W) for the real part of output o, n = 2 o + 1 takes
// (Im W, Re W) for its imaginary part, and columns n >= 6 are zero. The
// weights are staged in LDS as packed bf16 words (12 KB with the 25 KB output
// stage: four blocks per CU, so that a batch of 4096 is one round of blocks),
// and each mode's operand is built from them. Block: 32 modes x 32 patches, wave w takes modes 8 w .. 8 w + 7
// with the next mode's records loaded during the current one. The outputs
// are gathered in LDS and written as runs of 32 modes.
constexpr int HM_B = 32;
__global__ void __launch_bounds__(256) head_mix_bf16(const unsigned* __restrict__ F,
                                                     const cf* __restrict__ Wt, int B,
                                                     cf* __restrict__ out) {
  // weights as packed bf16 (Re, Im) words: 12 KB, so that 4 blocks fit a CU
  __shared__ unsigned wl[32][C * 3 + 1];   // [mode][i * 3 + o], rows 97 apart
  __shared__ cf ol[HM_B][3][33];           // [patch][o][mode]
  const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), l = t & 63,
            li = l & 31, hh = l >> 5;
  const int m0 = blockIdx.x * 32, b0 = blockIdx.y * HM_B, bb = b0 + li;
  for (int q = t; q < 32 * C * 3; q += 256) {
    const int mm = q & 31, io = q >> 5;  // io = i * 3 + o
    const cf v = m0 + mm < HNM ? Wt[(long long)io * HNM + m0 + mm] : cf{0.f, 0.f};
    wl[mm][io] = pk(v.x, v.y);
  }
  // A operand of K step s: chunk 2 s + hh of record (m, bb), channels 8 s + 4 hh .. + 3.
  // The loads are unconditional, the record clamped to the last mode and
  // patch: the products of records past the end are computed and not
  // written, so every path issues the same loads and the waits stay exact.
  const int bc = min(bb, B - 1);
  auto load = [&](int mm, u32x4* a) {
    const int m = min(m0 + mm, HNM - 1);
    const u32x4* p = reinterpret_cast<const u32x4*>(F + ((long long)m * B + bc) * C) + hh;
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = p[2 * s];
  };
  u32x4 cur[4], nxt[4];
  load(8 * w, cur);
  __syncthreads();  // weights staged
  const bool nlive = li < 6;
  const int on = nlive ? li >> 1 : 0, part = li & 1;
  // One formula for every lane, so that the weight words are not read under
  // a lane condition (a branch and a wait per word): (Im, Re) is the word
  // rotated by 16 bits, (Re, -Im) the word with its upper sign bit flipped,
  // and lanes past column 5 mask it to zero.
  const unsigned rot = part ? 16u : 0u, flip = part ? 0u : 0x80000000u;
  const unsigned live_mask = nlive ? 0xffffffffu : 0u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int mm = 8 * w + k;
    if (k < 7) load(mm + 1, nxt);
    const unsigned* wm = wl[mm];
    floatx16 d = {0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      unsigned v[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const unsigned c = wm[(8 * s + 4 * hh + p) * 3 + on];
        v[p] = (__builtin_amdgcn_alignbit(c, c, rot) ^ flip) & live_mask;
      }
      d = mma(cur[s], u32x4{v[0], v[1], v[2], v[3]}, d);
    }
    // lane (n, hh) holds patches 8 (r / 4) + 4 hh + r % 4 of column n, the
    // real part of output n in even lanes and the imaginary part in odd ones
    if (nlive) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        reinterpret_cast<float*>(&ol[8 * (r / 4) + 4 * hh + (r % 4)][on][mm])[part] = d[r];
    }
    if (k < 7)
#pragma unroll
      for (int s = 0; s < 4; ++s) cur[s] = nxt[s];
  }
  __syncthreads();
  // write: 3 x 32 patches rows of 32 modes
  for (int q = t; q < HM_B * 3 * 32; q += 256) {
    const int mm = q & 31, o = (q >> 5) % 3, pb_ = q / 96;
    if (b0 + pb_ < B && m0 + mm < HNM)
      out[((long long)(b0 + pb_) * 3 + o) * HNM + m0 + mm] = ol[pb_][o][mm];
  }
}

// Blocks that are resident at once for a kernel of 256 threads (the grid of
// the kernels that take their patches in turn); at least 1.
template <typename K>
int resident_blocks(K kern) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 256, 0) != hipSuccess)
    return 256;
  return std::max(1, cus * per);
}

}  // namespace

hipError_t sur_lift_bf16(const float* x, const float* lw, const float* lb, void* h, int B,
                         hipStream_t s) {
  lift_bf16<<<B, 256, 0, s>>>(x, lw, lb, reinterpret_cast<bf_t*>(h));
  return hipGetLastError();
}
hipError_t sur_fwd_bf16(const void* h, const float* fy, const float* fx, void* H, int B,
                        bool head, hipStream_t s) {
  const bf_t* hp = reinterpret_cast<const bf_t*>(h);
  const cf* y = reinterpret_cast<const cf*>(fy);
  const cf* x = reinterpret_cast<const cf*>(fx);
  unsigned* o = reinterpret_cast<unsigned*>(H);
  auto go = [&](auto kern) {
    static const int slots = resident_blocks(kern);
    kern<<<std::min(B, slots), 256, 0, s>>>(hp, y, x, o, B);
  };
  if (head) go(fwd_bf16<HK, HK>);
  else go(fwd_bf16<LKY, LKX>);
  return hipGetLastError();
}
hipError_t sur_mix_weights_bf16(const float* W, long long layer_stride_floats, int layers,
                                void* Wb, hipStream_t s) {
  if (layer_stride_floats % 2 != 0) return hipErrorInvalidValue;
  const long long per = (long long)LNM * 2 * 4 * 2 * C;
  dim3 grid((unsigned)((per + 255) / 256), layers);
  mix_weights_bf16<<<grid, 256, 0, s>>>(reinterpret_cast<const cf*>(W), layer_stride_floats / 2,
                                        LNM, reinterpret_cast<u32x4*>(Wb));
  return hipGetLastError();
}
size_t sur_mix_weights_bf16_bytes(int layers) { return (size_t)layers * LNM * 16 * C * 16; }
hipError_t sur_mix_bf16(const void* H, const void* Wb_layer, int B, void* G, hipStream_t s) {
  dim3 grid((LNM + 3) / 4, (B + MIX_TT * 32 - 1) / (MIX_TT * 32));
  mix_bf16<<<grid, 256, 0, s>>>(reinterpret_cast<const unsigned*>(H),
                                reinterpret_cast<const u32x4*>(Wb_layer), LNM, B,
                                reinterpret_cast<unsigned*>(G));
  return hipGetLastError();
}
hipError_t sur_inv_bf16(const void* G, const void* h, const float* iy, const float* ix,
                        const float* pw, const float* pb, void* h_out, bool gelu_on, int B,
                        hipStream_t s) {
  auto go = [&](auto kern) {
    static const int slots = resident_blocks(kern);
    kern<<<std::min(B, slots), 256, 0, s>>>(
        reinterpret_cast<const unsigned*>(G), reinterpret_cast<const bf_t*>(h),
        reinterpret_cast<const cf*>(iy), reinterpret_cast<const cf*>(ix), pw, pb,
        reinterpret_cast<bf_t*>(h_out), B);
  };
  if (gelu_on) go(inv_bf16<true>);
  else go(inv_bf16<false>);
  return hipGetLastError();
}
hipError_t sur_head_mix_bf16(const void* F, const float* W, int B, float* out, hipStream_t s) {
  dim3 grid((HNM + 31) / 32, (B + HM_B - 1) / HM_B);
  head_mix_bf16<<<grid, 256, 0, s>>>(reinterpret_cast<const unsigned*>(F),
                                     reinterpret_cast<const cf*>(W), B,
                                     reinterpret_cast<cf*>(out));
  return hipGetLastError();
}

}  // namespace scw

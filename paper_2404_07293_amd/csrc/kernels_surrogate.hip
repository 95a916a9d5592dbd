// Kernels of the spectral-convolution surrogate: one strided, batched GEMM
// for every linear step (pointwise channel maps, truncated DFTs, per-mode
// complex mixing, and their transposes in the backward pass), elementwise
// bias / GELU / loss kernels, and the Adam update.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "scw_internal.h"

namespace scw {
namespace {

struct f2 {
  float x, y;
};

// C[b] = op(A[b]) . op(B[b]) (+ beta C[b]). Operands are real or complex
// (interleaved); strides are in elements of the operand's type. The result is
// complex, or its real part. Tile 32x32, 256 threads (2x2 outputs each),
// K staged through LDS in steps of 16.
constexpr int TM = 32, TN = 32, TK = 16;

__global__ void __launch_bounds__(256) gemm_kernel(GemmOp op) {
  __shared__ f2 As[TK][TM + 1];
  __shared__ f2 Bs[TK][TN + 1];
  const int b = blockIdx.y;
  const int ntn = (op.N + TN - 1) / TN;
  const int m0 = (blockIdx.x / ntn) * TM, n0 = (blockIdx.x % ntn) * TN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const float* A = op.A + (long long)b * op.a_bs * (op.a_cplx ? 2 : 1);
  const float* B = op.B + (long long)b * op.b_bs * (op.b_cplx ? 2 : 1);
  f2 acc[2][2] = {{{0.f, 0.f}, {0.f, 0.f}}, {{0.f, 0.f}, {0.f, 0.f}}};
  const float ca = op.conj_a ? -1.f : 1.f, cb = op.conj_b ? -1.f : 1.f;
  for (int k0 = 0; k0 < op.K; k0 += TK) {
    for (int i = threadIdx.x; i < TM * TK; i += 256) {
      const int r = i / TK, k = i % TK;
      const int gm = m0 + r, gk = k0 + k;
      f2 v = {0.f, 0.f};
      if (gm < op.M && gk < op.K) {
        const long long o = (long long)gm * op.a_rs + (long long)gk * op.a_cs;
        if (op.a_cplx) v = {A[2 * o], ca * A[2 * o + 1]};
        else v = {A[o], 0.f};
      }
      As[k][r] = v;
    }
    for (int i = threadIdx.x; i < TK * TN; i += 256) {
      const int k = i / TN, c = i % TN;
      const int gk = k0 + k, gn = n0 + c;
      f2 v = {0.f, 0.f};
      if (gk < op.K && gn < op.N) {
        const long long o = (long long)gk * op.b_rs + (long long)gn * op.b_cs;
        if (op.b_cplx) v = {B[2 * o], cb * B[2 * o + 1]};
        else v = {B[o], 0.f};
      }
      Bs[k][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TK; ++k) {
      const f2 a0 = As[k][ty], a1 = As[k][ty + 16];
      const f2 b0 = Bs[k][tx], b1 = Bs[k][tx + 16];
#define CMA(acc, a, bb)                                \
  acc.x = fmaf(a.x, bb.x, fmaf(-a.y, bb.y, acc.x));     \
  acc.y = fmaf(a.x, bb.y, fmaf(a.y, bb.x, acc.y));
      CMA(acc[0][0], a0, b0) CMA(acc[0][1], a0, b1) CMA(acc[1][0], a1, b0) CMA(acc[1][1], a1, b1)
#undef CMA
    }
    __syncthreads();
  }
  float* C = op.C + (long long)b * op.c_bs * (op.c_cplx ? 2 : 1);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm >= op.M || gn >= op.N) continue;
      const long long o = (long long)gm * op.c_rs + (long long)gn * op.c_cs;
      if (op.c_cplx) {
        float re = acc[i][j].x, im = acc[i][j].y;
        if (op.beta != 0.f) {
          re += op.beta * C[2 * o];
          im += op.beta * C[2 * o + 1];
        }
        C[2 * o] = re;
        C[2 * o + 1] = im;
      } else {
        float re = acc[i][j].x;
        if (op.beta != 0.f) re += op.beta * C[o];
        C[o] = re;
      }
    }
}

// The same product on the matrix cores with BF16 operands and FP32
// accumulation: every operand element is rounded to bf16 (nearest even) as it
// is staged in LDS. Block tile 64 x 64, four waves of 32 x 32, K steps of 16
// (v_mfma_f32_32x32x16_bf16). A complex product takes four MFMAs per step:
//   Re C += Re A Re B + (-Im A) Im B,   Im C += Re A Im B + Im A Re B,
// with conjugation applied to the imaginary parts as they are staged.
// MFMA lane layout (one wave, 32 x 32 x 16): lane l holds A[l % 32][8 (l / 32)
// + 0..7] and B[8 (l / 32) + 0..7][l % 32]; accumulator r of lane l is
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, LROW = 24;  // LDS row: 16 k + 8 pad (bf16)

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmOp op) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * LROW];  // [re|im][row][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * LROW];  // [re|im][col][k]
  const int b = blockIdx.y;
  const int ntn = (op.N + BN - 1) / BN;
  const int m0 = (blockIdx.x / ntn) * BM, n0 = (blockIdx.x % ntn) * BN;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const float* A = op.A + (long long)b * op.a_bs * (op.a_cplx ? 2 : 1);
  const float* B = op.B + (long long)b * op.b_bs * (op.b_cplx ? 2 : 1);
  const float ca = op.conj_a ? -1.f : 1.f, cb = op.conj_b ? -1.f : 1.f;
  floatx16 cre = {0}, cim = {0};
  const int li = lane & 31, lk = 8 * (lane >> 5);
  for (int k0 = 0; k0 < op.K; k0 += BK) {
    // stage: 64 x 16 of A and 16 x 64 of B, four elements per thread each
    // consecutive threads walk the operand's contiguous index where it has one
    const bool a_kfast = op.a_cs == 1, b_kfast = op.b_rs == 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = t + 256 * e;
      const int r = a_kfast ? i / BK : i % BM, k = a_kfast ? i % BK : i / BM;
      const int gm = m0 + r, gk = k0 + k;
      float re = 0.f, im = 0.f;
      if (gm < op.M && gk < op.K) {
        const long long o = (long long)gm * op.a_rs + (long long)gk * op.a_cs;
        if (op.a_cplx) {
          re = A[2 * o];
          im = ca * A[2 * o + 1];
        } else {
          re = A[o];
        }
      }
      As[0][r * LROW + k] = (__bf16)re;
      As[1][r * LROW + k] = (__bf16)im;
      const int c = b_kfast ? i / BK : i % BN, kb = b_kfast ? i % BK : i / BN;
      const int gn = n0 + c, gkb = k0 + kb;
      float bre = 0.f, bim = 0.f;
      if (gn < op.N && gkb < op.K) {
        const long long o = (long long)gkb * op.b_rs + (long long)gn * op.b_cs;
        if (op.b_cplx) {
          bre = B[2 * o];
          bim = cb * B[2 * o + 1];
        } else {
          bre = B[o];
        }
      }
      Bs[0][c * LROW + kb] = (__bf16)bre;
      Bs[1][c * LROW + kb] = (__bf16)bim;
    }
    __syncthreads();
    const u32x4 ar = *reinterpret_cast<const u32x4*>(&As[0][(wm + li) * LROW + lk]);
    const u32x4 br = *reinterpret_cast<const u32x4*>(&Bs[0][(wn + li) * LROW + lk]);
    cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ar),
                                                  __builtin_bit_cast(bf16x8, br), cre, 0, 0, 0);
    if (op.b_cplx) {
      const u32x4 bi = *reinterpret_cast<const u32x4*>(&Bs[1][(wn + li) * LROW + lk]);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ar),
                                                    __builtin_bit_cast(bf16x8, bi), cim, 0, 0, 0);
      if (op.a_cplx) {
        const u32x4 ai = *reinterpret_cast<const u32x4*>(&As[1][(wm + li) * LROW + lk]);
        const u32x4 nai = ai ^ 0x80008000u;  // -Im A: flip every bf16 sign
        cre = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, nai),
                                                      __builtin_bit_cast(bf16x8, bi), cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ai),
                                                      __builtin_bit_cast(bf16x8, br), cim, 0, 0, 0);
      }
    } else if (op.a_cplx) {
      const u32x4 ai = *reinterpret_cast<const u32x4*>(&As[1][(wm + li) * LROW + lk]);
      cim = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ai),
                                                    __builtin_bit_cast(bf16x8, br), cim, 0, 0, 0);
    }
    __syncthreads();
  }
  float* C = op.C + (long long)b * op.c_bs * (op.c_cplx ? 2 : 1);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gm = m0 + wm + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
    const int gn = n0 + wn + li;
    if (gm >= op.M || gn >= op.N) continue;
    const long long o = (long long)gm * op.c_rs + (long long)gn * op.c_cs;
    if (op.c_cplx) {
      float re = cre[r], im = cim[r];
      if (op.beta != 0.f) {
        re += op.beta * C[2 * o];
        im += op.beta * C[2 * o + 1];
      }
      C[2 * o] = re;
      C[2 * o + 1] = im;
    } else {
      float re = cre[r];
      if (op.beta != 0.f) re += op.beta * C[o];
      C[o] = re;
    }
  }
}

// d GELU / dz for the backward pass (exact erf)
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void gelu_bwd(const float* z, float* g, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] *= gelu_grad_f(z[i]);
}

// out[c][k] = sum_b in[b][c][k] (reduction over the batch index)
__global__ void sum_batch(const float* in, float* out, int B, long long per) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += in[(long long)b * per + i];
  out[i] = s;
}

// bias gradient: out[c] = sum_{b,p} g[b][c][p]; one block per channel
__global__ void bias_grad(const float* g, float* out, int B, int C, int P) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (long long i = threadIdx.x; i < (long long)B * P; i += 256) {
    const long long b = i / P, p = i % P;
    s += g[(b * C + c) * P + p];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// sums[0] = sum |out - tgt|^2, sums[1] = sum |tgt|^2 (complex64 arrays of n)
__global__ void loss_sums(const float* out, const float* tgt, long long n, float* sums) {
  __shared__ float r0[256], r1[256];
  float a = 0.f, b = 0.f;
  for (long long i = threadIdx.x; i < n; i += 256) {
    const float dx = out[2 * i] - tgt[2 * i], dy = out[2 * i + 1] - tgt[2 * i + 1];
    a += dx * dx + dy * dy;
    b += tgt[2 * i] * tgt[2 * i] + tgt[2 * i + 1] * tgt[2 * i + 1];
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[0] = r0[0];
    sums[1] = r1[0];
  }
}

// g = 2 (out - tgt) / sum |tgt|^2
__global__ void loss_grad(const float* out, const float* tgt, const float* sums, float* g,
                          long long n2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) g[i] = 2.f * (out[i] - tgt[i]) / sums[1];
}

__global__ void adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                     float b1, float b2, float eps, float c1, float c2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- fused Fourier layer
// The two halves of one Fourier layer around its per-mode mixing (which stays
// a batched product over the patches, so that each mode's 32 x 32 weights are
// read once per tile of patches rather than once per patch):
//   forward  H[b][i][ky][kx] = sum_y fy[ky][y] sum_x h[b][i][y][x] fx[x][kx]
//   inverse  z[b][o][y][x] = Re sum_kx (sum_ky iy[y][ky] G[b][o][ky][kx]) ix[kx][x]
//                          + sum_i pw[i][o] h[b][i][y][x] + pb[o]
//            h'[b][o] = GELU(z[b][o]) (or z itself after the last layer)
// With BF16, both operands of every product are rounded to bf16 (nearest
// even) first, as the matrix-core products of the unfused path round them;
// sums stay FP32.
constexpr int SN = 32, SKY = 17, SKX = 9, SNM = SKY * SKX, SW = 32;

__device__ __forceinline__ float rbf(float x) {  // round to bf16, nearest even
  unsigned u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}
template <bool BF16>
__device__ __forceinline__ float op(float x) { return BF16 ? rbf(x) : x; }
template <bool BF16>
__device__ __forceinline__ f2 op(f2 x) { return BF16 ? f2{rbf(x.x), rbf(x.y)} : x; }

// Truncated forward DFT of 8 channels of one patch per block:
//   out[b][i][ky][kx] = sum_y fy[ky][y] sum_x h[b][i][y][x] fx[x][kx]
// (KY x KX modes; fy is [KY][32], fx is [32][KX], both complex). Grid (4, B),
// 256 threads. Thread (c, y) = (t / 32, t % 32) first transforms row y of
// channel c in registers; the column transform then runs over (c, mode).
// MM selects the mode-major output layout [mode][b][i] (a Fourier layer's
// spectra, read per mode by the mixing); otherwise [b][i][mode] (the head).
template <bool BF16, int KY, int KX, bool MM>
__global__ void __launch_bounds__(256) fused_dft_fwd(const float* __restrict__ h,
                                                     const f2* __restrict__ fy,
                                                     const f2* __restrict__ fx,
                                                     f2* __restrict__ H) {
  // Padded strides against LDS bank conflicts (16 lanes of 8 bytes per
  // cycle): a channel's rows start 2 (mod 16) complex values apart, so that 8
  // channels x 2 consecutive kx hit distinct banks; the ky rows of fy are 33
  // apart, so that a wave reading two ky groups hits two banks.
  constexpr int HXS = SN * KX + 2, FYS = SN + 1;
  __shared__ f2 hx[8 * HXS];
  __shared__ f2 fys[KY * FYS], fxs[SN * KX];
  const int t = threadIdx.x, b = blockIdx.y, c0 = blockIdx.x * 8;
  for (int i = t; i < KY * SN; i += 256) fys[(i / SN) * FYS + i % SN] = op<BF16>(fy[i]);
  if (BF16)
    for (int i = t; i < SN * KX; i += 256) fxs[i] = op<BF16>(fx[i]);
  const int c = t >> 5, y = t & 31;
  float row[SN];
  const float4* src =
      reinterpret_cast<const float4*>(h + (((long long)b * SW + c0 + c) * SN + y) * SN);
#pragma unroll
  for (int q = 0; q < SN / 4; ++q) {
    const float4 v = src[q];
    row[4 * q] = op<BF16>(v.x);
    row[4 * q + 1] = op<BF16>(v.y);
    row[4 * q + 2] = op<BF16>(v.z);
    row[4 * q + 3] = op<BF16>(v.w);
  }
  __syncthreads();
  if constexpr (BF16) {  // every product of two rounded operands, as defined
#pragma unroll 3
    for (int kx = 0; kx < KX; ++kx) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int x = 0; x < SN; ++x) {
        const f2 w = fxs[x * KX + kx];
        re = fmaf(row[x], w.x, re);
        im = fmaf(row[x], w.y, im);
      }
      hx[c * HXS + y * KX + kx] = op<BF16>(f2{re, im});
    }
  } else {
    // The twiddles of x and 32 - x are conjugate: with s = row[x] + row[32-x]
    // and d = row[x] - row[32-x], the pair adds s Re w to the real part and
    // d Im w to the imaginary part (x = 0 and 16 stand alone; a layer's table
    // holds kx = 0..8, the head's kx = -7..7 scaled by 1/32, both conjugate
    // symmetric). The index is wave-uniform, so the twiddles come through the
    // scalar cache.
    float sx[SN / 2], dx[SN / 2];
#pragma unroll
    for (int x = 1; x < SN / 2; ++x) {
      sx[x] = row[x] + row[SN - x];
      dx[x] = row[x] - row[SN - x];
    }
#pragma unroll 3
    for (int kx = 0; kx < KX; ++kx) {
      const f2 w0 = fx[kx], w16 = fx[(SN / 2) * KX + kx];
      float re = fmaf(row[0], w0.x, row[SN / 2] * w16.x);
      float im = fmaf(row[0], w0.y, row[SN / 2] * w16.y);
#pragma unroll
      for (int x = 1; x < SN / 2; ++x) {
        const f2 w = fx[x * KX + kx];
        re = fmaf(sx[x], w.x, re);
        im = fmaf(dx[x], w.y, im);
      }
      hx[c * HXS + y * KX + kx] = f2{re, im};
    }
  }
  __syncthreads();
  // column transform: items (ky group of KG, kx, channel), channel fastest;
  // each hx value read serves KG modes
  constexpr int NMODE = KY * KX;
  constexpr int KG = 3, NKG = (KY + KG - 1) / KG;
  for (int i = t; i < 8 * KX * NKG; i += 256) {
    const int cc = i % 8, kx = (i / 8) % KX, g = i / (8 * KX);
    float re[KG], im[KG];
#pragma unroll
    for (int j = 0; j < KG; ++j) re[j] = im[j] = 0.f;
    const f2* hc = hx + cc * HXS + kx;  // hc[yy * KX]
    if constexpr (BF16) {
#pragma unroll 4
      for (int yy = 0; yy < SN; ++yy) {
        const f2 v = hc[yy * KX];
#pragma unroll
        for (int j = 0; j < KG; ++j) {
          const f2 a = fys[min(g * KG + j, KY - 1) * FYS + yy];
          re[j] = fmaf(a.x, v.x, fmaf(-a.y, v.y, re[j]));
          im[j] = fmaf(a.x, v.y, fmaf(a.y, v.x, im[j]));
        }
      }
    } else {
      // rows yy and 32 - yy have conjugate twiddles: w a + conj(w) b =
      // Re w (a + b) + i Im w (a - b); rows 0 and 16 stand alone
#pragma unroll
      for (int yy = 0; yy <= SN / 2; yy += SN / 2) {
        const f2 v = hc[yy * KX];
#pragma unroll
        for (int j = 0; j < KG; ++j) {
          const f2 a = fys[min(g * KG + j, KY - 1) * FYS + yy];
          re[j] = fmaf(a.x, v.x, fmaf(-a.y, v.y, re[j]));
          im[j] = fmaf(a.x, v.y, fmaf(a.y, v.x, im[j]));
        }
      }
#pragma unroll 3
      for (int yy = 1; yy < SN / 2; ++yy) {
        const f2 va = hc[yy * KX], vb = hc[(SN - yy) * KX];
        const f2 p = f2{va.x + vb.x, va.y + vb.y}, q = f2{va.x - vb.x, va.y - vb.y};
#pragma unroll
        for (int j = 0; j < KG; ++j) {
          const f2 a = fys[min(g * KG + j, KY - 1) * FYS + yy];
          re[j] = fmaf(a.x, p.x, fmaf(-a.y, q.y, re[j]));
          im[j] = fmaf(a.x, p.y, fmaf(a.y, q.x, im[j]));
        }
      }
    }
#pragma unroll
    for (int j = 0; j < KG; ++j) {
      const int ky = g * KG + j;
      if (ky >= KY) break;
      const int m = ky * KX + kx;
      if (MM)
        H[((long long)m * gridDim.y + b) * SW + c0 + cc] = f2{re[j], im[j]};
      else
        H[((long long)b * SW + c0 + cc) * NMODE + m] = f2{re[j], im[j]};
    }
  }
}

// GELU(z) = z (1 + erf(z / sqrt 2)) / 2 for the forward pass, with erf from
// Abramowitz and Stegun 7.1.26 (Hastings' rational approximation, absolute
// error at most 1.5e-7): erf(x) = 1 - t (a1 + t (a2 + ... + t a5)) e^{-x^2},
// t = 1 / (1 + p x), x >= 0. Branch-free: one reciprocal and one exponential.
// For z < 0, 1 + erf(z / sqrt 2) is formed directly as the product, without
// the cancellation of 1 - (1 - product).
__device__ __forceinline__ float gelu_fwd_f(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.f));
  float q = fmaf(1.061405429f, t, -1.453152027f);
  q = fmaf(q, t, 1.421413741f);
  q = fmaf(q, t, -0.284496736f);
  q = fmaf(q, t, 0.254829592f);
  const float pe = q * t * __expf(-x * x);  // 1 - erf(x)
  return 0.5f * z * (z >= 0.f ? 2.f - pe : pe);
}

// The same inverse half of a Fourier layer with its two dense parts on the
// matrix cores. For one patch and image row y, the 32 outputs x 32 pixels
//   z[o][y][x] = sum_i pw[i][o] h[i][y][x]
//              + sum_kx (Re gy[o][y][kx] Re ix[kx][x] - Im gy[o][y][kx] Im ix[kx][x])
//              + pb[o]
// are one 32 x 32 FP32 tile with K = 32 + 18: the pointwise weights and the
// row transform's twiddles are fixed operands held in registers, the pixels
// come straight from memory (32 consecutive x per half-wave) and the column
// transform gy[o][y][kx] = sum_ky iy[y][ky] G[o][ky][kx] is formed on the
// vector units, 8 rows at a time, into LDS. The rows y and 32 - y have
// conjugate twiddles, so one set of products gives both: with A = sum Re iy G
// and B = sum Im iy G, gy[y] = A + i B and gy[32 - y] = A - i B (per complex
// part below); each group of 8 rows is 4 such pairs (rows 0 and 16 use direct
// sums). With BF16 these are still products of two rounded operands: rounding
// to nearest even is symmetric, so the rounded twiddles of 32 - y remain the
// conjugates of those of y.
// One patch per block of 8 waves; wave w takes slot w of each group, and its
// pixel loads for the next group are issued once the current ones are used.
constexpr int INVM_T = 512, GYS = 19;  // gy row stride (floats), odd against bank conflicts
// The image rows of group k (0..3), slot w (0..7): conjugate pairs (y, 32 - y)
// in slots w and w + 4, y = 4k + 1 + (w mod 4); the last group's slots 3 and
// 7 hold the self-paired rows 0 and 16.
__device__ __forceinline__ int inv_row(int k, int w) {
  const int base = 4 * k + 1 + (w & 3);
  if (k == 3 && (w & 3) == 3) return w < 4 ? 0 : SN / 2;
  return w < 4 ? base : SN - base;
}
template <bool BF16>
__global__ void __launch_bounds__(INVM_T) __attribute__((amdgpu_waves_per_eu(4)))
fused_dft_inv_mfma(
    const f2* __restrict__ G, const float* __restrict__ h, const f2* __restrict__ iy,
    const f2* __restrict__ ix, const float* __restrict__ pw, const float* __restrict__ pb,
    float* __restrict__ z_out, float* __restrict__ h_out, int apply_gelu) {
  __shared__ f2 gsm[SNM][SW];            // the patch's G, [mode][o]
  __shared__ f2 iys[SN * SKY];           // [y][ky]
  __shared__ float gyl[8][SW][GYS];      // [row of the group][o][kx re | kx im]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 31, lh = lane >> 5;
  const int b = blockIdx.x;
  const f2* gb = G + (long long)b * SNM * SW;
  for (int i = t; i < SNM * SW; i += INVM_T) (&gsm[0][0])[i] = op<BF16>(gb[i]);
  for (int i = t; i < SN * SKY; i += INVM_T) iys[i] = op<BF16>(iy[i]);
  // fixed operands: A = pw^T (row o = li, k = i), B = row-transform twiddles
  // (k' < 9: Re ix[k'][x], else -Im ix[k' - 9][x]; column x = li)
  float pwa[SW / 2], ixb[SKX];
#pragma unroll
  for (int s = 0; s < SW / 2; ++s) pwa[s] = op<BF16>(pw[(2 * s + lh) * SW + li]);
#pragma unroll
  for (int s = 0; s < SKX; ++s) {
    const int k = 2 * s + lh;
    ixb[s] = k < SKX ? op<BF16>(ix[k * SN + li]).x : -op<BF16>(ix[(k - SKX) * SN + li]).y;
  }
  const float* hb = h + (long long)b * SW * SN * SN;
  // this wave's pixels of its row: B operand of the pointwise part (k = i);
  // the next row's are loaded as soon as the current ones are consumed
  float hv[SW / 2];
#pragma unroll
  for (int s = 0; s < SW / 2; ++s) hv[s] = hb[((2 * s + lh) * SN + inv_row(0, wave)) * SN + li];
  for (int yc = 0; yc < SN / 8; ++yc) {
    const int y = inv_row(yc, wave);
    __syncthreads();  // G staged (first group) / the previous group's gy consumed
    // column transform of the group's 4 row pairs: items (pair, kx, o), o fastest
    for (int it = t; it < 4 * SKX * SW; it += INVM_T) {
      const int o = it % SW, kx = (it / SW) % SKX, pr = it / (SW * SKX);
      const int ya = inv_row(yc, pr), yb = inv_row(yc, pr + 4);
      float ra = 0.f, ia = 0.f, rb = 0.f, ib = 0.f;
      if (ya == 0) {  // rows 0 and 16
#pragma unroll 4
        for (int ky = 0; ky < SKY; ++ky) {
          const f2 v = gsm[ky * SKX + kx][o], a = iys[ya * SKY + ky], c = iys[yb * SKY + ky];
          ra = fmaf(a.x, v.x, fmaf(-a.y, v.y, ra));
          ia = fmaf(a.x, v.y, fmaf(a.y, v.x, ia));
          rb = fmaf(c.x, v.x, fmaf(-c.y, v.y, rb));
          ib = fmaf(c.x, v.y, fmaf(c.y, v.x, ib));
        }
      } else {
        float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
#pragma unroll
        for (int ky = 0; ky < SKY; ++ky) {
          const f2 v = gsm[ky * SKX + kx][o], a = iys[ya * SKY + ky];
          ar = fmaf(a.x, v.x, ar);
          ai = fmaf(a.x, v.y, ai);
          br = fmaf(a.y, v.y, br);
          bi = fmaf(a.y, v.x, bi);
        }
        ra = ar - br;
        ia = ai + bi;
        rb = ar + br;
        ib = ai - bi;
      }
      gyl[pr][o][kx] = op<BF16>(ra);
      gyl[pr][o][SKX + kx] = op<BF16>(ia);
      gyl[pr + 4][o][kx] = op<BF16>(rb);
      gyl[pr + 4][o][SKX + kx] = op<BF16>(ib);
    }
    __syncthreads();
    floatx16 acc = {0};
#pragma unroll
    for (int s = 0; s < SW / 2; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(pwa[s], op<BF16>(hv[s]), acc, 0, 0, 0);
    if (yc + 1 < SN / 8)  // rounded (BF16) where used, so the loads stay in flight
#pragma unroll
      for (int s = 0; s < SW / 2; ++s)
        hv[s] = hb[((2 * s + lh) * SN + inv_row(yc + 1, wave)) * SN + li];
#pragma unroll
    for (int s = 0; s < SKX; ++s)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(gyl[wave][li][2 * s + lh], ixb[s], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = 8 * (r / 4) + 4 * lh + (r % 4);
      const float z = acc[r] + pb[o];
      const long long off = (((long long)b * SW + o) * SN + y) * SN + li;
      if (z_out) z_out[off] = z;
      if (apply_gelu) h_out[off] = gelu_fwd_f(z);
      else if (h_out != z_out) h_out[off] = z;
    }
  }
}

// The head's mixing, 3 outputs: out[b][o][m] = sum_i A[b][i][m] W[i][o][m].
// One thread per (patch, mode), modes fastest: every channel's spectra of a
// patch are read as 64 consecutive modes per wave, the weights (small, cached)
// likewise, and each spectral value serves the three outputs.
template <bool BF16>
__global__ void __launch_bounds__(256) mode_mix_head(const f2* __restrict__ A,
                                                     const f2* __restrict__ Wt, int nmode, int B,
                                                     f2* __restrict__ out) {
  constexpr int O = 3;
  const int m = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (m >= nmode || b >= B) return;
  const f2* a = A + (long long)b * SW * nmode + m;
  const f2* w = Wt + m;
  f2 acc[O];
#pragma unroll
  for (int o = 0; o < O; ++o) acc[o] = f2{0.f, 0.f};
#pragma unroll 8
  for (int i = 0; i < SW; ++i) {
    const f2 v = op<BF16>(a[(long long)i * nmode]);
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const f2 c = op<BF16>(w[(i * O + o) * nmode]);
      acc[o].x = fmaf(v.x, c.x, fmaf(-v.y, c.y, acc[o].x));
      acc[o].y = fmaf(v.x, c.y, fmaf(v.y, c.x, acc[o].y));
    }
  }
#pragma unroll
  for (int o = 0; o < O; ++o) out[((long long)b * O + o) * nmode + m] = acc[o];
}

// Per-mode channel mixing of a Fourier layer on the matrix cores:
//   out[b][m][o] = sum_i A[m][b][i] Wm[m][i][o]   (complex, i, o < 32)
// with the spectra and the weights mode-major, as one real contraction over
// k = (part, i), K = 64, per mode:
//   Re(b, o) = sum_i Ar Wr - Ai Wi,   Im(b, o) = sum_i Ar Wi + Ai Wr,
// into two 32 x 32 FP32 accumulators (patches x outputs). Block = 32 patches x
// MM_G modes, one wave per mode. A mode's 32 x 32 tile of spectra is one
// contiguous 8 KB run, staged in LDS (rows padded); each lane reads its
// sixteen weights W[2s + half][lane] straight from memory (32 consecutive
// outputs per half-wave) and uses them for both halves of K; each half-wave
// writes the 32 outputs of one (patch, mode), one 256-byte run. With BF16 the operands are
// rounded to bf16 as they are read (their products are exact in FP32).
constexpr int MM_G = 4;
template <bool BF16>
__global__ void __launch_bounds__(256) mode_mix_mm(const f2* __restrict__ A,
                                                   const f2* __restrict__ Wm, int nmode, int B,
                                                   f2* __restrict__ out) {
  __shared__ f2 as[MM_G][32][SW + 1];  // [mode][patch][i]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 31, lh = lane >> 5;
  const int b0 = blockIdx.x * 32, m0 = blockIdx.y * MM_G;
  for (int q = t; q < MM_G * 32 * SW; q += 256) {
    const int mm = q / (32 * SW), bb = (q / SW) % 32, i = q % SW;
    const int m = m0 + mm, b = b0 + bb;
    as[mm][bb][i] = (m < nmode && b < B) ? op<BF16>(A[((long long)m * B + b) * SW + i])
                                         : f2{0.f, 0.f};
  }
  __syncthreads();
  const int m = m0 + wave;
  if (m >= nmode) return;  // no barrier follows
  const f2* wm = Wm + (long long)m * SW * SW + li;
  f2 wv[SW / 2];
#pragma unroll
  for (int s = 0; s < SW / 2; ++s) wv[s] = op<BF16>(wm[(2 * s + lh) * SW]);
  floatx16 cre = {0}, cim = {0};
#pragma unroll
  for (int s = 0; s < SW / 2; ++s) {  // real parts of A
    const float a = as[wave][li][2 * s + lh].x;
    cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a, wv[s].x, cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a, wv[s].y, cim, 0, 0, 0);
  }
#pragma unroll
  for (int s = 0; s < SW / 2; ++s) {  // imaginary parts of A
    const float a = as[wave][li][2 * s + lh].y;
    cre = __builtin_amdgcn_mfma_f32_32x32x2f32(a, -wv[s].y, cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_32x32x2f32(a, wv[s].x, cim, 0, 0, 0);
  }
  f2* dst = out + ((long long)b0 * nmode + m) * SW + li;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int bb = 8 * (r / 4) + 4 * lh + (r % 4);
    if (b0 + bb < B) dst[(long long)bb * nmode * SW] = f2{cre[r], cim[r]};
  }
}

// Mode-major copy of the layers' spectral weights: Wm[k][m][i][o] from
// W_k[i][o][m] (layer k at W + k * layer_stride complex values).
__global__ void spec_mode_major(const f2* __restrict__ W, long long layer_stride, int nmode,
                                f2* __restrict__ Wm) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // (m, i, o), o fastest
  if (q >= (long long)nmode * SW * SW) return;
  const int k = blockIdx.y;
  const int o = (int)(q % SW), i = (int)((q / SW) % SW), m = (int)(q / (SW * SW));
  Wm[(long long)k * nmode * SW * SW + q] = W[k * layer_stride + ((long long)i * SW + o) * nmode + m];
}

// The lift: h[b][o][p] = sum_c lw[c][o] x[b][c][p] + lb[o], 16 input and 32
// output channels; grid (B), 512 threads of 2 pixels each.
template <bool BF16>
__global__ void __launch_bounds__(512) lift_kernel(const float* __restrict__ x,
                                                   const float* __restrict__ lw,
                                                   const float* __restrict__ lb,
                                                   float* __restrict__ h) {
  constexpr int CI = 16;
  __shared__ float lws[CI * SW], lbs[SW];
  const int t = threadIdx.x, b = blockIdx.x;
  for (int i = t; i < CI * SW; i += 512) lws[i] = op<BF16>(lw[i]);
  if (t < SW) lbs[t] = lb[t];
  float xr[CI][2];
  const float* xb = x + (long long)b * CI * SN * SN;
#pragma unroll
  for (int c = 0; c < CI; ++c) {
    const float2 v = *reinterpret_cast<const float2*>(xb + c * SN * SN + 2 * t);
    xr[c][0] = op<BF16>(v.x);
    xr[c][1] = op<BF16>(v.y);
  }
  __syncthreads();
  float* hb = h + (long long)b * SW * SN * SN + 2 * t;
#pragma unroll 4
  for (int o = 0; o < SW; ++o) {
    float a0 = lbs[o], a1 = lbs[o];
#pragma unroll
    for (int c = 0; c < CI; ++c) {
      const float w = lws[c * SW + o];
      a0 = fmaf(w, xr[c][0], a0);
      a1 = fmaf(w, xr[c][1], a1);
    }
    *reinterpret_cast<float2*>(hb + o * SN * SN) = make_float2(a0, a1);
  }
}

// complex64 index patches [B][8][32][32] -> channels [B][16][32][32]
__global__ void encode(const float* n, float* x, long long per_layer_total, int P) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // over B*8*P
  if (i >= per_layer_total) return;
  const long long p = i % P, bl = i / P;  // bl = b*8 + l
  const long long b = bl / 8, l = bl % 8;
  x[((b * 16) + 2 * l) * P + p] = (n[2 * i] - 1.45f) / 0.15f;
  x[((b * 16) + 2 * l + 1) * P + p] = n[2 * i + 1] / 0.05f;
}

inline unsigned blocks(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_gemm(const GemmOp& op, hipStream_t s) {
  if (op.M <= 0 || op.N <= 0 || op.K <= 0 || op.batch <= 0) return hipSuccess;
  const int tm = op.bf16 ? BM : TM, tn = op.bf16 ? BN : TN;
  const long long tiles = (long long)((op.M + tm - 1) / tm) * ((op.N + tn - 1) / tn);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  // the batch runs on grid.y in chunks of at most 65535
  for (int b0 = 0; b0 < op.batch; b0 += 65535) {
    GemmOp c = op;
    c.batch = std::min(65535, op.batch - b0);
    c.A += (long long)b0 * op.a_bs * (op.a_cplx ? 2 : 1);
    c.B += (long long)b0 * op.b_bs * (op.b_cplx ? 2 : 1);
    c.C += (long long)b0 * op.c_bs * (op.c_cplx ? 2 : 1);
    dim3 grid((unsigned)tiles, c.batch);
    if (op.bf16)
      gemm_bf16_kernel<<<grid, 256, 0, s>>>(c);
    else
      gemm_kernel<<<grid, 256, 0, s>>>(c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t sur_gelu_bwd(const float* z, float* g, long long n, hipStream_t s) {
  gelu_bwd<<<blocks(n), 256, 0, s>>>(z, g, n);
  return hipGetLastError();
}
hipError_t sur_sum_batch(const float* in, float* out, int B, long long per, hipStream_t s) {
  sum_batch<<<blocks(per), 256, 0, s>>>(in, out, B, per);
  return hipGetLastError();
}
hipError_t sur_bias_grad(const float* g, float* out, int B, int C, int P, hipStream_t s) {
  bias_grad<<<C, 256, 0, s>>>(g, out, B, C, P);
  return hipGetLastError();
}
hipError_t sur_loss(const float* out, const float* tgt, long long n, float* sums, float* g,
                    hipStream_t s) {
  loss_sums<<<1, 256, 0, s>>>(out, tgt, n, sums);
  if (g) loss_grad<<<blocks(2 * n), 256, 0, s>>>(out, tgt, sums, g, 2 * n);
  return hipGetLastError();
}
hipError_t sur_adam(float* p, const float* g, float* m, float* v, long long n, float lr, int t,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  adam<<<blocks(n), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}
hipError_t sur_fused_dft_fwd(const float* h, const float* fy, const float* fx, float* H, int B,
                            bool head, bool bf16, hipStream_t s) {
  dim3 grid(SW / 8, B);
  auto go = [&](auto kern) {
    kern<<<grid, 256, 0, s>>>(h, reinterpret_cast<const f2*>(fy), reinterpret_cast<const f2*>(fx),
                              reinterpret_cast<f2*>(H));
  };
  if (head) {  // the head's centred 15 x 15 band, [b][i][mode]
    if (bf16) go(fused_dft_fwd<true, 15, 15, false>);
    else go(fused_dft_fwd<false, 15, 15, false>);
  } else {  // a Fourier layer's 17 x 9 half plane, [mode][b][i]
    if (bf16) go(fused_dft_fwd<true, SKY, SKX, true>);
    else go(fused_dft_fwd<false, SKY, SKX, true>);
  }
  return hipGetLastError();
}
hipError_t sur_fused_dft_inv(const float* G, const float* h, const float* iy, const float* ix,
                             const float* pw, const float* pb, float* z_out, float* h_out,
                             bool gelu, int B, bool bf16, hipStream_t s) {
  auto go = [&](auto kern) {
    kern<<<B, INVM_T, 0, s>>>(reinterpret_cast<const f2*>(G), h, reinterpret_cast<const f2*>(iy),
                            reinterpret_cast<const f2*>(ix), pw, pb, z_out, h_out, gelu ? 1 : 0);
  };
  if (bf16) go(fused_dft_inv_mfma<true>);
  else go(fused_dft_inv_mfma<false>);
  return hipGetLastError();
}
hipError_t sur_mode_mix(const float* A, const float* W, int nmode, int B, int O, float* out,
                        bool bf16, hipStream_t s) {
  const f2* a = reinterpret_cast<const f2*>(A);
  const f2* w = reinterpret_cast<const f2*>(W);
  f2* o = reinterpret_cast<f2*>(out);
  if (O == 3) {
    dim3 grid((nmode + 63) / 64, (B + 3) / 4);
    if (bf16) mode_mix_head<true><<<grid, 256, 0, s>>>(a, w, nmode, B, o);
    else mode_mix_head<false><<<grid, 256, 0, s>>>(a, w, nmode, B, o);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t sur_mode_mix_layer(const float* A, const float* Wm, int nmode, int B, float* out,
                              bool bf16, hipStream_t s) {
  dim3 grid((B + 31) / 32, (nmode + MM_G - 1) / MM_G);
  const f2* a = reinterpret_cast<const f2*>(A);
  const f2* w = reinterpret_cast<const f2*>(Wm);
  f2* o = reinterpret_cast<f2*>(out);
  if (bf16) mode_mix_mm<true><<<grid, 256, 0, s>>>(a, w, nmode, B, o);
  else mode_mix_mm<false><<<grid, 256, 0, s>>>(a, w, nmode, B, o);
  return hipGetLastError();
}
hipError_t sur_spec_mode_major(const float* W, long long layer_stride_floats, int nmode,
                               int layers, float* Wm, hipStream_t s) {
  if (layer_stride_floats % 2 != 0) return hipErrorInvalidValue;
  dim3 grid(blocks((long long)nmode * SW * SW), layers);
  spec_mode_major<<<grid, 256, 0, s>>>(reinterpret_cast<const f2*>(W), layer_stride_floats / 2,
                                       nmode, reinterpret_cast<f2*>(Wm));
  return hipGetLastError();
}
hipError_t sur_lift(const float* x, const float* lw, const float* lb, float* h, int B, bool bf16,
                    hipStream_t s) {
  if (bf16) lift_kernel<true><<<B, 512, 0, s>>>(x, lw, lb, h);
  else lift_kernel<false><<<B, 512, 0, s>>>(x, lw, lb, h);
  return hipGetLastError();
}
hipError_t sur_encode(const float* n, float* x, int B, hipStream_t s) {
  const long long tot = (long long)B * 8 * 1024;
  encode<<<blocks(tot), 256, 0, s>>>(n, x, tot, 1024);
  return hipGetLastError();
}

}  // namespace scw

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

// x[b][c][p] += bias[c]
__global__ void bias_add(float* x, const float* bias, int C, int P, long long total) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) x[i] += bias[(i / P) % C];
}

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__global__ void gelu_fwd(const float* z, float* h, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = gelu_f(z[i]);
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

hipError_t sur_bias_add(float* x, const float* bias, int B, int C, int P, hipStream_t s) {
  const long long n = (long long)B * C * P;
  bias_add<<<blocks(n), 256, 0, s>>>(x, bias, C, P, n);
  return hipGetLastError();
}
hipError_t sur_gelu_fwd(const float* z, float* h, long long n, hipStream_t s) {
  gelu_fwd<<<blocks(n), 256, 0, s>>>(z, h, n);
  return hipGetLastError();
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
hipError_t sur_encode(const float* n, float* x, int B, hipStream_t s) {
  const long long tot = (long long)B * 8 * 1024;
  encode<<<blocks(tot), 256, 0, s>>>(n, x, tot, 1024);
  return hipGetLastError();
}

}  // namespace scw

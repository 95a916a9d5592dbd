// Inverse 2D transform of the field spectra on the matrix cores (Eq. 10).
//
// For one plane/component with spectrum S[v][u] (V x U):
//   x pass (VALU, Horner):  T[v][f] = sum_u S[v][u] exp(2 pi i (u - U/2) f / fx)
//   y pass (MFMA GEMM):     E[g][f] = sum_v W[g][v] T[v][f],
//                           W[g][v] = exp(2 pi i (v - V/2) g / fy)
// The complex y pass is two real GEMMs with K = 2V:
//   Re E = [Re W, -Im W] . [Re T; Im T],   Im E = [Im W, Re W] . [Re T; Im T].
//
// Precision modes:
//   F32     v_mfma_f32_32x32x2_f32 on FP32 operands.
//   BF16X3  operands split x = hi + lo in bf16; products hi.hi + hi.lo + lo.hi
//           accumulated in FP32 by v_mfma_f32_32x32x16_bf16.
//   FP16X3  the same split in fp16 (v_mfma_f32_32x32x16_f16); the T operand of
//           each plane/component is scaled by a power of two chosen from the
//           largest row 1-norm of S, so that |T| stays below 2^14 and the lo
//           parts stay clear of the fp16 subnormal range; the scale is removed
//           from the FP32 accumulators.
//
// Operand layouts in global memory (written by the x pass / the plan):
//   F32:    B[pc][k][fx] float,             A[re|im][k][fy] float
//   split:  B[pc][hi|lo][k/8][fx][8],       A[re|im][hi|lo][k/8][fy][8]  (16-bit)
// with Kp = 2V rounded up to the MFMA K step and zero padded, so that the 32
// lanes of a half-wave read 32 consecutive elements (f32) or 16-byte chunks.
//
// 32x32 MFMA lane layouts (one wave): A[i][k] for lane i + 32*(k / KL), B[k][j]
// for lane j + 32*(k / KL), KL = 1 (f32) or 8 (16-bit, 8 consecutive k per
// lane); accumulator register r of lane l holds D[8(r/4) + 4(l/32) + r%4][l%32].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "scw_internal.h"

namespace scw {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

enum Mode { kF32 = 0, kBF16 = 1, kFP16 = 2 };

__device__ __forceinline__ unsigned short to16(float x, int mode) {
  if (mode == kBF16) {
    __bf16 h = (__bf16)x;
    return __builtin_bit_cast(unsigned short, h);
  }
  _Float16 h = (_Float16)x;
  return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float from16(unsigned short b, int mode) {
  if (mode == kBF16) return (float)__builtin_bit_cast(__bf16, b);
  return (float)__builtin_bit_cast(_Float16, b);
}

struct c32 {
  float x, y;
};
__device__ __forceinline__ c32 muladd(c32 a, c32 w, c32 c) {  // a*w + c
  return {fmaf(a.x, w.x, fmaf(-a.y, w.y, c.x)), fmaf(a.x, w.y, fmaf(a.y, w.x, c.y))};
}
__device__ __forceinline__ c32 mul(c32 a, c32 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// ---------------------------------------------------------------- x pass
// Block = one plane/component and 64 columns f; its 256 threads are 64
// columns x 4 row groups (group q takes rows v = q, q+4, ...), so each Horner
// chain is U long and a block has 4 independent chains per column.
constexpr int XC = 64;

template <int MODE>
__global__ void __launch_bounds__(256) idft_x_kernel(
    const c32* __restrict__ spec, const c32* __restrict__ wx, int U, int V, int fx, int Kp,
    void* __restrict__ bmat, float* __restrict__ bscale) {
  extern __shared__ unsigned char smem_raw[];
  c32* S = reinterpret_cast<c32*>(smem_raw);  // [V*U]
  c32* Tt = S + U * V;                        // [V][XC]
  __shared__ float s_norm[64];
  const int M = U * V;
  const int pc = blockIdx.y;
  const int t = threadIdx.x, col = t % XC, q = t / XC;
  const int f = blockIdx.x * XC + col;
  const c32* src = spec + (long long)pc * M;
  for (int i = t; i < M; i += 256) S[i] = src[i];
  __syncthreads();
  float scale = 1.f;
  if (MODE == kFP16) {
    if (t < V) {
      float s = 0.f;
      for (int u = 0; u < U; ++u) s += fabsf(S[t * U + u].x) + fabsf(S[t * U + u].y);
      s_norm[t] = s;
    }
    __syncthreads();
    float mx = 0.f;
    for (int v = 0; v < V; ++v) mx = fmaxf(mx, s_norm[v]);
    // largest power of two with scale * max row 1-norm <= 2^14 (bounds |T|)
    if (mx > 0.f) scale = exp2f(floorf(14.f - log2f(mx)));
    if (blockIdx.x == 0 && t == 0) bscale[pc] = scale;
  }
  const bool live = f < fx;
  const c32 w = live ? wx[f] : c32{0.f, 0.f}, sh = live ? wx[fx + f] : c32{0.f, 0.f};
  for (int v = q; v < V; v += 4) {
    const c32* row = S + v * U;
    c32 acc = row[U - 1];
    for (int u = U - 2; u >= 0; --u) acc = muladd(acc, w, row[u]);
    const c32 o = mul(acc, sh);
    Tt[v * XC + col] = {o.x * scale, o.y * scale};
  }
  if (MODE == kF32) {
    // B[pc][k][fx]: rows k < V real parts, V <= k < 2V imaginary parts
    if (!live) return;
    float* B = reinterpret_cast<float*>(bmat) + (long long)pc * Kp * fx;
    for (int v = q; v < V; v += 4) {
      B[(long long)v * fx + f] = Tt[v * XC + col].x;
      B[(long long)(V + v) * fx + f] = Tt[v * XC + col].y;
    }
    for (int k = 2 * V + q; k < Kp; k += 4) B[(long long)k * fx + f] = 0.f;
  } else {
    // B[pc][hi|lo][Kp/8][fx][8]: 8 consecutive k of one column per 16 bytes
    __syncthreads();
    if (!live) return;
    unsigned short* Bh = reinterpret_cast<unsigned short*>(bmat) + (long long)pc * 2 * fx * Kp;
    unsigned short* Bl = Bh + (long long)fx * Kp;
    for (int c8 = q; c8 < Kp / 8; c8 += 4) {
      u16x8 hv, lv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = c8 * 8 + e;
        float x = 0.f;
        if (k < V) x = Tt[k * XC + col].x;
        else if (k < 2 * V) x = Tt[(k - V) * XC + col].y;
        const unsigned short h = to16(x, MODE);
        hv[e] = h;
        lv[e] = to16(x - from16(h, MODE), MODE);
      }
      const long long off = ((long long)c8 * fx + f) * 8;
      *reinterpret_cast<u16x8*>(Bh + off) = hv;
      *reinterpret_cast<u16x8*>(Bl + off) = lv;
    }
  }
}

// ---------------------------------------------------------------- y pass
// Block = 4 waves; wave w owns output rows g0 + 32w .. +31 and 64 columns
// (two 32x32 MFMA tiles). The twiddle fragments of the wave's rows are loaded
// once into registers and reused for the block's run of plane/components; the
// T fragments are read straight from global memory in the k-chunk-major layout,
// so each half-wave reads 32 consecutive 16-byte (or 4-byte) chunks.
constexpr int GB = 128;
constexpr int FB = 64;
constexpr int KSMAX_F32 = 32;   // V <= 32
constexpr int KSMAX_16 = 4;     // Kp <= 64

// Block index -> tile so that the tiles of one run of plane/components, which
// share the twiddle rows, go to the same XCD (blocks reach the 8 XCDs round
// robin).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

template <int MODE>
__global__ void __launch_bounds__(256) idft_y_kernel(
    const void* __restrict__ amat, const void* __restrict__ bmat,
    const float* __restrict__ bscale, int fx, int fy, int fz, int Kp, int ngt, int nft,
    int pcb, c32* __restrict__ E) {
  const int n_pc = fz * 3;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ft = tile % nft;
  const int gt = (tile / nft) % ngt;
  const int pg = tile / (nft * ngt);
  const int pc0 = pg * pcb, pc1 = min(n_pc, pc0 + pcb);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int li = lane & 31, lh = lane >> 5;
  const int g0 = gt * GB + wave * 32, f0 = ft * FB;
  const int ga = min(g0 + li, fy - 1);  // A row of this lane (rows past fy are not stored)
  const int fb0 = min(f0 + li, fx - 1), fb1 = min(f0 + 32 + li, fx - 1);
  typedef float f2v __attribute__((ext_vector_type(2)));

  if constexpr (MODE == kF32) {
    const int KS = Kp / 2;
    const float* Ar = reinterpret_cast<const float*>(amat);   // [re|im][Kp][fy]
    const float* Ai = Ar + (long long)Kp * fy;
    float ar[KSMAX_F32], ai[KSMAX_F32];
#pragma unroll
    for (int ks = 0; ks < KSMAX_F32; ++ks) {
      if (ks < KS) {
        ar[ks] = Ar[(long long)(2 * ks + lh) * fy + ga];
        ai[ks] = Ai[(long long)(2 * ks + lh) * fy + ga];
      }
    }
    for (int pc = pc0; pc < pc1; ++pc) {
      const float* B = reinterpret_cast<const float*>(bmat) + (long long)pc * Kp * fx;
      floatx16 cr0 = {0}, ci0 = {0}, cr1 = {0}, ci1 = {0};
#pragma unroll
      for (int ks = 0; ks < KSMAX_F32; ++ks) {
        if (ks < KS) {
          const float b0 = B[(long long)(2 * ks + lh) * fx + fb0];
          const float b1 = B[(long long)(2 * ks + lh) * fx + fb1];
          cr0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[ks], b0, cr0, 0, 0, 0);
          ci0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[ks], b0, ci0, 0, 0, 0);
          cr1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[ks], b1, cr1, 0, 0, 0);
          ci1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[ks], b1, ci1, 0, 0, 0);
        }
      }
      const int plane = pc / 3, comp = pc % 3;
      c32* dst = E + (((long long)comp * fz + plane) * fy) * fx;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int g = g0 + 8 * (r / 4) + 4 * lh + (r % 4);
        if (g < fy) {
          if (f0 + li < fx)
            __builtin_nontemporal_store(f2v{cr0[r], ci0[r]},
                                        reinterpret_cast<f2v*>(dst + (long long)g * fx + f0 + li));
          if (f0 + 32 + li < fx)
            __builtin_nontemporal_store(
                f2v{cr1[r], ci1[r]}, reinterpret_cast<f2v*>(dst + (long long)g * fx + f0 + 32 + li));
        }
      }
    }
  } else {
    const int KS = Kp / 16;
    // A[re|im][hi|lo][Kp/8][fy][8]
    const unsigned short* A = reinterpret_cast<const unsigned short*>(amat);
    const long long aq = (long long)Kp * fy;  // elements per (re|im, hi|lo) plane
    u16x8 arh[KSMAX_16], arl[KSMAX_16], aih[KSMAX_16], ail[KSMAX_16];
#pragma unroll
    for (int ks = 0; ks < KSMAX_16; ++ks) {
      if (ks < KS) {
        const long long o = ((long long)(2 * ks + lh) * fy + ga) * 8;
        arh[ks] = *reinterpret_cast<const u16x8*>(A + 0 * aq + o);
        arl[ks] = *reinterpret_cast<const u16x8*>(A + 1 * aq + o);
        aih[ks] = *reinterpret_cast<const u16x8*>(A + 2 * aq + o);
        ail[ks] = *reinterpret_cast<const u16x8*>(A + 3 * aq + o);
      }
    }
    for (int pc = pc0; pc < pc1; ++pc) {
      const unsigned short* Bh = reinterpret_cast<const unsigned short*>(bmat) +
                                 (long long)pc * 2 * fx * Kp;
      const unsigned short* Bl = Bh + (long long)fx * Kp;
      floatx16 cr0 = {0}, ci0 = {0}, cr1 = {0}, ci1 = {0};
#pragma unroll
      for (int ks = 0; ks < KSMAX_16; ++ks) {
        if (ks < KS) {
          const long long o0 = ((long long)(2 * ks + lh) * fx + fb0) * 8;
          const long long o1 = ((long long)(2 * ks + lh) * fx + fb1) * 8;
          const u16x8 bh0 = *reinterpret_cast<const u16x8*>(Bh + o0);
          const u16x8 bl0 = *reinterpret_cast<const u16x8*>(Bl + o0);
          const u16x8 bh1 = *reinterpret_cast<const u16x8*>(Bh + o1);
          const u16x8 bl1 = *reinterpret_cast<const u16x8*>(Bl + o1);
          if constexpr (MODE == kBF16) {
#define MF(a, b, c) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), \
                                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0)
            MF(arh[ks], bh0, cr0); MF(arh[ks], bl0, cr0); MF(arl[ks], bh0, cr0);
            MF(aih[ks], bh0, ci0); MF(aih[ks], bl0, ci0); MF(ail[ks], bh0, ci0);
            MF(arh[ks], bh1, cr1); MF(arh[ks], bl1, cr1); MF(arl[ks], bh1, cr1);
            MF(aih[ks], bh1, ci1); MF(aih[ks], bl1, ci1); MF(ail[ks], bh1, ci1);
#undef MF
          } else {
#define MF(a, b, c) c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), \
                                                               __builtin_bit_cast(halfx8, b), c, 0, 0, 0)
            MF(arh[ks], bh0, cr0); MF(arh[ks], bl0, cr0); MF(arl[ks], bh0, cr0);
            MF(aih[ks], bh0, ci0); MF(aih[ks], bl0, ci0); MF(ail[ks], bh0, ci0);
            MF(arh[ks], bh1, cr1); MF(arh[ks], bl1, cr1); MF(arl[ks], bh1, cr1);
            MF(aih[ks], bh1, ci1); MF(aih[ks], bl1, ci1); MF(ail[ks], bh1, ci1);
#undef MF
          }
        }
      }
      const float inv = (MODE == kFP16) ? 1.f / bscale[pc] : 1.f;
      const int plane = pc / 3, comp = pc % 3;
      c32* dst = E + (((long long)comp * fz + plane) * fy) * fx;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int g = g0 + 8 * (r / 4) + 4 * lh + (r % 4);
        if (g < fy) {
          if (f0 + li < fx)
            __builtin_nontemporal_store(f2v{cr0[r] * inv, ci0[r] * inv},
                                        reinterpret_cast<f2v*>(dst + (long long)g * fx + f0 + li));
          if (f0 + 32 + li < fx)
            __builtin_nontemporal_store(
                f2v{cr1[r] * inv, ci1[r] * inv},
                reinterpret_cast<f2v*>(dst + (long long)g * fx + f0 + 32 + li));
        }
      }
    }
  }
}

template <int MODE>
hipError_t launch_mode(const MfmaArgs& a, hipStream_t s) {
  const int n_pc = a.fz * 3;
  {
    const size_t lds = ((size_t)a.U * a.V + (size_t)a.V * XC) * sizeof(c32);
    dim3 grid((a.fx + XC - 1) / XC, n_pc);
    idft_x_kernel<MODE><<<grid, 256, lds, s>>>(
        reinterpret_cast<const c32*>(a.spec), reinterpret_cast<const c32*>(a.wx), a.U, a.V,
        a.fx, a.Kp, a.bmat, a.bscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int ngt = (a.fy + GB - 1) / GB, nft = (a.fx + FB - 1) / FB;
  // plane/components per block: about four blocks per CU
  int pcb = a.pcb > 0 ? a.pcb : (int)std::max<long long>(1, (long long)n_pc * ngt * nft / 1024);
  pcb = std::min(pcb, n_pc);
  const long long nb = (long long)((n_pc + pcb - 1) / pcb) * ngt * nft;
  idft_y_kernel<MODE><<<(unsigned)nb, 256, 0, s>>>(a.amat, a.bmat, a.bscale, a.fx, a.fy, a.fz,
                                                   a.Kp, ngt, nft, pcb,
                                                   reinterpret_cast<c32*>(a.E));
  return hipGetLastError();
}

}  // namespace

int mfma_kstep(int precision) { return precision == SCW_FP32 ? 2 : 16; }

hipError_t launch_idft_mfma(const MfmaArgs& a, int precision, hipStream_t s) {
  switch (precision) {
    case SCW_FP32: return launch_mode<kF32>(a, s);
    case SCW_BF16X3: return launch_mode<kBF16>(a, s);
    case SCW_FP16X3: return launch_mode<kFP16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace scw

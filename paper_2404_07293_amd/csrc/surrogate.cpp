// Spectral-convolution surrogate of the CWT transmitted field, trained and
// run on the GPU by the kernels of kernels_surrogate.hip.
//
// Input: a complex-index patch of 8 layers x 32 x 32 voxels at pitch lambda/4
// (lambda = 1), normal x-polarised plane wave, index 1 above and below. Output:
// the transmitted plane-wave coefficients p_trn of Eq. 9 on the 15 x 15 band
// (3 components, mode order of Sec. 2.2). Network (FP32 storage; the matrix
// products in FP32 on the vector units or in bf16 on the matrix cores):
//   x (16 ch: Re and Im of each layer, normalised) -> lift to 32 channels ->
//   4 x [ truncated DFT2 (ky in [-8,8], kx in [0,8]) -> per-mode complex 32x32
//         mix -> real inverse DFT2  +  pointwise 32x32 map + bias -> GELU
//         (not after the last) ] ->
//   DFT2 / 1024 on ky, kx in [-7,7] -> per-mode complex 32 -> 3 map.
// Parameters are one flat FP32 array in the order lift_w [16][32], lift_b
// [32], then per layer spec [32][32][17][9] complex, pw [32][32], pb [32],
// then head [32][3][15][15] complex (complex values interleaved).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <new>
#include <random>
#include <utility>
#include <vector>

#include "scw_internal.h"

namespace scw {
namespace {

constexpr int CIN = 16, W = 32, NP = 1024, NL = 4;
constexpr int KYN = 17, KXN = 9, NM = KYN * KXN;  // 153 spectral modes
constexpr int HN = 15, HM = HN * HN;              // 225 head modes
constexpr int OUT = 3;

constexpr long long SZ_LW = CIN * W, SZ_LB = W;
constexpr long long SZ_SPEC = 2LL * W * W * NM, SZ_PW = W * W, SZ_PB = W;
constexpr long long SZ_HEAD = 2LL * W * OUT * HM;
constexpr long long SZ_LAYER = SZ_SPEC + SZ_PW + SZ_PB;
constexpr long long N_PARAMS = SZ_LW + SZ_LB + NL * SZ_LAYER + SZ_HEAD;

struct Off {
  long long lw = 0, lb = SZ_LW;
  long long spec(int k) const { return SZ_LW + SZ_LB + k * SZ_LAYER; }
  long long pw(int k) const { return spec(k) + SZ_SPEC; }
  long long pb(int k) const { return pw(k) + SZ_PW; }
  long long head() const { return SZ_LW + SZ_LB + NL * SZ_LAYER; }
};

}  // namespace

struct SurNet {
  Context* ctx = nullptr;
  int max_batch = 0;
  int step = 0;
  bool bf16 = false;  // GEMM operands in bf16 on the matrix cores (FP32 accumulate)
  DevBuf params, grads, adam_m, adam_v;
  DevBuf dft;  // fy, fx, iy, ix, hy, hx (complex64)
  long long o_fy, o_fx, o_iy, o_ix, o_hy, o_hx;
  DevBuf x, h[NL + 1], z[NL], Hk[NL], G, Wm, F, out, gout, gF, T1, gh, gh2, T2, gG, gH,
      tmp, sums, enc_in;
  DevBuf Wb;  // mixing weights as bf16 matrix-core operands (inference)
  // the parameters change only in sur_set_params and Adam steps; Wb is rebuilt
  // when its version lags behind theirs
  unsigned long long params_version = 1, wb_version = 0;
};

namespace {

int alloc(DevBuf& b, long long floats) { return b.reserve((size_t)std::max(1LL, floats) * 4); }

struct G {
  GemmOp op{};
  G(int M, int N, int K, int batch) {
    op.M = M;
    op.N = N;
    op.K = K;
    op.batch = batch;
  }
  G& a(const float* p, bool cplx, long long rs, long long cs, long long bs, bool conj = false) {
    op.A = p;
    op.a_cplx = cplx;
    op.a_rs = rs;
    op.a_cs = cs;
    op.a_bs = bs;
    op.conj_a = conj;
    return *this;
  }
  G& b(const float* p, bool cplx, long long rs, long long cs, long long bs, bool conj = false) {
    op.B = p;
    op.b_cplx = cplx;
    op.b_rs = rs;
    op.b_cs = cs;
    op.b_bs = bs;
    op.conj_b = conj;
    return *this;
  }
  G& c(float* p, bool cplx, long long rs, long long cs, long long bs, float beta = 0.f) {
    op.C = p;
    op.c_cplx = cplx;
    op.c_rs = rs;
    op.c_cs = cs;
    op.c_bs = bs;
    op.beta = beta;
    return *this;
  }
  hipError_t run(hipStream_t s, bool bf16) {
    op.bf16 = bf16 ? 1 : 0;
    return launch_gemm(op, s);
  }
};

#define SUR_HIP(x)                                                        \
  do {                                                                    \
    hipError_t e__ = (x);                                                 \
    if (e__ != hipSuccess)                                                \
      return fail(SCW_EHIP, std::string("surrogate: ") + hipGetErrorString(e__)); \
  } while (0)

int build_dft(SurNet& n) {
  std::vector<std::complex<double>> v;
  auto e = [](double ang) { return std::complex<double>(std::cos(ang), std::sin(ang)); };
  const double tp = 2.0 * M_PI / 32.0;
  n.o_fy = 0;
  for (int ky = -8; ky <= 8; ++ky)
    for (int y = 0; y < 32; ++y) v.push_back(e(-tp * ((ky * y) % 32)));
  n.o_fx = (long long)v.size();
  for (int x = 0; x < 32; ++x)
    for (int kx = 0; kx <= 8; ++kx) v.push_back(e(-tp * ((kx * x) % 32)));
  n.o_iy = (long long)v.size();
  for (int y = 0; y < 32; ++y)
    for (int ky = -8; ky <= 8; ++ky) v.push_back(e(tp * ((ky * y) % 32)));
  n.o_ix = (long long)v.size();
  for (int kx = 0; kx <= 8; ++kx)
    for (int x = 0; x < 32; ++x)
      v.push_back((kx > 0 ? 2.0 : 1.0) / 1024.0 * e(tp * ((kx * x) % 32)));
  n.o_hy = (long long)v.size();
  for (int ky = -7; ky <= 7; ++ky)
    for (int y = 0; y < 32; ++y) v.push_back(e(-tp * ((ky * y) % 32)) / 32.0);
  n.o_hx = (long long)v.size();
  for (int x = 0; x < 32; ++x)
    for (int kx = -7; kx <= 7; ++kx) v.push_back(e(-tp * ((kx * x) % 32)) / 32.0);
  std::vector<float> f(2 * v.size());
  for (size_t i = 0; i < v.size(); ++i) {
    f[2 * i] = (float)v[i].real();
    f[2 * i + 1] = (float)v[i].imag();
  }
  int rc = n.dft.reserve(f.size() * 4);
  if (rc) return rc;
  SUR_HIP(hipMemcpy(n.dft.p, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  return SCW_OK;
}

const float* cx(const SurNet& n, long long off) { return n.dft.as<float>() + 2 * off; }

// Forward pass; with keep, the per-layer H spectra and pre-activations stay
// for the backward pass (h[] is always kept).
int forward(SurNet& n, const float* x, int B, hipStream_t s, bool keep) {
  const Off o;
  const float* P = n.params.as<float>();
  // mode-major copy of the spectral weights, for the mixing
  SUR_HIP(sur_spec_mode_major(P + o.spec(0), SZ_LAYER, NM, NL, n.Wm.as<float>(), s));
  // lift
  SUR_HIP(sur_lift(x, P + o.lw, P + o.lb, n.h[0].as<float>(), B, n.bf16, s));
  for (int k = 0; k < NL; ++k) {
    const float* hin = n.h[k].as<float>();
    float* Hk = n.Hk[k].as<float>();
    const bool last = k == NL - 1;
    // H = fy h fx per channel (the layer's truncated forward transform)
    SUR_HIP(sur_fused_dft_fwd(hin, cx(n, n.o_fy), cx(n, n.o_fx), Hk, B, false, n.bf16, s));
    // G[b][m] = H[m][b] W_k[m] per mode over the patches (H mode-major)
    SUR_HIP(sur_mode_mix_layer(Hk, n.Wm.as<float>() + 2LL * k * NM * W * W, NM, B,
                               n.G.as<float>(), n.bf16, s));
    // z = Re(iy G ix) + P_k^T h + c_k; h' = GELU(z) except after the last layer
    // the pre-activation is kept only for the backward pass
    float* zk = last ? n.h[k + 1].as<float>() : (keep ? n.z[k].as<float>() : nullptr);
    SUR_HIP(sur_fused_dft_inv(n.G.as<float>(), hin, cx(n, n.o_iy), cx(n, n.o_ix),
                              P + o.pw(k), P + o.pb(k), zk, n.h[k + 1].as<float>(), !last, B,
                              n.bf16, s));
  }
  // head: F = hy h hx per channel on the centred 15 x 15 band
  SUR_HIP(sur_fused_dft_fwd(n.h[NL].as<float>(), cx(n, n.o_hy), cx(n, n.o_hx), n.F.as<float>(),
                            B, true, n.bf16, s));
  SUR_HIP(sur_mode_mix(n.F.as<float>(), P + o.head(), HM, B, OUT, n.out.as<float>(), n.bf16, s));
  return SCW_OK;
}

// Inference in the matrix-core mode with bf16 storage: the same network and
// the same rounded operands as forward() with n.bf16, every activation and
// spectrum kept in bf16 (h ping-pongs between the memory of h[0] and h[1]).
int forward_bf16(SurNet& n, const float* x, int B, hipStream_t s) {
  const Off o;
  const float* P = n.params.as<float>();
  if (n.wb_version != n.params_version) {
    SUR_HIP(sur_mix_weights_bf16(P + o.spec(0), SZ_LAYER, NL, n.Wb.p, s));
    n.wb_version = n.params_version;
  }
  void* ha = n.h[0].p;
  void* hb = n.h[1].p;
  SUR_HIP(sur_lift_bf16(x, P + o.lw, P + o.lb, ha, B, s));
  const size_t wl = sur_mix_weights_bf16_bytes(1);
  for (int k = 0; k < NL; ++k) {
    SUR_HIP(sur_fwd_bf16(ha, cx(n, n.o_fy), cx(n, n.o_fx), n.Hk[0].p, B, false, s));
    SUR_HIP(sur_mix_bf16(n.Hk[0].p, static_cast<char*>(n.Wb.p) + k * wl, B, n.G.p, s));
    SUR_HIP(sur_inv_bf16(n.G.p, ha, cx(n, n.o_iy), cx(n, n.o_ix), P + o.pw(k), P + o.pb(k), hb,
                         k < NL - 1, B, s));
    std::swap(ha, hb);
  }
  SUR_HIP(sur_fwd_bf16(ha, cx(n, n.o_hy), cx(n, n.o_hx), n.F.p, B, true, s));
  SUR_HIP(sur_head_mix_bf16(n.F.p, P + o.head(), B, n.out.as<float>(), s));
  return SCW_OK;
}

int infer(SurNet& n, const float* x, int B, hipStream_t s) {
  return n.bf16 ? forward_bf16(n, x, B, s) : forward(n, x, B, s, false);
}

// Backward pass from gout (= dL/dout) into grads.
int backward(SurNet& n, int B, hipStream_t s) {
  const Off o;
  const float* P = n.params.as<float>();
  float* Gr = n.grads.as<float>();
  const long long act = (long long)W * NP;
  // head
  SUR_HIP(G(W, OUT, B, HM).a(n.F.as<float>(), true, HM, (long long)W * HM, 1, true)
              .b(n.gout.as<float>(), true, (long long)OUT * HM, HM, 1)
              .c(Gr + o.head(), true, (long long)OUT * HM, HM, 1).run(s, n.bf16));
  SUR_HIP(G(B, W, OUT, HM).a(n.gout.as<float>(), true, (long long)OUT * HM, HM, 1)
              .b(P + o.head(), true, HM, (long long)OUT * HM, 1, true)
              .c(n.gF.as<float>(), true, (long long)W * HM, HM, 1).run(s, n.bf16));
  SUR_HIP(G(32, HN, HN, B * W).a(cx(n, n.o_hy), true, 1, 32, 0, true)
              .b(n.gF.as<float>(), true, HN, 1, HM).c(n.T1.as<float>(), true, HN, 1, 32 * HN)
              .run(s, n.bf16));
  SUR_HIP(G(B * NP, 32, HN, 1).a(n.T1.as<float>(), true, HN, 1, 0)
              .b(cx(n, n.o_hx), true, 1, HN, 0, true).c(n.gh.as<float>(), false, 32, 1, 0)
              .run(s, n.bf16));
  DevBuf* gh = &n.gh;
  DevBuf* gh2 = &n.gh2;
  for (int k = NL - 1; k >= 0; --k) {
    float* gz = gh->as<float>();
    if (k < NL - 1) SUR_HIP(sur_gelu_bwd(n.z[k].as<float>(), gz, (long long)B * act, s));
    const float* hin = n.h[k].as<float>();
    // pointwise weight and bias
    SUR_HIP(G(W, W, NP, B).a(hin, false, NP, 1, act).b(gz, false, 1, NP, act)
                .c(n.tmp.as<float>(), false, W, 1, W * W).run(s, n.bf16));
    SUR_HIP(sur_sum_batch(n.tmp.as<float>(), Gr + o.pw(k), B, W * W, s));
    SUR_HIP(sur_bias_grad(gz, Gr + o.pb(k), B, W, NP, s));
    float* g2 = gh2->as<float>();
    SUR_HIP(G(W, NP, W, B).a(P + o.pw(k), false, W, 1, 0).b(gz, false, NP, 1, act)
                .c(g2, false, NP, 1, act).run(s, n.bf16));
    // spectral branch
    SUR_HIP(G(B * NP, KXN, 32, 1).a(gz, false, 32, 1, 0).b(cx(n, n.o_ix), true, 1, 32, 0, true)
                .c(n.T2.as<float>(), true, KXN, 1, 0).run(s, n.bf16));
    SUR_HIP(G(KYN, KXN, 32, B * W).a(cx(n, n.o_iy), true, 1, KYN, 0, true)
                .b(n.T2.as<float>(), true, KXN, 1, 32 * KXN).c(n.gG.as<float>(), true, KXN, 1, NM)
                .run(s, n.bf16));
    SUR_HIP(G(W, W, B, NM).a(n.Hk[k].as<float>(), true, 1, W, (long long)B * W, true)
                .b(n.gG.as<float>(), true, (long long)W * NM, NM, 1)
                .c(Gr + o.spec(k), true, (long long)W * NM, NM, 1).run(s, n.bf16));
    SUR_HIP(G(B, W, W, NM).a(n.gG.as<float>(), true, (long long)W * NM, NM, 1)
                .b(P + o.spec(k), true, NM, (long long)W * NM, 1, true)
                .c(n.gH.as<float>(), true, (long long)W * NM, NM, 1).run(s, n.bf16));
    SUR_HIP(G(32, KXN, KYN, B * W).a(cx(n, n.o_fy), true, 1, 32, 0, true)
                .b(n.gH.as<float>(), true, KXN, 1, NM).c(n.T2.as<float>(), true, KXN, 1, 32 * KXN)
                .run(s, n.bf16));
    SUR_HIP(G(B * NP, 32, KXN, 1).a(n.T2.as<float>(), true, KXN, 1, 0)
                .b(cx(n, n.o_fx), true, 1, KXN, 0, true).c(g2, false, 32, 1, 0, 1.f).run(s, n.bf16));
    std::swap(gh, gh2);
  }
  // lift
  SUR_HIP(G(CIN, W, NP, B).a(n.x.as<float>(), false, NP, 1, (long long)CIN * NP)
              .b(gh->as<float>(), false, 1, NP, act).c(n.tmp.as<float>(), false, W, 1, CIN * W)
              .run(s, n.bf16));
  SUR_HIP(sur_sum_batch(n.tmp.as<float>(), Gr + o.lw, B, CIN * W, s));
  SUR_HIP(sur_bias_grad(gh->as<float>(), Gr + o.lb, B, W, NP, s));
  return SCW_OK;
}

int check_batch(const SurNet& n, int B) {
  if (B < 1 || B > n.max_batch)
    return fail(SCW_EINVAL, "surrogate batch must be in [1, " + std::to_string(n.max_batch) + "]");
  return SCW_OK;
}

}  // namespace

long long sur_param_count() { return N_PARAMS; }

int sur_create(Context& ctx, int max_batch, unsigned long long seed, SurNet** out) {
  if (max_batch < 1 || max_batch > 65536) return fail(SCW_EINVAL, "max_batch out of range");
  SCW_HIP(hipSetDevice(ctx.device));
  std::unique_ptr<SurNet> n(new (std::nothrow) SurNet());
  if (!n) return fail(SCW_ENOMEM, "surrogate allocation failed");
  n->ctx = &ctx;
  n->max_batch = max_batch;
  const long long B = max_batch, act = (long long)B * W * NP;
  int rc;
  if ((rc = alloc(n->params, N_PARAMS)) || (rc = alloc(n->grads, N_PARAMS)) ||
      (rc = alloc(n->adam_m, N_PARAMS)) || (rc = alloc(n->adam_v, N_PARAMS)) ||
      (rc = alloc(n->x, B * CIN * NP)) || (rc = alloc(n->enc_in, B * 8 * NP * 2)) ||
      (rc = alloc(n->G, B * W * NM * 2)) || (rc = alloc(n->Wm, (long long)NL * NM * W * W * 2)) ||
      (rc = alloc(n->F, B * W * HM * 2)) || (rc = alloc(n->out, B * OUT * HM * 2)) ||
      (rc = alloc(n->gout, B * OUT * HM * 2)) || (rc = alloc(n->gF, B * W * HM * 2)) ||
      (rc = alloc(n->T1, B * W * 32 * HN * 2)) || (rc = alloc(n->gh, act)) ||
      (rc = alloc(n->gh2, act)) || (rc = alloc(n->T2, B * W * 32 * KXN * 2)) ||
      (rc = alloc(n->gG, B * W * NM * 2)) || (rc = alloc(n->gH, B * W * NM * 2)) ||
      (rc = alloc(n->tmp, B * W * W)) || (rc = alloc(n->sums, 16)) ||
      (rc = n->Wb.reserve(sur_mix_weights_bf16_bytes(NL))))
    return rc;
  for (int k = 0; k <= NL; ++k)
    if ((rc = alloc(n->h[k], act))) return rc;
  for (int k = 0; k < NL; ++k)
    if ((rc = alloc(n->z[k], act)) || (rc = alloc(n->Hk[k], B * W * NM * 2))) return rc;
  if ((rc = build_dft(*n))) return rc;
  // initial weights: N(0, 1/fan_in) for real maps, complex with the same total
  // variance (spectral mixing scaled down by 4), zero biases
  std::vector<float> p(N_PARAMS, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  const Off o;
  auto fill = [&](long long off, long long cnt, double sd) {
    for (long long i = 0; i < cnt; ++i) p[off + i] = (float)(sd * nd(rng));
  };
  fill(o.lw, SZ_LW, 1.0 / std::sqrt((double)CIN));
  for (int k = 0; k < NL; ++k) {
    fill(o.spec(k), SZ_SPEC, 1.0 / std::sqrt(2.0 * W) / 4.0);
    fill(o.pw(k), SZ_PW, 1.0 / std::sqrt((double)W));
  }
  fill(o.head(), SZ_HEAD, 1.0 / std::sqrt(2.0 * W));
  SCW_HIP(hipMemcpy(n->params.p, p.data(), N_PARAMS * 4, hipMemcpyHostToDevice));
  SCW_HIP(hipMemset(n->adam_m.p, 0, N_PARAMS * 4));
  SCW_HIP(hipMemset(n->adam_v.p, 0, N_PARAMS * 4));
  *out = n.release();
  return SCW_OK;
}

void sur_free(SurNet* n) { delete n; }

int sur_set_params(SurNet& n, const float* host) {
  SCW_HIP(hipMemcpy(n.params.p, host, N_PARAMS * 4, hipMemcpyHostToDevice));
  n.params_version++;
  SCW_HIP(hipMemset(n.adam_m.p, 0, N_PARAMS * 4));
  SCW_HIP(hipMemset(n.adam_v.p, 0, N_PARAMS * 4));
  n.step = 0;
  return SCW_OK;
}

int sur_set_compute(SurNet& n, bool bf16) {
  n.bf16 = bf16;
  return SCW_OK;
}

int sur_get_params(SurNet& n, float* host) {
  SCW_HIP(hipDeviceSynchronize());
  SCW_HIP(hipMemcpy(host, n.params.p, N_PARAMS * 4, hipMemcpyDeviceToHost));
  return SCW_OK;
}

int sur_encode(SurNet& n, const void* n_dev, int B, void* x_dev, hipStream_t s) {
  int rc = check_batch(n, B);
  if (rc) return rc;
  SCW_HIP(sur_encode(reinterpret_cast<const float*>(n_dev), reinterpret_cast<float*>(x_dev), B, s));
  return SCW_OK;
}

int sur_forward(SurNet& n, const void* x_dev, int B, void* out_dev, hipStream_t s) {
  int rc = check_batch(n, B);
  if (rc) return rc;
  if ((rc = infer(n, reinterpret_cast<const float*>(x_dev), B, s))) return rc;
  SCW_HIP(hipMemcpyAsync(out_dev, n.out.p, (size_t)B * OUT * HM * 8, hipMemcpyDeviceToDevice, s));
  return SCW_OK;
}

int sur_loss_grad(SurNet& n, const void* x_dev, const void* tgt_dev, int B, double* loss,
                  float* grad_host, hipStream_t s) {
  int rc = check_batch(n, B);
  if (rc) return rc;
  SCW_HIP(hipMemcpyAsync(n.x.p, x_dev, (size_t)B * CIN * NP * 4, hipMemcpyDeviceToDevice, s));
  if ((rc = forward(n, n.x.as<float>(), B, s, true))) return rc;
  SCW_HIP(sur_loss(n.out.as<float>(), reinterpret_cast<const float*>(tgt_dev),
                   (long long)B * OUT * HM, n.sums.as<float>(), n.gout.as<float>(), s));
  if ((rc = backward(n, B, s))) return rc;
  if (loss) {
    float sums[2];
    SCW_HIP(hipMemcpyAsync(sums, n.sums.p, 8, hipMemcpyDeviceToHost, s));
    SCW_HIP(hipStreamSynchronize(s));
    *loss = (double)sums[0] / (double)sums[1];
  }
  if (grad_host) {
    SCW_HIP(hipMemcpyAsync(grad_host, n.grads.p, N_PARAMS * 4, hipMemcpyDeviceToHost, s));
    SCW_HIP(hipStreamSynchronize(s));
  }
  return SCW_OK;
}

int sur_train_step(SurNet& n, const void* x_dev, const void* tgt_dev, int B, float lr,
                   double* loss, hipStream_t s) {
  int rc = sur_loss_grad(n, x_dev, tgt_dev, B, loss, nullptr, s);
  if (rc) return rc;
  n.step++;
  n.params_version++;
  SCW_HIP(sur_adam(n.params.as<float>(), n.grads.as<float>(), n.adam_m.as<float>(),
                   n.adam_v.as<float>(), N_PARAMS, lr, n.step, s));
  return SCW_OK;
}

// Inference with a sampled CWT check: the surrogate runs on the whole batch;
// n_check seeded patches are also solved by plain CWT (scw_solve_batch); if
// the rel-L2 of the surrogate on them exceeds tol, every patch of the batch
// is solved by CWT and those results are returned instead.
int sur_infer_checked(Context& ctx, SurNet& n, const double* n_host, int B, int n_check,
                      unsigned long long seed, double tol, double* out_host, int* fell_back,
                      double* check_err) {
  int rc = check_batch(n, B);
  if (rc) return rc;
  if (!n_host || !out_host || n_check < 0) return fail(SCW_EINVAL, "null argument");
  const size_t nvox = (size_t)8 * NP;
  std::vector<float> f((size_t)B * nvox * 2);
  for (size_t i = 0; i < f.size(); ++i) f[i] = (float)n_host[i];
  SCW_HIP(hipMemcpy(n.enc_in.p, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  SCW_HIP(sur_encode(n.enc_in.as<float>(), n.x.as<float>(), B, nullptr));
  if ((rc = infer(n, n.x.as<float>(), B, nullptr))) return rc;
  std::vector<float> o((size_t)B * OUT * HM * 2);
  SCW_HIP(hipMemcpy(o.data(), n.out.p, o.size() * 4, hipMemcpyDeviceToHost));
  for (size_t i = 0; i < o.size(); ++i) out_host[i] = o[i];
  std::vector<int> idx(B);
  for (int i = 0; i < B; ++i) idx[i] = i;
  std::mt19937_64 rng(seed);
  std::shuffle(idx.begin(), idx.end(), rng);
  idx.resize(std::min(n_check, B));
  // plain CWT of a set of patches: scw_solve_batch with the device eigensolver
  // and the device elimination, in groups of at most 128 problems
  const size_t per = (size_t)OUT * HM * 2;
  auto solve_set = [&](const std::vector<int>& set, std::vector<double>& res) -> int {
    res.assign(set.size() * per, 0.0);
    constexpr int group = 128;
    for (size_t g0 = 0; g0 < set.size(); g0 += group) {
      const int cnt = (int)std::min<size_t>(group, set.size() - g0);
      std::vector<scw_problem> probs(cnt);
      for (int i = 0; i < cnt; ++i) {
        scw_problem& pr = probs[i];
        pr = scw_problem{};
        pr.nx = pr.ny = 32;
        pr.nz = 8;
        pr.px = pr.py = pr.pz = 0.25;
        pr.n = n_host + (size_t)set[g0 + i] * nvox * 2;
        pr.lambda = 1.0;
        pr.n_top = 1.0;
        pr.n_bot_re = 1.0;
        pr.U = pr.V = HN;
        pr.pw_ex[0] = 1.0;
        pr.route = SCW_ROUTE_STABLE_DEVICE;
        pr.eig = SCW_EIG_DEVICE;
      }
      std::vector<scw_solution*> sols(cnt, nullptr);
      int r = scw_solve_batch(reinterpret_cast<scw_ctx*>(&ctx), probs.data(), cnt, sols.data());
      for (int i = 0; i < cnt && r == SCW_OK; ++i)
        r = scw_solution_exterior(sols[i], nullptr, nullptr, res.data() + (g0 + i) * per);
      for (scw_solution* so : sols)
        if (so) scw_solution_free(so);
      if (r) return r;
    }
    return SCW_OK;
  };
  std::vector<double> ref;
  if ((rc = solve_set(idx, ref))) return rc;
  double num = 0, den = 0;
  for (size_t k = 0; k < idx.size(); ++k)
    for (size_t i = 0; i < per; ++i) {
      const double r = ref[k * per + i];
      const double d = out_host[(size_t)idx[k] * per + i] - r;
      num += d * d;
      den += r * r;
    }
  const double err = den > 0 ? std::sqrt(num / den) : 0.0;
  if (check_err) *check_err = err;
  const bool fb = !idx.empty() && err > tol;
  if (fell_back) *fell_back = fb ? 1 : 0;
  if (fb) {
    std::vector<int> all(B);
    for (int b = 0; b < B; ++b) all[b] = b;
    if ((rc = solve_set(all, ref))) return rc;
    std::copy(ref.begin(), ref.end(), out_host);
  }
  return SCW_OK;
}

}  // namespace scw

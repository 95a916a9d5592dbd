// C ABI of the library (declared in include/scw.h): contexts, the FP64 solve,
// synthesis plans and the synthesis launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <memory>
#include <thread>
#include <cstdio>

#include "scw_internal.h"

namespace scw {

namespace {
thread_local std::string g_err;
}

void set_error(int code, const std::string& msg) {
  g_err = "scw error " + std::to_string(code) + ": " + msg;
}

int fail(int code, const std::string& msg) {
  set_error(code, msg);
  return code;
}

namespace {

int elem_bytes(int precision) { return precision == SCW_FP64 ? 16 : 8; }

// exp(2 pi i * idx / n) with idx reduced modulo n in integers.
zc twiddle_inv(long long idx, int n) {
  long long r = idx % n;
  if (r < 0) r += n;
  const double ang = 2.0 * M_PI * (double)r / (double)n;
  return zc(std::cos(ang), std::sin(ang));
}

template <typename T>
void pack(const std::vector<zc>& in, std::vector<T>& out) {
  out.resize(2 * in.size());
  for (size_t i = 0; i < in.size(); ++i) {
    out[2 * i] = (T)in[i].real();
    out[2 * i + 1] = (T)in[i].imag();
  }
}

int upload(DevBuf& buf, const void* src, size_t bytes) {
  int rc = buf.reserve(std::max<size_t>(bytes, 16));
  if (rc) return rc;
  if (bytes) SCW_HIP(hipMemcpy(buf.p, src, bytes, hipMemcpyHostToDevice));
  return SCW_OK;
}

// Round-to-nearest-even conversions to the 16-bit MFMA operand formats.
uint16_t f32_to_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}
uint16_t f32_to_f16(float x) {
  _Float16 h = (_Float16)x;
  uint16_t b;
  memcpy(&b, &h, 2);
  return b;
}
float f16_to_f32(uint16_t b) {
  _Float16 h;
  memcpy(&h, &b, 2);
  return (float)h;
}

// Twiddle operand of the MFMA y pass: A_re = [Re W, -Im W], A_im = [Im W, Re W]
// with W[g][v] = exp(2 pi i (v - V/2) g / fy), K padded to kp with zeros.
int build_amat(Solution& s, const scw_grid& g, int precision, Plan& pl) {
  const int V = s.V, kp = pl.kp, fy = g.fy;
  std::vector<float> are((size_t)fy * kp, 0.f), aim((size_t)fy * kp, 0.f);
  for (int gg = 0; gg < fy; ++gg)
    for (int v = 0; v < V; ++v) {
      const zc w = twiddle_inv((long long)(v - V / 2) * gg, fy);
      are[(size_t)gg * kp + v] = (float)w.real();
      are[(size_t)gg * kp + V + v] = (float)-w.imag();
      aim[(size_t)gg * kp + v] = (float)w.imag();
      aim[(size_t)gg * kp + V + v] = (float)w.real();
    }
  if (precision == SCW_FP32) {
    std::vector<float> kmaj(2 * (size_t)fy * kp);
    for (int gg = 0; gg < fy; ++gg)
      for (int k = 0; k < kp; ++k) {
        kmaj[(size_t)k * fy + gg] = are[(size_t)gg * kp + k];
        kmaj[((size_t)kp + k) * fy + gg] = aim[(size_t)gg * kp + k];
      }
    return upload(pl.d_amat, kmaj.data(), kmaj.size() * 4);
  }
  const bool bf = precision == SCW_BF16X3;
  std::vector<uint16_t> out(4 * (size_t)fy * kp);
  const std::vector<float>* src[2] = {&are, &aim};
  for (int q = 0; q < 2; ++q)
    for (int gg = 0; gg < fy; ++gg)
      for (int k = 0; k < kp; ++k) {
        const float x = (*src[q])[(size_t)gg * kp + k];
        const uint16_t hi = bf ? f32_to_bf16(x) : f32_to_f16(x);
        const float r = x - (bf ? bf16_to_f32(hi) : f16_to_f32(hi));
        const size_t o = ((size_t)(k / 8) * fy + gg) * 8 + k % 8;
        out[(size_t)(2 * q) * fy * kp + o] = hi;
        out[(size_t)(2 * q + 1) * fy * kp + o] = bf ? f32_to_bf16(r) : f32_to_f16(r);
      }
  return upload(pl.d_amat, out.data(), out.size() * 2);
}

// Plane classification, task grouping and device tables for one grid.
// The configuration a plan is built with: the solution's explicit one, its
// zero fields filled from the context's tuned entry for the same shape.
}  // namespace

scw_synth_config resolve_config(const Context& ctx, const Solution& s, const scw_grid& g,
                                int precision) {
  scw_synth_config c = s.cfg;
  auto it = ctx.tuned_synth.find(synth_key(s, g, precision));
  if (it != ctx.tuned_synth.end()) {
    const scw_synth_config& t = it->second;
    if (!c.modal_rows) c.modal_rows = t.modal_rows;
    if (!c.transform) {
      c.transform = t.transform;
      if (!c.fft_radix) c.fft_radix = t.fft_radix;
      if (!c.tiles) c.tiles = t.tiles;
    }
  }
  return c;
}

namespace {

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// LDS bytes of the factored transform block for radix P (64 columns).
size_t fft_lds_bytes(const Solution& s, const scw_grid& g, int precision, int P) {
  const size_t eb = precision == SCW_FP64 ? 16 : 8;
  return ((size_t)s.U * s.V + 32 * 64 + 32 * (size_t)(g.fy / P)) * eb;
}

}  // namespace

PlaneInfo classify_plane(const scw_grid& g, int L, double d, int j) {
  const double zL = L * d;
  const double dz = (g.z_end - g.z_begin) / g.fz;
  const double z = g.z_begin + (j + 0.5) * dz;
  if (z < 0.0) return {0, -1, z, 0.0};
  if (z >= zL) return {2, L, z - zL, 0.0};
  const int l = std::min((int)std::floor(z / d), L - 1);
  return {1, l, z - l * d, z - (l + 1) * d};
}

PlaneGroups plane_group_shape(const scw_grid& g, int L, double d) {
  // Interior planes of one layer are consecutive (z grows with the index),
  // so runs of equal layer are the per-layer plane counts.
  PlaneGroups r{1, 0, 0};
  int maxc = 0, run = 0, prev = -1;
  for (int j = 0; j < g.fz; ++j) {
    const PlaneInfo pi = classify_plane(g, L, d, j);
    if (pi.kind != 1) {
      ++r.n_ext;
      run = 0;
      prev = -1;
      continue;
    }
    run = pi.layer == prev ? run + 1 : 1;
    prev = pi.layer;
    maxc = std::max(maxc, run);
  }
  while (r.zt < std::min(maxc, 8)) r.zt *= 2;
  run = 0;
  prev = -1;
  for (int j = 0; j < g.fz; ++j) {
    const PlaneInfo pi = classify_plane(g, L, d, j);
    if (pi.kind != 1) {
      prev = -1;
      continue;
    }
    run = pi.layer == prev ? run + 1 : 0;
    prev = pi.layer;
    if (run % r.zt == 0) ++r.ntasks;
  }
  return r;
}

int choose_shape(const Solution& s, const scw_grid& g, int precision,
                 const scw_synth_config& cfg, int zt, KernelShape* out) {
  const bool split = precision == SCW_BF16X3 || precision == SCW_FP16X3;
  if (cfg.transform < SCW_XFORM_AUTO || cfg.transform > SCW_XFORM_DIRECT)
    return fail(SCW_EINVAL, "unknown transform kind " + std::to_string(cfg.transform));
  if (cfg.modal_rows && !(is_pow2(cfg.modal_rows) && cfg.modal_rows >= 2 && cfg.modal_rows <= 16))
    return fail(SCW_EINVAL, "modal_rows must be 2, 4, 8 or 16");
  if (cfg.tiles < 0 || cfg.tiles > 4096) return fail(SCW_EINVAL, "tiles out of range");
  // FP32 modal sum: rows per wave, so that rows x planes stays <= 32
  int rw = cfg.modal_rows ? cfg.modal_rows : (zt >= 8 ? 4 : (zt == 4 ? 8 : 16));
  while (rw > 2 && rw * zt > 32) rw /= 2;
  out->modal_rw = rw;
  out->tiles = cfg.tiles;
  // factored y pass: fy = R * P, P <= 32 a power of two, spectra V <= 32 rows
  const int p_default = std::min(32, std::max(2, g.fy / 16));
  const int P = cfg.fft_radix ? cfg.fft_radix : p_default;
  const bool fft_ok = !split && s.V <= 32 && g.fy >= 2 && is_pow2(g.fy) && is_pow2(P) &&
                      P >= 2 && P <= 32 && P <= g.fy &&
                      fft_lds_bytes(s, g, precision, P) <= 64 * 1024;
  int kind = cfg.transform;
  if (kind == SCW_XFORM_AUTO)
    kind = split ? SCW_XFORM_MFMA
                 : (fft_ok ? SCW_XFORM_FFT
                           : (precision == SCW_FP32 && s.V <= 32 ? SCW_XFORM_MFMA
                                                                 : SCW_XFORM_DIRECT));
  if (split && kind != SCW_XFORM_MFMA)
    return fail(SCW_EINVAL, "split-precision synthesis evaluates the transform on the matrix cores");
  if (kind == SCW_XFORM_FFT && !fft_ok)
    return fail(SCW_EINVAL, "factored transform needs FP64/FP32, V <= 32, fy a power of two and "
                            "a radix P (2..32, power of two) whose tables fit in 64 KB of LDS");
  if (kind == SCW_XFORM_FFT && cfg.tiles != 0 && cfg.tiles != 32 && cfg.tiles != 64)
    return fail(SCW_EINVAL, "factored transform takes 32 or 64 columns per block (tiles)");
  if (kind == SCW_XFORM_MFMA && (precision == SCW_FP64 || s.V > 32))
    return fail(SCW_EINVAL, "matrix-core transform needs FP32 or split precision and V <= 32");
  out->kind = kind;
  out->fft_p = kind == SCW_XFORM_FFT ? P : 0;
  out->fft_ok = fft_ok;
  return SCW_OK;
}

namespace {

int build_plan(Solution& s, Plan& pl, const scw_grid& g, int precision,
               const scw_synth_config& cfg, bool direct_only) {
  pl.valid = false;
  pl.direct_only = direct_only;
  pl.grid = g;
  pl.precision = precision;
  pl.planes.assign(g.fz, PlaneInfo{});
  std::vector<ExtPlane> ext;
  for (int j = 0; j < g.fz; ++j) {
    PlaneInfo& pi = pl.planes[j];
    pi = classify_plane(g, s.L, s.d, j);
    if (pi.kind != 1) ext.push_back({j, pi.kind, pi.dz_top});
  }
  const int zt = plane_group_shape(g, s.L, s.d).zt;
  pl.zt = zt;
  pl.tasks.clear();
  std::vector<double> tdz;
  for (int j = 0; j < g.fz;) {
    if (pl.planes[j].kind != 1) {
      ++j;
      continue;
    }
    const int l = pl.planes[j].layer;
    Task t{l, j, 0, 0};
    while (j < g.fz && t.count < zt && pl.planes[j].kind == 1 && pl.planes[j].layer == l) {
      tdz.push_back(pl.planes[j].dz_top);
      tdz.push_back(pl.planes[j].dz_bot);
      ++t.count;
      ++j;
    }
    for (int p = t.count; p < zt; ++p) {  // padding planes: zero offsets
      tdz.push_back(0.0);
      tdz.push_back(0.0);
    }
    pl.tasks.push_back(t);
  }
  pl.n_exterior = (int)ext.size();
  int rc;
  std::vector<float> tdz32(tdz.begin(), tdz.end());
  if ((rc = upload(pl.d_tasks, pl.tasks.data(), pl.tasks.size() * sizeof(Task))) ||
      (rc = upload(pl.d_task_dz, tdz.data(), tdz.size() * sizeof(double))) ||
      (rc = upload(pl.d_task_dz32, tdz32.data(), tdz32.size() * sizeof(float))) ||
      (rc = upload(pl.d_ext, ext.data(), ext.size() * sizeof(ExtPlane))))
    return rc;
  const int eb = elem_bytes(precision);
  const size_t n2 = 2 * (size_t)s.M;
  if ((rc = pl.d_w.reserve(std::max<size_t>(16, pl.tasks.size() * 2 * zt * n2 * eb))) ||
      (rc = pl.d_spec.reserve((size_t)g.fz * 3 * s.M * eb)))
    return rc;
  // inverse-transform factors: wx[0][f] = e^{2 pi i f/fx}, wx[1][f] = e^{-2 pi i (U/2) f/fx}
  std::vector<zc> twx(2 * (size_t)g.fx), twy(2 * (size_t)g.fy);
  for (int f = 0; f < g.fx; ++f) {
    twx[f] = twiddle_inv(f, g.fx);
    twx[g.fx + f] = twiddle_inv(-(long long)(s.U / 2) * f, g.fx);
  }
  for (int gg = 0; gg < g.fy; ++gg) {
    twy[gg] = twiddle_inv(gg, g.fy);
    twy[g.fy + gg] = twiddle_inv(-(long long)(s.V / 2) * gg, g.fy);
  }
  if (precision == SCW_FP64) {
    std::vector<double> a, b;
    pack(twx, a);
    pack(twy, b);
    if ((rc = upload(pl.d_twx, a.data(), a.size() * 8)) ||
        (rc = upload(pl.d_twy, b.data(), b.size() * 8)))
      return rc;
  } else {
    std::vector<float> a, b;
    pack(twx, a);
    pack(twy, b);
    if ((rc = upload(pl.d_twx, a.data(), a.size() * 4)) ||
        (rc = upload(pl.d_twy, b.data(), b.size() * 4)))
      return rc;
  }
  // kernel configuration: explicit, tuned, or the built-in default
  pl.cfg = cfg;
  KernelShape ks;
  if ((rc = choose_shape(s, g, precision, cfg, pl.zt, &ks))) return rc;
  pl.modal_rw = ks.modal_rw;
  pl.tiles = ks.tiles;
  const int kind = ks.kind, P = ks.fft_p;
  pl.fft_p = 0;
  pl.mfma = false;
  if (kind == SCW_XFORM_FFT) {
    const int R = g.fy / P;
    pl.fft_p = P;
    std::vector<zc> tw(32 * (size_t)R);
    for (int g1 = 0; g1 < R; ++g1)  // [R][32]: e^{2 pi i (slot - 16) g1 / fy}
      for (int sl = 0; sl < 32; ++sl)
        tw[(size_t)g1 * 32 + sl] = twiddle_inv((long long)(sl - 16) * g1, g.fy);
    if (precision == SCW_FP64) {
      std::vector<double> b;
      pack(tw, b);
      if ((rc = upload(pl.d_fft_tw, b.data(), b.size() * 8))) return rc;
    } else {
      std::vector<float> b;
      pack(tw, b);
      if ((rc = upload(pl.d_fft_tw, b.data(), b.size() * 4))) return rc;
    }
  } else if (kind == SCW_XFORM_MFMA) {
    pl.mfma = true;
    const int ks = mfma_kstep(precision);
    pl.kp = ((2 * s.V + ks - 1) / ks) * ks;
    if ((rc = build_amat(s, g, precision, pl))) return rc;
    const size_t ebyte = 4;  // f32, or hi + lo 16-bit
    if ((rc = pl.d_bmat.reserve((size_t)g.fz * 3 * pl.kp * g.fx * ebyte)) ||
        (rc = pl.d_bscale.reserve((size_t)g.fz * 3 * sizeof(float))))
      return rc;
  }
  pl.valid = true;
  return SCW_OK;
}

bool same_grid(const scw_grid& a, const scw_grid& b) {
  return a.fx == b.fx && a.fy == b.fy && a.fz == b.fz && a.z_begin == b.z_begin &&
         a.z_end == b.z_end;
}


}  // namespace

int check_grid(const scw_grid* g) {
  if (!g) return fail(SCW_EINVAL, "grid is null");
  if (g->fx < 1 || g->fy < 1 || g->fz < 1)
    return fail(SCW_EINVAL, "grid sizes must be positive");
  if ((long long)g->fz * 3 > 65535) return fail(SCW_EINVAL, "fz above 21845");
  if ((long long)g->fy > 65535 * 8LL) return fail(SCW_EINVAL, "fy too large");
  if (!(g->z_end > g->z_begin)) return fail(SCW_EINVAL, "z_end must exceed z_begin");
  return SCW_OK;
}

}  // namespace scw

using namespace scw;

extern "C" {

const char* scw_last_error(void) { return g_err.c_str(); }

int scw_create(scw_ctx** out, int hip_device, int host_threads) {
  if (!out) return fail(SCW_EINVAL, "out is null");
  *out = nullptr;
  int ndev = 0;
  SCW_HIP(hipGetDeviceCount(&ndev));
  if (hip_device < 0 || hip_device >= ndev)
    return fail(SCW_EINVAL, "no HIP device " + std::to_string(hip_device));
  scw_ctx* c = new (std::nothrow) scw_ctx();
  if (!c) return fail(SCW_ENOMEM, "context allocation failed");
  c->c.device = hip_device;
  unsigned hw = std::thread::hardware_concurrency();
  c->c.host_threads = host_threads > 0 ? host_threads : (int)std::max(1u, hw);
  if (hipSetDevice(hip_device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->c.setup_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(SCW_EHIP, "could not create the setup stream");
  }
  int rc = noalloc_attach(hip_device);  // the device's scratch array, with the device current
  if (rc) {
    (void)hipStreamDestroy(c->c.setup_stream);
    delete c;
    return rc;
  }
  *out = c;
  return SCW_OK;
}

static void profile_free(scw::Context& c);

void scw_destroy(scw_ctx* ctx) {
  if (!ctx) return;
  profile_free(ctx->c);
  release_blas(ctx->c);
  if (ctx->c.setup_stream) (void)hipStreamDestroy(ctx->c.setup_stream);
  delete ctx;
}

static int solve_into(scw_ctx* ctx, const scw_problem* prob, int n_waves,
                      const scw_plane_wave* waves, scw_solution** out) {
  if (!ctx || !prob || !out) return fail(SCW_EINVAL, "null argument");
  *out = nullptr;
  scw_solution* sol = new (std::nothrow) scw_solution();
  if (!sol) return fail(SCW_ENOMEM, "solution allocation failed");
  int rc;
  try {
    rc = solve_problem(ctx->c, *prob, sol->s, n_waves, waves);
  } catch (const std::bad_alloc&) {
    rc = fail(SCW_ENOMEM, "host allocation failed during setup");
  } catch (const std::exception& e) {
    rc = fail(SCW_EINVAL, std::string("setup failed: ") + e.what());
  }
  if (rc) {
    delete sol;
    return rc;
  }
  *out = sol;
  return SCW_OK;
}

int scw_solve(scw_ctx* ctx, const scw_problem* prob, scw_solution** out) {
  return solve_into(ctx, prob, 0, nullptr, out);
}

int scw_solve_batch(scw_ctx* ctx, const scw_problem* probs, int n, scw_solution** out) {
  if (!ctx || !probs || !out || n < 1) return fail(SCW_EINVAL, "null argument or n < 1");
  for (int i = 0; i < n; ++i) out[i] = nullptr;
  std::vector<scw_solution*> made(n, nullptr);
  std::vector<Solution*> sols(n, nullptr);
  for (int i = 0; i < n; ++i) {
    made[i] = new (std::nothrow) scw_solution();
    if (!made[i]) {
      for (scw_solution* m : made) delete m;
      return fail(SCW_ENOMEM, "solution allocation failed");
    }
    sols[i] = &made[i]->s;
  }
  const int rc = solve_problems(ctx->c, probs, n, sols.data());
  if (rc) {
    for (scw_solution* m : made) delete m;
    return rc;
  }
  for (int i = 0; i < n; ++i) out[i] = made[i];
  return SCW_OK;
}

int scw_solve_illuminations(scw_ctx* ctx, const scw_problem* prob, int n_waves,
                            const scw_plane_wave* waves, scw_solution** out) {
  if (n_waves < 1 || n_waves > 4096 || !waves)
    return fail(SCW_EINVAL, "n_waves must be 1..4096 with a non-null list");
  return solve_into(ctx, prob, n_waves, waves, out);
}

int scw_synthesize_illuminations(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid,
                                 int precision, void* E_dev, void* hip_stream) {
  if (!ctx || !sol || !E_dev) return fail(SCW_EINVAL, "null argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision != SCW_FP32)
    return fail(SCW_EINVAL, "illuminations are synthesized in SCW_FP32");
  return synthesize_illuminations(ctx->c, sol->s, *grid, E_dev,
                                  reinterpret_cast<hipStream_t>(hip_stream));
}

void scw_solution_free(scw_solution* sol) { delete sol; }

int scw_solution_info_get(const scw_solution* sol, scw_solution_info* info) {
  if (!sol || !info) return fail(SCW_EINVAL, "null argument");
  *info = sol->s.info;
  return SCW_OK;
}

int scw_solution_exterior(const scw_solution* sol, double* p_inc, double* p_ref,
                          double* p_trn) {
  if (!sol) return fail(SCW_EINVAL, "null solution");
  const Solution& s = sol->s;
  const size_t n = 3 * (size_t)s.M;
  // illumination 0 (the first 3M of each)
  if (p_inc) std::copy(s.p_inc.begin(), s.p_inc.begin() + n, reinterpret_cast<zc*>(p_inc));
  if (p_ref) std::copy(s.p_ref.begin(), s.p_ref.begin() + n, reinterpret_cast<zc*>(p_ref));
  if (p_trn) std::copy(s.p_trn.begin(), s.p_trn.begin() + n, reinterpret_cast<zc*>(p_trn));
  return SCW_OK;
}

}  // extern "C"

namespace scw {

std::string synth_key(const Solution& s, const scw_grid& g, int precision) {
  char buf[160];
  snprintf(buf, sizeof buf, "p%d U%d V%d L%d d%.17g fx%d fy%d fz%d z%.17g:%.17g", precision,
           s.U, s.V, s.L, s.d, g.fx, g.fy, g.fz, g.z_begin, g.z_end);
  return buf;
}

static bool same_config(const scw_synth_config& a, const scw_synth_config& b) {
  return a.modal_rows == b.modal_rows && a.transform == b.transform &&
         a.fft_radix == b.fft_radix && a.tiles == b.tiles;
}

int get_plan(Context& c, Solution& s, const scw_grid& g, int precision, bool direct_only,
             Plan** out) {
  if (s.device != c.device) return fail(SCW_EINVAL, "solution belongs to another device");
  SCW_HIP(hipSetDevice(c.device));
  if (precision != SCW_FP64 && !s.d_P32.p)
    return fail(SCW_EINVAL, "solution has no FP32 synthesis matrices");
  scw_synth_config cfg = resolve_config(c, s, g, precision);
  if (direct_only) cfg = scw_synth_config{cfg.modal_rows, SCW_XFORM_DIRECT, 0, 0};
  for (auto& p : s.plans)
    if (p->valid && p->precision == precision && p->direct_only == direct_only &&
        same_grid(p->grid, g) && same_config(p->cfg, cfg)) {
      *out = p.get();
      return SCW_OK;
    }
  // A new plan: fresh buffers, so work in flight on older plans is untouched;
  // its tables are uploaded synchronously before any kernel can read them.
  std::unique_ptr<Plan> pl(new (std::nothrow) Plan());
  if (!pl) return fail(SCW_ENOMEM, "plan allocation failed");
  int rc = build_plan(s, *pl, g, precision, cfg, direct_only);
  if (rc) return rc;
  s.plans.push_back(std::move(pl));
  *out = s.plans.back().get();
  return SCW_OK;
}

static SynthArgs synth_args(const Solution& s, const Plan& pl, const scw_grid& g, int precision,
                            void* E, int stages) {
  SynthArgs a{};
  a.M = s.M;
  a.U = s.U;
  a.V = s.V;
  a.L = s.L;
  a.fx = g.fx;
  a.fy = g.fy;
  a.fz = g.fz;
  a.zt = pl.zt;
  a.ntasks = (int)pl.tasks.size();
  a.n_ext = pl.n_exterior;
  a.P = precision == SCW_FP64 ? s.d_P64.p : s.d_P32.p;
  a.kg = s.d_kg.as<double>();
  a.a = s.d_a.as<double>();
  a.b = s.d_b.as<double>();
  a.ext = s.d_ext.as<double>();
  a.ksz = s.d_ksz.as<double>();
  a.tasks = pl.d_tasks.as<Task>();
  a.task_dz = pl.d_task_dz.as<double>();
  a.ext_planes = pl.d_ext.p;
  a.w = pl.d_w.p;
  a.spec = pl.d_spec.p;
  a.twx = pl.d_twx.p;
  a.twy = pl.d_twy.p;
  a.E = E;
  a.kgab32 = s.d_kgab32.p;
  a.task_dz32 = pl.d_task_dz32.p;
  a.precision = precision;
  a.mfma = pl.mfma;
  a.kp = pl.kp;
  a.fft_p = pl.fft_p;
  a.fft_tw = pl.d_fft_tw.p;
  a.bmat = pl.d_bmat.p;
  a.bscale = pl.d_bscale.as<float>();
  a.amat = pl.d_amat.p;
  a.idft_gtiles = pl.tiles;
  a.modal_rw = pl.modal_rw;
  a.stages = stages;
  return a;
}

int synthesize(Context& c, Solution& s, const scw_grid& g, int precision, void* E,
               hipStream_t st, int stages, hipEvent_t* ev, bool direct_only, Plan** used) {
  Plan* pl = nullptr;
  int rc = get_plan(c, s, g, precision, direct_only, &pl);
  if (rc) return rc;
  if (used) *used = pl;
  const SynthArgs a = synth_args(s, *pl, g, precision, E, stages);
  SCW_HIP(precision == SCW_FP64 ? launch_synthesis_fp64(a, st, ev)
                                : launch_synthesis_fp32(a, st, ev));
  return SCW_OK;
}

// Every illumination of a solution: the modal sum of up to 32 / zt
// illuminations per launch on the matrix cores, then each illumination's
// exterior planes and transform into its block of E.
int synthesize_illuminations(Context& c, Solution& s, const scw_grid& g, void* E,
                             hipStream_t st) {
  Plan* plp = nullptr;
  int rc = get_plan(c, s, g, SCW_FP32, false, &plp);
  if (rc) return rc;
  Plan& pl = *plp;
  const size_t per = (size_t)g.fz * 3 * s.M;
  // sized once per plan (K is fixed for a solution): never reallocated
  if (!pl.d_spec_multi.p && (rc = pl.d_spec_multi.reserve(per * s.K * 8))) return rc;
  const size_t wb = multi_table_bytes((int)pl.tasks.size(), s.M);
  if (!pl.d_wmulti.p && (rc = pl.d_wmulti.reserve(wb))) return rc;
  const size_t lm = (size_t)s.L * 2 * s.M;  // complex per [L][2M] block
  // with one illumination, (a, b) are the last two blocks of k*gamma, a, b
  const void* ab = s.K > 1 ? s.d_ab32.p : (const void*)(s.d_kgab32.as<float>() + 2 * lm);
  const int group = 32 / pl.zt;
  for (int k0 = 0; k0 < s.K && !pl.tasks.empty(); k0 += group)
    SCW_HIP(launch_modal_multi(s.d_P32.p, s.d_kgab32.p, ab, pl.d_tasks.as<Task>(),
                               pl.d_task_dz32.p, (int)pl.tasks.size(), pl.zt, s.M, s.L, g.fz,
                               k0, std::min(group, s.K - k0), pl.d_wmulti.p,
                               pl.d_spec_multi.p, st));
  const size_t vol = (size_t)3 * g.fz * g.fy * g.fx;
  for (int k = 0; k < s.K; ++k) {
    SynthArgs a = synth_args(s, pl, g, SCW_FP32, static_cast<char*>(E) + k * vol * 8,
                             kStageExterior | kStageTransform);
    a.ext = s.d_ext.as<double>() + (size_t)k * 9 * s.M * 2;
    a.spec = pl.d_spec_multi.as<char>() + k * per * 8;
    SCW_HIP(launch_synthesis_fp32(a, st, nullptr));
  }
  return SCW_OK;
}

}  // namespace scw

extern "C" {

int scw_synthesize(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                   void* E_dev, void* hip_stream) {
  if (!ctx || !sol || !E_dev) return fail(SCW_EINVAL, "null argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision < SCW_FP64 || precision > SCW_FP16X3)
    return fail(SCW_EINVAL, "unknown precision " + std::to_string(precision));
  if ((precision == SCW_BF16X3 || precision == SCW_FP16X3) && sol->s.V > 32)
    return fail(SCW_EINVAL, "split-precision transform needs V <= 32");
  hipEvent_t* ev = nullptr;
  Context& c = ctx->c;
  if (c.prof_used < c.prof_max) ev = c.prof_events.data() + (size_t)c.prof_used++ * (kNumStages + 1);
  return synthesize(c, sol->s, *grid, precision, E_dev, reinterpret_cast<hipStream_t>(hip_stream),
                    kStageAll, ev);
}

int scw_synthesize_stages(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                          int stages, void* E_dev, void* hip_stream) {
  if (!ctx || !sol) return fail(SCW_EINVAL, "null argument");
  if (stages < 1 || stages > SCW_STAGE_ALL)
    return fail(SCW_EINVAL, "stage mask must be in 1..7");
  if ((stages & SCW_STAGE_TRANSFORM) && !E_dev) return fail(SCW_EINVAL, "null output");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision < SCW_FP64 || precision > SCW_FP16X3)
    return fail(SCW_EINVAL, "unknown precision " + std::to_string(precision));
  if ((precision == SCW_BF16X3 || precision == SCW_FP16X3) && sol->s.V > 32)
    return fail(SCW_EINVAL, "split-precision transform needs V <= 32");
  static_assert(SCW_STAGE_MODAL == kStageModal && SCW_STAGE_EXTERIOR == kStageExterior &&
                    SCW_STAGE_TRANSFORM == kStageTransform && SCW_STAGE_ALL == kStageAll,
                "public and internal stage masks agree");
  return synthesize(ctx->c, sol->s, *grid, precision, E_dev,
                    reinterpret_cast<hipStream_t>(hip_stream), stages, nullptr);
}

// One period of sol's field into its plan's tile workspace, then placed.
static int synthesize_placed(Context& c, Solution& s, const scw_grid& g, int precision, void* E,
                             int dfx, int dfy, int ox, int oy, int rx, int ry, hipStream_t st) {
  Plan* pl = nullptr;
  int rc = get_plan(c, s, g, precision, false, &pl);
  if (rc) return rc;
  const size_t eb = precision == SCW_FP64 ? 16 : 8;
  const size_t bytes = (size_t)3 * g.fz * g.fy * g.fx * eb;
  if (pl->d_tile.bytes < bytes && (rc = pl->d_tile.reserve(bytes))) return rc;
  if ((rc = synthesize(c, s, g, precision, pl->d_tile.p, st, kStageAll, nullptr))) return rc;
  SCW_HIP(launch_place(pl->d_tile.p, g.fx, g.fy, g.fz, E, dfx, dfy, ox, oy, rx, ry,
                       precision == SCW_FP64, st));
  return SCW_OK;
}

int scw_synthesize_tiled(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int tx, int ty,
                         int precision, void* E_dev, void* hip_stream) {
  if (!ctx || !sol || !E_dev) return fail(SCW_EINVAL, "null argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision < SCW_FP64 || precision > SCW_FP16X3)
    return fail(SCW_EINVAL, "unknown precision " + std::to_string(precision));
  if (tx < 1 || ty < 1 || (long long)tx * grid->fx > (1LL << 30) ||
      (long long)ty * grid->fy > (1LL << 30))
    return fail(SCW_EINVAL, "tile counts must be positive");
  return synthesize_placed(ctx->c, sol->s, *grid, precision, E_dev, tx * grid->fx,
                           ty * grid->fy, 0, 0, tx, ty, reinterpret_cast<hipStream_t>(hip_stream));
}

int scw_synthesize_composed(scw_ctx* ctx, scw_solution* const* patches, int px, int py,
                            const scw_grid* grid, int precision, void* E_dev, void* hip_stream) {
  if (!ctx || !patches || !E_dev) return fail(SCW_EINVAL, "null argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision < SCW_FP64 || precision > SCW_FP16X3)
    return fail(SCW_EINVAL, "unknown precision " + std::to_string(precision));
  if (px < 1 || py < 1 || (long long)px * grid->fx > (1LL << 30) ||
      (long long)py * grid->fy > (1LL << 30))
    return fail(SCW_EINVAL, "patch counts must be positive");
  for (int i = 0; i < px * py; ++i)
    if (!patches[i]) return fail(SCW_EINVAL, "null patch " + std::to_string(i));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  for (int j = 0; j < py; ++j)
    for (int i = 0; i < px; ++i)
      if ((rc = synthesize_placed(ctx->c, patches[j * px + i]->s, *grid, precision, E_dev,
                                  px * grid->fx, py * grid->fy, i * grid->fx, j * grid->fy, 1, 1,
                                  st)))
        return rc;
  return SCW_OK;
}

int scw_synthesize_slice(scw_ctx* ctx, scw_solution* sol, const scw_slice* slice, int precision,
                         void* E_dev, void* hip_stream) {
  if (!ctx || !sol || !slice || !E_dev) return fail(SCW_EINVAL, "null argument");
  if (slice->axis != SCW_SLICE_XZ && slice->axis != SCW_SLICE_YZ)
    return fail(SCW_EINVAL, "slice axis must be SCW_SLICE_XZ or SCW_SLICE_YZ");
  if (precision != SCW_FP64 && precision != SCW_FP32)
    return fail(SCW_EINVAL, "a slice is synthesized in SCW_FP64 or SCW_FP32");
  if (!std::isfinite(slice->position)) return fail(SCW_EINVAL, "slice position is not finite");
  // the planes and lateral tables of an n x n grid; only its spectra are formed
  const scw_grid g{slice->n, slice->n, slice->fz, slice->z_begin, slice->z_end};
  int rc = check_grid(&g);
  if (rc) return rc;
  Solution& s = sol->s;
  const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  Plan* plp = nullptr;
  if ((rc = synthesize(ctx->c, s, g, precision, nullptr, st, kStageModal | kStageExterior,
                       nullptr, true, &plp)))
    return rc;
  const Plan& pl = *plp;
  SliceArgs a{};
  a.spec = pl.d_spec.p;
  a.tw = slice->axis == SCW_SLICE_XZ ? pl.d_twx.p : pl.d_twy.p;
  a.U = s.U;
  a.V = s.V;
  a.n = slice->n;
  a.fz = slice->fz;
  a.axis = slice->axis;
  a.frac = slice->axis == SCW_SLICE_XZ ? slice->position / s.Y : slice->position / s.X;
  a.E = E_dev;
  SCW_HIP(launch_slice(a, precision == SCW_FP64, st));
  return SCW_OK;
}

// The spectra of the grid's planes, `op` on them, then Eq. 10 and (when I_dev
// is not null) the intensity.
static int synthesize_with(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                           void* E_dev, void* I_dev, void* hip_stream,
                           const std::function<hipError_t(Solution&, Plan&, hipStream_t)>& op) {
  if (!ctx || !sol || !E_dev) return fail(SCW_EINVAL, "null argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision < SCW_FP64 || precision > SCW_FP16X3)
    return fail(SCW_EINVAL, "unknown precision " + std::to_string(precision));
  if ((precision == SCW_BF16X3 || precision == SCW_FP16X3) && sol->s.V > 32)
    return fail(SCW_EINVAL, "split-precision transform needs V <= 32");
  Context& c = ctx->c;
  Solution& s = sol->s;
  const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  Plan* pl = nullptr;
  if ((rc = synthesize(c, s, *grid, precision, E_dev, st, kStageModal | kStageExterior, nullptr,
                       false, &pl)))
    return rc;
  SCW_HIP(op(s, *pl, st));
  if ((rc = synthesize(c, s, *grid, precision, E_dev, st, kStageTransform, nullptr))) return rc;
  if (I_dev)
    SCW_HIP(launch_intensity(E_dev, I_dev, (long long)grid->fz * grid->fy * grid->fx,
                             precision == SCW_FP64, st));
  return SCW_OK;
}

int scw_synthesize_image(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                         double na, void* E_dev, void* I_dev, void* hip_stream) {
  if (!(na >= 0.0) || !std::isfinite(na)) return fail(SCW_EINVAL, "na must be finite and >= 0");
  return synthesize_with(ctx, sol, grid, precision, E_dev, I_dev, hip_stream,
                         [&](Solution& s, Plan& pl, hipStream_t st) {
                           return launch_objective(pl.d_spec.p,
                                                   (long long)grid->fz * 3 * s.M, s.M, s.U, s.V,
                                                   s.lam / s.X, s.lam / s.Y, na,
                                                   precision == SCW_FP64, st);
                         });
}

int scw_synthesize_filtered(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                            const void* H_dev, void* E_dev, void* I_dev, void* hip_stream) {
  if (!H_dev) return fail(SCW_EINVAL, "null transfer function");
  return synthesize_with(ctx, sol, grid, precision, E_dev, I_dev, hip_stream,
                         [&](Solution& s, Plan& pl, hipStream_t st) {
                           return launch_transfer(pl.d_spec.p,
                                                  (long long)grid->fz * 3 * s.M, s.M, H_dev,
                                                  precision == SCW_FP64, st);
                         });
}

int scw_synthesis_configure(scw_solution* sol, const scw_synth_config* cfg) {
  if (!sol) return fail(SCW_EINVAL, "null solution");
  sol->s.cfg = cfg ? *cfg : scw_synth_config{};
  return SCW_OK;
}

static void profile_free(Context& c) {
  for (hipEvent_t e : c.prof_events) (void)hipEventDestroy(e);
  c.prof_events.clear();
  c.prof_max = c.prof_used = 0;
}

int scw_profile_begin(scw_ctx* ctx, int max_calls) {
  if (!ctx || max_calls < 1 || max_calls > 100000) return fail(SCW_EINVAL, "bad profile request");
  Context& c = ctx->c;
  SCW_HIP(hipSetDevice(c.device));
  profile_free(c);
  c.prof_events.resize((size_t)max_calls * (kNumStages + 1));
  for (auto& e : c.prof_events) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      profile_free(c);
      return fail(SCW_EHIP, "hipEventCreate failed");
    }
  }
  c.prof_max = max_calls;
  c.prof_used = 0;
  return SCW_OK;
}

int scw_profile_end(scw_ctx* ctx, double* stage_ms, int n_stages, int* calls) {
  if (!ctx || !stage_ms || n_stages < 1 || n_stages > 8) return fail(SCW_EINVAL, "bad profile query");
  Context& c = ctx->c;
  SCW_HIP(hipSetDevice(c.device));
  std::vector<double> acc(kNumStages, 0.0);
  for (int k = 0; k < c.prof_used; ++k) {
    hipEvent_t* ev = c.prof_events.data() + (size_t)k * (kNumStages + 1);
    SCW_HIP(hipEventSynchronize(ev[kNumStages]));
    for (int i = 0; i < kNumStages; ++i) {
      float ms = 0;
      SCW_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      acc[i] += ms;
    }
  }
  for (int i = 0; i < n_stages; ++i)
    stage_ms[i] = (i < kNumStages && c.prof_used) ? acc[i] / c.prof_used : 0.0;
  if (calls) *calls = c.prof_used;
  profile_free(c);
  return SCW_OK;
}

const char* scw_stage_name(int stage) {
  static const char* names[kNumStages] = {"phase", "modal_sum", "exterior", "idft"};
  return (stage >= 0 && stage < kNumStages) ? names[stage] : "";
}

int scw_field(scw_ctx* ctx, const scw_problem* prob, const scw_grid* grid, int precision,
              void* E_dev, void* hip_stream) {
  scw_solution* sol = nullptr;
  int rc = scw_solve(ctx, prob, &sol);
  if (rc) return rc;
  rc = scw_synthesize(ctx, sol, grid, precision, E_dev, hip_stream);
  if (rc == SCW_OK && hipStreamSynchronize(reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
    rc = fail(SCW_EHIP, "stream synchronize failed");
  scw_solution_free(sol);
  return rc;
}

double scw_synthesis_bytes(const scw_solution* sol, const scw_grid* grid, int precision) {
  if (!sol || !grid || grid->fz < 1) return 0.0;
  const Solution& s = sol->s;
  const double eb = precision == SCW_FP64 ? 16.0 : 8.0;
  const double zL = s.L * s.d;
  const double dz = (grid->z_end - grid->z_begin) / grid->fz;
  std::vector<char> touched(s.L, 0);
  for (int j = 0; j < grid->fz; ++j) {
    const double z = grid->z_begin + (j + 0.5) * dz;
    if (z >= 0.0 && z < zL) touched[std::min((int)std::floor(z / s.d), s.L - 1)] = 1;
  }
  double layers = 0;
  for (char t : touched) layers += t;
  const double pbytes = layers * 3.0 * s.M * 2.0 * s.M * eb;
  const double ebytes = 3.0 * grid->fx * grid->fy * grid->fz * eb;
  return pbytes + ebytes;
}

}  // extern "C"

namespace scw {

std::string batch_key(const scw_grid& g) {
  char buf[96];
  snprintf(buf, sizeof buf, "fx%d fy%d fz%d", g.fx, g.fy, g.fz);
  return buf;
}

int batch_set_shape(scw_batch* b, int P, int blocks_per_cu, int chunk) {
  const int fy = b->grid.fy;
  if (!is_pow2(P) || P < 2 || P > 32 || P > fy || fy % P != 0)
    return fail(SCW_EINVAL, "batch radix must be a power of two in [2, min(32, fy)]");
  const int R = fy / P;
  if ((32 * (size_t)R + 3 * (size_t)b->mmax) * 8 > 48 * 1024)
    return fail(SCW_EINVAL, "batch radix too small for fy");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(SCW_EINVAL, "blocks per CU out of range");
  if (chunk < 1 || chunk > 1024) return fail(SCW_EINVAL, "items per grab out of range");
  std::vector<float> wfull(2 * (size_t)b->grid.fx), tw(2 * (32 * (size_t)R));
  for (int k = 0; k < b->grid.fx; ++k) {
    const zc w = twiddle_inv(k, b->grid.fx);
    wfull[2 * k] = (float)w.real();
    wfull[2 * k + 1] = (float)w.imag();
  }
  for (int g1 = 0; g1 < R; ++g1)  // [R][32]: e^{2 pi i (slot - 16) g1 / fy}
    for (int sl = 0; sl < 32; ++sl) {
      const zc w = twiddle_inv((long long)(sl - 16) * g1, fy);
      tw[2 * ((size_t)g1 * 32 + sl)] = (float)w.real();
      tw[2 * ((size_t)g1 * 32 + sl) + 1] = (float)w.imag();
    }
  int rc;
  if ((rc = upload(b->d_wfull, wfull.data(), wfull.size() * 4)) ||
      (rc = upload(b->d_tw, tw.data(), tw.size() * 4)))
    return rc;
  b->P = P;
  b->chunk = chunk;
  b->grid_blocks = std::max(1, std::min(b->n_items, b->cus * blocks_per_cu));
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  b->graph_E = nullptr;
  return SCW_OK;
}

BatchArgs batch_args(const scw_batch* b, void* E) {
  BatchArgs a{};
  a.jobs = b->d_jobs.as<BatchJob>();
  a.items = b->d_items.as<BatchItem>();
  a.n_items = b->n_items;
  a.planes = b->d_planes.as<BatchPlane>();
  a.coef = b->d_coef.p;
  a.wfull = b->d_wfull.p;
  a.tw1 = b->d_tw.p;
  a.fx = b->grid.fx;
  a.fy = b->grid.fy;
  a.fz = b->grid.fz;
  a.P = b->P;
  a.grid = b->grid_blocks;
  a.mmax = b->mmax;
  a.chunk = b->chunk;
  a.counter = b->d_counter.as<unsigned int>();
  a.E = E;
  return a;
}

}  // namespace scw

extern "C" {

int scw_batch_plan(scw_ctx* ctx, scw_solution* const* jobs, int njobs, const scw_grid* grid,
                   int precision, scw_batch** out) {
  if (!ctx || !jobs || njobs < 1 || !out) return fail(SCW_EINVAL, "null or empty batch");
  *out = nullptr;
  int rc = check_grid(grid);
  if (rc) return rc;
  if (precision != SCW_FP32) return fail(SCW_EINVAL, "batched synthesis runs in SCW_FP32");
  if (grid->fy < 2 || (grid->fy & (grid->fy - 1)) != 0)
    return fail(SCW_EINVAL, "batched synthesis needs fy a power of two");
  SCW_HIP(hipSetDevice(ctx->c.device));
  std::unique_ptr<scw_batch> b(new (std::nothrow) scw_batch());
  if (!b) return fail(SCW_ENOMEM, "batch allocation failed");
  b->ctx = &ctx->c;
  b->njobs = njobs;
  b->grid = *grid;
  const int fz = grid->fz;
  std::vector<BatchJob> jt(njobs);
  std::vector<BatchPlane> pt((size_t)njobs * fz);
  std::vector<float> coef;
  const double dz = (grid->z_end - grid->z_begin) / fz;
  for (int j = 0; j < njobs; ++j) {
    if (!jobs[j]) return fail(SCW_EINVAL, "null job");
    const Solution& s = jobs[j]->s;
    if (s.device != ctx->c.device) return fail(SCW_EINVAL, "job on another device");
    if (s.U > 31 || s.V > 31) return fail(SCW_EINVAL, "batched synthesis needs U, V <= 31");
    const double zL = s.L * s.d;
    for (int p = 0; p < fz; ++p) {
      const double z = grid->z_begin + (p + 0.5) * dz;
      if (z < 0.0) pt[(size_t)j * fz + p] = {0, (float)z};
      else if (z >= zL) pt[(size_t)j * fz + p] = {2, (float)(z - zL)};
      else return fail(SCW_EINVAL, "batched grid plane inside job " + std::to_string(j));
    }
    const int M = s.M;
    jt[j] = {s.U, s.V, (long long)(coef.size() / 2)};
    auto put = [&](zc c) {
      coef.push_back((float)c.real());
      coef.push_back((float)c.imag());
    };
    for (int i = 0; i < 3 * M; ++i) put(s.p_inc[i]);  // illumination 0
    for (int i = 0; i < 3 * M; ++i) put(s.p_ref[i]);
    for (int i = 0; i < 3 * M; ++i) put(s.p_trn[i]);
    for (int m = 0; m < M; ++m) put(s.k * s.sz_top[m]);
    for (int m = 0; m < M; ++m) put(s.k * s.sz_bot[m]);
  }
  // work items, costliest jobs first
  std::vector<int> order(njobs);
  for (int j = 0; j < njobs; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return jt[x].U * jt[x].V > jt[y].U * jt[y].V;
  });
  const int nft = (grid->fx + 63) / 64;
  std::vector<BatchItem> items;
  items.reserve((size_t)njobs * fz * nft);
  for (int j : order)
    for (int p = 0; p < fz; ++p)
      for (int ft = 0; ft < nft; ++ft) items.push_back({j, p, ft, 0});
  b->mmax = 1;
  for (int j = 0; j < njobs; ++j) b->mmax = std::max(b->mmax, jt[j].U * jt[j].V);
  b->n_items = (int)items.size();
  if ((rc = upload(b->d_jobs, jt.data(), jt.size() * sizeof(BatchJob))) ||
      (rc = upload(b->d_items, items.data(), items.size() * sizeof(BatchItem))) ||
      (rc = upload(b->d_planes, pt.data(), pt.size() * sizeof(BatchPlane))) ||
      (rc = upload(b->d_coef, coef.data(), coef.size() * 4)) ||
      (rc = b->d_counter.reserve(256)))
    return rc;
  SCW_HIP(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, ctx->c.device));
  Context::BatchShape sh{std::min(32, std::max(2, grid->fy / 16)), 4, 1};
  auto it = ctx->c.tuned_batch.find(batch_key(*grid));
  if (it != ctx->c.tuned_batch.end()) sh = it->second;
  if ((rc = batch_set_shape(b.get(), sh.P, sh.blocks_per_cu, sh.chunk))) return rc;
  SCW_HIP(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
  *out = b.release();
  return SCW_OK;
}

int scw_batch_launch(scw_batch* b, void* E_dev, void* hip_stream) {
  if (!b || !E_dev) return fail(SCW_EINVAL, "null argument");
  SCW_HIP(hipSetDevice(b->ctx->device));
  if (!b->exec || b->graph_E != E_dev) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (b->graph) {
      (void)hipGraphDestroy(b->graph);
      b->graph = nullptr;
    }
    const BatchArgs a = batch_args(b, E_dev);
    SCW_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = launch_batch(a, b->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(b->capture_stream, &g);
    if (le != hipSuccess || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(SCW_EHIP, std::string("batch graph capture failed: ") +
                                hipGetErrorString(le != hipSuccess ? le : ce));
    }
    b->graph = g;
    SCW_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_E = E_dev;
  }
  SCW_HIP(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(hip_stream)));
  return SCW_OK;
}

void scw_batch_free(scw_batch* b) { delete b; }

int scw_batch_configure(scw_batch* b, int radix, int blocks_per_cu, int chunk) {
  if (!b) return fail(SCW_EINVAL, "null argument");
  SCW_HIP(hipSetDevice(b->ctx->device));
  // validates every argument before it changes the batch
  return batch_set_shape(b, radix, blocks_per_cu, chunk);
}

long long scw_sur_param_count(void) { return sur_param_count(); }

int scw_sur_create(scw_ctx* ctx, int max_batch, unsigned long long seed, scw_sur** out) {
  if (!ctx || !out) return fail(SCW_EINVAL, "null argument");
  *out = nullptr;
  SurNet* n = nullptr;
  int rc = sur_create(ctx->c, max_batch, seed, &n);
  if (rc) return rc;
  *out = reinterpret_cast<scw_sur*>(n);
  return SCW_OK;
}

void scw_sur_free(scw_sur* s) { sur_free(reinterpret_cast<SurNet*>(s)); }

#define SUR(s) (*reinterpret_cast<SurNet*>(s))

int scw_sur_get_params(scw_sur* s, float* host) {
  if (!s || !host) return fail(SCW_EINVAL, "null argument");
  return sur_get_params(SUR(s), host);
}
int scw_sur_set_params(scw_sur* s, const float* host) {
  if (!s || !host) return fail(SCW_EINVAL, "null argument");
  return sur_set_params(SUR(s), host);
}
int scw_sur_set_compute(scw_sur* s, int bf16) {
  if (!s) return fail(SCW_EINVAL, "null argument");
  if (bf16 != 0 && bf16 != 1) return fail(SCW_EINVAL, "bf16 must be 0 or 1");
  return sur_set_compute(SUR(s), bf16 == 1);
}
int scw_sur_encode(scw_sur* s, const void* n_dev, int batch, void* x_dev, void* stream) {
  if (!s || !n_dev || !x_dev) return fail(SCW_EINVAL, "null argument");
  return sur_encode(SUR(s), n_dev, batch, x_dev, reinterpret_cast<hipStream_t>(stream));
}
int scw_sur_forward(scw_sur* s, const void* x_dev, int batch, void* out_dev, void* stream) {
  if (!s || !x_dev || !out_dev) return fail(SCW_EINVAL, "null argument");
  return sur_forward(SUR(s), x_dev, batch, out_dev, reinterpret_cast<hipStream_t>(stream));
}
int scw_sur_loss_grad(scw_sur* s, const void* x_dev, const void* target_dev, int batch,
                      double* loss, float* grad_host, void* stream) {
  if (!s || !x_dev || !target_dev) return fail(SCW_EINVAL, "null argument");
  return sur_loss_grad(SUR(s), x_dev, target_dev, batch, loss, grad_host,
                       reinterpret_cast<hipStream_t>(stream));
}
int scw_sur_train_step(scw_sur* s, const void* x_dev, const void* target_dev, int batch,
                       float lr, double* loss, void* stream) {
  if (!s || !x_dev || !target_dev) return fail(SCW_EINVAL, "null argument");
  return sur_train_step(SUR(s), x_dev, target_dev, batch, lr, loss,
                        reinterpret_cast<hipStream_t>(stream));
}
int scw_sur_infer_checked(scw_ctx* ctx, scw_sur* s, const double* n_host, int batch,
                          int n_check, unsigned long long seed, double tol, double* out_host,
                          int* fell_back, double* check_err) {
  if (!ctx || !s) return fail(SCW_EINVAL, "null argument");
  return sur_infer_checked(ctx->c, SUR(s), n_host, batch, n_check, seed, tol, out_host,
                           fell_back, check_err);
}
#undef SUR

}  // extern "C"

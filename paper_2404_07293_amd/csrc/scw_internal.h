// Internal types shared by the host setup, the kernel launchers and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/scw.h"

namespace scw {

using zc = std::complex<double>;

// ------------------------------------------------------------------ errors
struct Error {
  int code;
  std::string msg;
};
void set_error(int code, const std::string& msg);
int fail(int code, const std::string& msg);

#define SCW_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return ::scw::fail(SCW_EHIP, std::string(#call) + ": " +                 \
                                       hipGetErrorString(e_) + " (" +          \
                                       std::to_string((int)e_) + ")");         \
  } while (0)

// ------------------------------------------------------------------ device memory
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Grows (never shrinks); contents are not preserved.
  int reserve(size_t n) {
    if (n <= bytes) return SCW_OK;
    release();
    if (n == 0) return SCW_OK;
    if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      return fail(SCW_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
    return SCW_OK;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// ------------------------------------------------------------------ synthesis plan
// One interior task = one layer and up to `zt` consecutive planes inside it.
struct Task {
  int layer;
  int plane0;   // first output plane index
  int count;    // planes in this task (<= zt)
  int pad;
};

// Exterior plane entry of a plan (device table).
struct ExtPlane {
  int plane;
  int kind;   // 0 above, 2 below
  double dz;  // z - z0 (above) or z - zL (below)
};

struct PlaneInfo {
  int kind;     // 0 above, 1 inside, 2 below
  int layer;
  double dz_top;  // z - z_top(layer) inside; z - z0 above; z - zL below
  double dz_bot;  // z - z_bot(layer) inside
};

struct Plan {
  scw_grid grid{};
  int precision = -1;
  int zt = 0;                       // planes per task (1, 2, 4 or 8)
  std::vector<Task> tasks;
  std::vector<PlaneInfo> planes;
  int n_exterior = 0;
  DevBuf d_tasks;                   // Task[ntasks]
  DevBuf d_task_dz;                 // double2 [ntasks][zt] (dz_top, dz_bot)
  DevBuf d_task_dz32;               // float2 [ntasks][zt]
  DevBuf d_ext;                     // int2 + double: exterior plane table
  DevBuf d_w;                       // W  [ntasks][2][zt][2M] complex<T>
  DevBuf d_spec;                    // [fz][3M] complex<T>
  DevBuf d_amat;                    // MFMA twiddle operand of the y pass
  DevBuf d_bmat;                    // MFMA T operand written by the x pass
  DevBuf d_bscale;                  // float [fz*3] power-of-two operand scales
  int kp = 0;                       // padded K of the y-pass GEMM
  int fft_p = 0;                    // factored y pass (fy = R * P) when > 0
  DevBuf d_fft_tw;                  // its twiddles
  bool mfma = false;                // inverse transform on the matrix cores
  int modal_rw = 0;                 // rows per wave of the FP32 modal sum
  int tiles = 0;                    // DIRECT row tiles / MFMA plane-components per block
  scw_synth_config cfg{};           // the configuration the plan was built for
  bool direct_only = false;         // built for the direct-sum transform (slices)
  DevBuf d_twx;                     // [2][fx] complex<T>: e^{2 pi i f/fx}, e^{-2 pi i (U/2) f/fx}
  DevBuf d_twy;                     // [2][fy] complex<T>: same for g, V
  DevBuf d_spec_multi;              // [K][fz][3M] complex64: spectra of every illumination
  DevBuf d_wmulti;                  // phase table of one illumination group
  DevBuf d_tile;                    // [3][fz][fy][fx]: one period, for tiled / composed fields
  bool valid = false;
};

// ------------------------------------------------------------------ solution
struct Solution {
  int U = 0, V = 0, M = 0, L = 0;
  int K = 1;  // illuminations sharing the eigendecomposition
  double lam = 0, k = 0, X = 0, Y = 0, d = 0;
  std::vector<int> u, v;
  std::vector<double> sx, sy;
  std::vector<zc> sz_top, sz_bot;
  std::vector<zc> p_inc, p_ref, p_trn;   // [K][3M]
  // per layer, forward-branch eigenvalues and mode coefficients
  std::vector<zc> gamma;                 // [L][2M]
  std::vector<zc> a, b;                  // [K][L][2M]
  scw_solution_info info{};

  // device copies
  DevBuf d_P64;      // [L][3M][2M] complex128, row-major
  DevBuf d_P32;      // [L][3M][2M] complex64
  DevBuf d_kg;       // [L][2M] complex128: k * gamma
  DevBuf d_a, d_b;   // [K][L][2M] complex128
  DevBuf d_kgab32;   // [3][L][2M] complex64: k*gamma, a, b of illumination 0
  DevBuf d_ab32;     // [K][2][L][2M] complex64: a, b of every illumination (K > 1)
  DevBuf d_ext;      // [K][3][3M] complex128: p_inc, p_ref, p_trn
  DevBuf d_ksz;      // [2][M] complex128: k*sz_top, k*sz_bot
  // Synthesis plans, one per (grid, precision, resolved configuration, slice
  // or volume). A plan is never rebuilt in place and lives until the solution
  // is freed, so work enqueued (or captured in a graph) with one plan stays
  // valid when later calls use another grid, precision or configuration.
  std::vector<std::unique_ptr<Plan>> plans;
  scw_synth_config cfg{};  // explicit kernel configuration (0 fields: library choice)
  int device = 0;
};

// ------------------------------------------------------------------ context
constexpr int kNumStages = 4;  // phase (FP64 path), modal sum, exterior, inverse DFT

struct Context {
  int device = 0;
  void* blas = nullptr;  // rocBLAS handle of the device elimination (created on first use)
  int host_threads = 1;
  hipStream_t setup_stream = nullptr;
  // profiling: (kNumStages + 1) events per recorded call
  std::vector<hipEvent_t> prof_events;
  int prof_max = 0;
  int prof_used = 0;
  // autotuner results, keyed by problem and grid shape
  std::map<std::string, scw_synth_config> tuned_synth;
  struct BatchShape {
    int P, blocks_per_cu, chunk;
  };
  std::map<std::string, BatchShape> tuned_batch;
};

// Stages of one synthesis call, selectable for timing.
enum StageMask { kStageModal = 1, kStageExterior = 2, kStageTransform = 4, kStageAll = 7 };

// The plan of (grid, precision, the configuration resolve_config gives, and
// direct_only) for solution s: found among s.plans or built (synchronously)
// and added. direct_only builds it for the direct-sum transform, which
// accepts any lateral size (the slices use only its tables).
int get_plan(Context& ctx, Solution& s, const scw_grid& g, int precision, bool direct_only,
             Plan** out);
// Plan (if needed) and enqueue one synthesis; `stages` selects kernels, `ev`
// (nullable) receives kNumStages + 1 stage events and `used` (nullable) the
// plan whose workspaces the kernels use.
int synthesize(Context& ctx, Solution& s, const scw_grid& g, int precision, void* E,
               hipStream_t st, int stages, hipEvent_t* ev, bool direct_only = false,
               Plan** used = nullptr);
std::string synth_key(const Solution& s, const scw_grid& g, int precision);
// Plane j of grid g against a stack of L layers of thickness d: above the
// sample, inside layer `layer`, or below it (a plane on an interface belongs
// to the layer below).
PlaneInfo classify_plane(const scw_grid& g, int L, double d, int j);
// Interior planes are grouped per layer in tasks of zt (1, 2, 4 or 8) planes.
struct PlaneGroups {
  int zt, ntasks, n_ext;
};
PlaneGroups plane_group_shape(const scw_grid& g, int L, double d);
// The configuration of a synthesis: the solution's explicit one with the
// context's tuned entry filling its zero fields.
scw_synth_config resolve_config(const Context& ctx, const Solution& s, const scw_grid& g,
                                int precision);
// Kernel shape from a configuration: modal-sum rows per wave, transform kind
// (SCW_XFORM_*), factored-transform radix (0 unless kind is FFT), tiles, and
// whether the factored transform applies to this grid at all.
struct KernelShape {
  int modal_rw, kind, fft_p, tiles;
  bool fft_ok;
};
int choose_shape(const Solution& s, const scw_grid& g, int precision,
                 const scw_synth_config& cfg, int zt, KernelShape* out);
// SCW_OK for a grid every synthesis accepts, else SCW_EINVAL with a message.
int check_grid(const scw_grid* g);
// Allocation-free synthesis: attach the device's static scratch array (once
// per device, from scw_create).
int noalloc_attach(int device);
// FP32 fields of every illumination, E: [K][3][fz][fy][fx] complex64.
int synthesize_illuminations(Context& ctx, Solution& s, const scw_grid& g, void* E,
                             hipStream_t st);

// ------------------------------------------------------------------ setup
// n_waves > 0: one plane-wave illumination per entry of `waves` (the
// problem's own incident field is then ignored), sharing one setup.
int solve_problem(Context& ctx, const scw_problem& prob, Solution& sol, int n_waves = 0,
                  const scw_plane_wave* waves = nullptr);
// n problems solved together: their device eigendecompositions
// (SCW_EIG_DEVICE) of equal truncation share launches; each other step runs
// per problem as in solve_problem. sols[i] receives problem i.
int solve_problems(Context& ctx, const scw_problem* probs, int n, Solution** sols);
void release_blas(Context& ctx);
// Elementwise steps of the device elimination, column-major complex128
// n x n blocks: A = I; A1, A2 <- (A1 + A2)/2, (A1 - A2)/2 over n entries;
// P1, P2 = I +- E r E with E diagonal; out = diag(E) A for n x k A.
hipError_t launch_eye(double* A, int n, hipStream_t s);
// Top-surface system [[I, -Fe], [Hr, -Fh]] (4M x 4M) of the stable route.
hipError_t launch_top_system(const double* Hr, const double* Fe, const double* Fh, int n2,
                             double* S, hipStream_t s);
// The 6M x 6M connection system of Eq. 29 from K C_r, C_t (4M x 3M) and the
// Gauss rows (sx, sy real [M]; szt, szb complex [M]).
hipError_t launch_connection_system(const double* KCr, const double* Ct, const double* sx,
                                    const double* sy, const double* szt, const double* szb,
                                    int M, double* A, hipStream_t s);
// Column sums of |A| of a column-major n x n complex matrix (its 1-norm is the largest).
hipError_t launch_col_abs_sum(const double* A, int n, double* out, hipStream_t s);
hipError_t launch_half_sum_diff(double* A1, double* A2, long long n, hipStream_t s);
hipError_t launch_i_pm_ere(const double* r, const double* E, int n, double* P1, double* P2,
                           hipStream_t s);
hipError_t launch_scale_rows(const double* E, const double* A, int n, int k, double* out,
                             hipStream_t s);
// T = W diag(I, E), B = W diag(E, I) with W = [[X, X], [Y, -Y]] (4M x 4M).
hipError_t launch_build_tb(const double* X, const double* Y, const double* E, int n2, double* T,
                           double* B, hipStream_t s);

// ------------------------------------------------------------------ eigensolver
// Batched FP64 eigendecomposition on the device (kernels_eig.hip, eig.cpp).
constexpr int kEigMaxN = SCW_EIG_MAX_N;
// count matrices n x n column-major complex128 (A overwritten): eigenvalues w
// [count][n] and unit-norm eigenvectors X [count][n][n]. Blocks until done.
int device_eig_batched(Context& ctx, int n, int count, double* A, double* w, double* X,
                       hipStream_t st);
// The context's rocBLAS handle (created on first use), bound to stream st.
int blas_handle(Context& ctx, hipStream_t st, void** out);
hipError_t launch_eig_hessenberg(int n, int count, double* A, double* Z, hipStream_t s);
hipError_t launch_eig_schur(int n, int count, double* H, double* Z, double* w, int* info,
                            hipStream_t s);
// T (column-major Schur factors) -> Tt (row-major copies) -> Y (eigenvectors
// of T, column-major; Y may be T).
hipError_t launch_eig_vectors(int n, int count, const double* T, double* Tt, const double* w,
                              double* Y, hipStream_t s);
hipError_t launch_eig_normalize(int n, long long ncols, double* X, hipStream_t s);
// X[:, j] *= f[j] over ncols columns of length n (f: complex128 [ncols]).
hipError_t launch_eig_scale_cols(int n, long long ncols, const double* f, double* X,
                                 hipStream_t s);

// ------------------------------------------------------------------ surrogate
struct SurNet;
long long sur_param_count();
int sur_create(Context& ctx, int max_batch, unsigned long long seed, SurNet** out);
void sur_free(SurNet* n);
int sur_set_params(SurNet& n, const float* host);
int sur_get_params(SurNet& n, float* host);
int sur_set_compute(SurNet& n, bool bf16);
int sur_encode(SurNet& n, const void* n_dev, int B, void* x_dev, hipStream_t s);
int sur_forward(SurNet& n, const void* x_dev, int B, void* out_dev, hipStream_t s);
int sur_loss_grad(SurNet& n, const void* x_dev, const void* tgt_dev, int B, double* loss,
                  float* grad_host, hipStream_t s);
int sur_train_step(SurNet& n, const void* x_dev, const void* tgt_dev, int B, float lr,
                   double* loss, hipStream_t s);
int sur_infer_checked(Context& ctx, SurNet& n, const double* n_host, int B, int n_check,
                      unsigned long long seed, double tol, double* out_host, int* fell_back,
                      double* check_err);

// ------------------------------------------------------------------ kernels
// All launchers enqueue on `s` and return a HIP status code.
hipError_t launch_band_dft(const double* n, int L, int ny, int nx, int hu, int hv,
                           bool inverse_eps_too, bool square, double* rowbuf,
                           double* out_eps, double* out_inv, hipStream_t s);
hipError_t launch_assemble_ac(const double* phi, const double* psi,
                              const int* u, const int* v, const double* sx,
                              const double* sy, int U, int V, int L,
                              double* A, double* C, hipStream_t s);
hipError_t launch_build_p(const double* X, const double* Y, const double* psi,
                          const int* u, const int* v, const double* sx,
                          const double* sy, int U, int V, int nlayers,
                          double* P, hipStream_t s);
hipError_t launch_p_to_fp32(const double* P64, float* P32, size_t n_complex,
                            hipStream_t s);

struct SynthArgs {
  int M, U, V, L, fx, fy, fz, zt, ntasks, n_ext;
  const void* P;           // [L][3M][2M] complex<T>
  const double* kg;        // [L][2M] complex128
  const double* a;         // [L][2M]
  const double* b;         // [L][2M]
  const double* ext;       // [3][3M]
  const double* ksz;       // [2][M]
  const Task* tasks;
  const double* task_dz;   // [ntasks][zt][2]
  const void* ext_planes;  // exterior plane table
  void* w;                 // [ntasks][2][zt][2M] complex<T>
  void* spec;              // [fz][3M]
  const void* twx;         // [2][fx]: e^{2 pi i f/fx}, e^{-2 pi i (U/2) f/fx}
  const void* twy;         // [2][fy]: e^{2 pi i g/fy}, e^{-2 pi i (V/2) g/fy}
  void* E;                 // [3][fz][fy][fx]
  const void* kgab32;      // complex64 [3][L][2M]: k*gamma, a, b
  const void* task_dz32;   // float2 [ntasks][zt]
  int idft_gtiles;         // 0 = automatic
  int modal_rw;            // rows per wave of the FP32 modal sum (2, 4, 8, 16)
  int stages;              // StageMask
  int precision;           // scw_precision
  bool mfma;               // inverse transform on the matrix cores
  int kp;
  int fft_p;               // > 0: factored transform with this P (fy = R * P)
  const void* fft_tw;      // [R][32] first-stage twiddles of the factored transform
  void* bmat;
  float* bscale;
  const void* amat;
};

struct MfmaArgs {
  int U, V, fx, fy, fz, Kp;
  int pcb;            // plane/components per y-pass block (0 = automatic)
  const void* spec;   // [fz*3][M] complex64
  const void* wx;     // [2][fx] complex64
  void* bmat;
  float* bscale;
  const void* amat;
  void* E;
};
int mfma_kstep(int precision);

// ------------------------------------------------------------------ batched synthesis
struct BatchJob {
  int U, V;
  long long coef_offset;  // complex64 elements into the coefficient buffer
};
struct BatchItem {  // one (job, plane, 64-column tile), all three components
  int job, plane, ftile, pad;
};
struct BatchPlane {
  int kind;   // 0 above the sample, 2 below it
  float dz;   // z - z0 above, z - zL below
};
struct BatchArgs {
  const BatchJob* jobs;
  const BatchItem* items;
  int n_items;
  const BatchPlane* planes;  // [njobs][fz]
  const void* coef;          // complex64 per job: p_inc, p_ref, p_trn [3][M] each, k sz_top, k sz_bot [M]
  const void* wfull;         // [fx]: e^{2 pi i k / fx}
  const void* tw1;           // [32][R]
  int fx, fy, fz, P, grid;
  int mmax;                  // largest U * V of the jobs (LDS spectra)
  int chunk;                 // items per grab from the work counter
  unsigned int* counter;
  void* E;                   // [njobs][3][fz][fy][fx] complex64
};
hipError_t launch_batch(const BatchArgs& a, hipStream_t s);

}  // namespace scw

// ------------------------------------------------------------------ ABI handles
struct scw_ctx {
  scw::Context c;
};
struct scw_solution {
  scw::Solution s;
};
struct scw_batch {
  scw::Context* ctx = nullptr;
  int njobs = 0, n_items = 0, P = 0, grid_blocks = 0, cus = 0, chunk = 1, mmax = 1;
  scw_grid grid{};
  scw::DevBuf d_jobs, d_items, d_planes, d_coef, d_wfull, d_tw, d_counter;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* graph_E = nullptr;
  ~scw_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

namespace scw {

// Batched synthesis shape: P of the factored y pass (fy = R * P) and the
// persistent grid; rebuilds the twiddles and drops the captured graph.
int batch_set_shape(scw_batch* b, int P, int blocks_per_cu, int chunk);
BatchArgs batch_args(const scw_batch* b, void* E);
std::string batch_key(const scw_grid& g);

// ------------------------------------------------------------------ surrogate kernels
// C[b] = op(A[b]) op(B[b]) + beta C[b]; strides in elements of each operand's
// type (complex operands interleaved). c_cplx = 0 keeps the real part.
struct GemmOp {
  int M, N, K, batch;
  int a_cplx, b_cplx, c_cplx;
  int conj_a, conj_b;
  const float* A;
  long long a_rs, a_cs, a_bs;
  const float* B;
  long long b_rs, b_cs, b_bs;
  float* C;
  long long c_rs, c_cs, c_bs;
  float beta;
  int bf16;  // operands rounded to bf16, products on the matrix cores (FP32 accumulate)
};
hipError_t launch_gemm(const GemmOp& op, hipStream_t s);
hipError_t sur_gelu_bwd(const float* z, float* g, long long n, hipStream_t s);
hipError_t sur_sum_batch(const float* in, float* out, int B, long long per, hipStream_t s);
hipError_t sur_bias_grad(const float* g, float* out, int B, int C, int P, hipStream_t s);
hipError_t sur_loss(const float* out, const float* tgt, long long n, float* sums, float* g,
                    hipStream_t s);
hipError_t sur_adam(float* p, const float* g, float* m, float* v, long long n, float lr, int t,
                    hipStream_t s);
hipError_t sur_encode(const float* n, float* x, int B, hipStream_t s);
// One Fourier layer around its mixing: H = fy h fx per channel (17 x 9
// modes, mode-major [mode][b][i]; or the head's 15 x 15 with head, [b][i][mode]),
// and z = Re(iy G ix) + pw^T h + pb with G laid out [b][mode][o] and
// h' = GELU(z) (gelu) or z; z_out may be null; h_out may equal z_out when
// gelu is false.
hipError_t sur_fused_dft_fwd(const float* h, const float* fy, const float* fx, float* H, int B,
                            bool head, bool bf16, hipStream_t s);
// The head's mixing, out[b][o][m] = sum_i A[b][i][m] W[i][o][m] for 32 input
// and O = 3 output channels.
hipError_t sur_mode_mix(const float* A, const float* W, int nmode, int B, int O, float* out,
                        bool bf16, hipStream_t s);
// A layer's mixing on the matrix cores, from mode-major spectra and weights:
// out[b][m][o] = sum_i A[m][b][i] Wm[m][i][o], 32 input and output channels.
hipError_t sur_mode_mix_layer(const float* A, const float* Wm, int nmode, int B, float* out,
                              bool bf16, hipStream_t s);
// Wm[k][m][i][o] = W_k[i][o][m] for `layers` layers whose weights start
// layer_stride_floats apart.
hipError_t sur_spec_mode_major(const float* W, long long layer_stride_floats, int nmode,
                               int layers, float* Wm, hipStream_t s);
// h[b][o] = sum_c lw[c][o] x[b][c] + lb[o] over 16 input, 32 output channels.
hipError_t sur_lift(const float* x, const float* lw, const float* lb, float* h, int B, bool bf16,
                    hipStream_t s);
hipError_t sur_fused_dft_inv(const float* G, const float* h, const float* iy, const float* ix,
                             const float* pw, const float* pb, float* z_out, float* h_out,
                             bool gelu, int B, bool bf16, hipStream_t s);
// Matrix-core inference with bf16 storage (kernels_surrogate_bf16.hip):
// activations h bf16 [b][c][32][32]; spectra packed complex bf16 words,
// mode-major H[m][b][c] (the layer's 153 modes, or the head's 225 with head)
// and G[b][m][o]; Wb the mixing weights as matrix-core operands,
// sur_mix_weights_bf16_bytes(layers) bytes built from the parameters by
// sur_mix_weights_bf16; out the head's FP32 complex [b][3][225].
hipError_t sur_lift_bf16(const float* x, const float* lw, const float* lb, void* h, int B,
                         hipStream_t s);
hipError_t sur_fwd_bf16(const void* h, const float* fy, const float* fx, void* H, int B,
                        bool head, hipStream_t s);
hipError_t sur_mix_weights_bf16(const float* W, long long layer_stride_floats, int layers,
                                void* Wb, hipStream_t s);
size_t sur_mix_weights_bf16_bytes(int layers);
hipError_t sur_mix_bf16(const void* H, const void* Wb_layer, int B, void* G, hipStream_t s);
hipError_t sur_inv_bf16(const void* G, const void* h, const float* iy, const float* ix,
                        const float* pw, const float* pb, void* h_out, bool gelu_on, int B,
                        hipStream_t s);
hipError_t sur_head_mix_bf16(const void* F, const float* W, int B, float* out, hipStream_t s);
hipError_t launch_idft_mfma(const MfmaArgs& a, int precision, hipStream_t s);
// `ev`, when non-null, holds kNumStages + 1 events recorded around the stages.
hipError_t launch_synthesis_fp64(const SynthArgs& a, hipStream_t s, hipEvent_t* ev);
hipError_t launch_synthesis_fp32(const SynthArgs& a, hipStream_t s, hipEvent_t* ev);
// FP32 modal sum of illuminations k0 .. k0 + kcount - 1 on the matrix cores:
// spec[k][plane][r] = sum_j P_l[r][j] W_k(sign(r))[plane][j] for every
// interior plane, kcount * zt <= 32. kg: complex64 [L][2M] (k * gamma);
// ab: complex64 [K][2][L][2M]; W: workspace of multi_table_bytes(ntasks, M)
// for the group's phase table; spec: complex64 [K][fz][3M].
inline int multi_row_pitch(int M) { return (2 * M + 15) / 16 * 16; }
inline size_t multi_table_bytes(int ntasks, int M) {
  return (size_t)ntasks * 2 * 32 * multi_row_pitch(M) * 8;
}
hipError_t launch_modal_multi(const void* P, const void* kg, const void* ab, const Task* tasks,
                              const void* task_dz32, int ntasks, int zt, int M, int L, int fz,
                              int k0, int kcount, void* W, void* spec, hipStream_t s);
// A lateral slice from the per-plane spectra [fz][3M] (complex<T>): axis 0
// sums over v with e^{2 pi i (v - V/2) frac} and runs u on the n samples with
// tw = [2][n] (e^{2 pi i f/n}, e^{-2 pi i (U/2) f/n}); axis 1 the same with
// u and v exchanged. E: [3][fz][n] complex<T>.
struct SliceArgs {
  const void* spec;
  const void* tw;
  int U, V, n, fz, axis;
  double frac;  // position / period of the summed axis
  void* E;
};
hipError_t launch_slice(const SliceArgs& a, bool fp64, hipStream_t s);
// Zero the spectra [n / M][M] (complex<T>) of the modes with
// (u sx_step)^2 + (v sy_step)^2 > na^2 (u, v the mode's frequency indices).
hipError_t launch_objective(void* spec, long long n, int M, int U, int V, double sx_step,
                            double sy_step, double na, bool fp64, hipStream_t s);
// spec[i] *= H[i mod M] over the spectra [n / M][M] (H: complex128 [M]).
hipError_t launch_transfer(void* spec, long long n, int M, const void* H, bool fp64,
                           hipStream_t s);
// dst[pc][oy + ty fy + g][ox + tx fx + f] = src[pc][g][f] for the 3 fz
// plane-components, tx < rx, ty < ry (dst is [3 fz][dfy][dfx]).
hipError_t launch_place(const void* src, int fx, int fy, int fz, void* dst, int dfx, int dfy,
                        int ox, int oy, int rx, int ry, bool fp64, hipStream_t s);
// I[i] = sum_c |E[c][i]|^2 over the three components of [3][npix].
hipError_t launch_intensity(const void* E, void* I, long long npix, bool fp64, hipStream_t s);

}  // namespace scw

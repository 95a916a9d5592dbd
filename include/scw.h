/*
 * scw.h -- C ABI of the MI355X coupled-wave-theory (CWT) field-synthesis
 * library.
 *
 * The library takes a sample of complex refractive index on a voxel grid and
 * an incident field (a 2D image at the top surface, or one plane wave), solves
 * the coupled-wave boundary-value problem in FP64, and synthesises the 3D
 * electric field on a regular grid on the GPU (gfx950).
 *
 * Section and equation numbers refer to Sun, Reddy and Mayerich, "sCWatter:
 * Open source coupled wave scattering simulation for spectroscopy and
 * microscopy".
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im) pairs of double (complex128) or
 *     float (complex64).
 *   - Host arrays passed in are read-only and owned by the caller; they may be
 *     freed as soon as the call returns.
 *   - Device buffers passed in are owned by the caller and must be allocated
 *     on the context's device. The library never frees them.
 *   - Handles (scw_ctx, scw_solution) are owned by the library and freed with
 *     their destroy call.
 *   - Every int-returning call returns SCW_OK (0) or a negative scw_status;
 *     scw_last_error() then describes the failure. No C++ exception crosses
 *     this boundary.
 *   - A context may be used from one host thread at a time.
 */
#ifndef SCW_H
#define SCW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCW_OK = 0,
    SCW_EINVAL = -1,      /* bad shape, even truncation, null pointer, bad enum */
    SCW_ENOMEM = -2,      /* host or device allocation failed */
    SCW_EHIP = -3,        /* HIP runtime error (message keeps the HIP code) */
    SCW_ELAPACK = -4,     /* LAPACK returned info != 0, or no LAPACK found */
    SCW_EGRAZING = -5,    /* |s_z| < 1e-9 in a half-space (Eq. 2 at grazing) */
    SCW_EDEFECTIVE = -6,  /* |gamma| < 1e-9 max|gamma| in a layer: D defective */
    SCW_EILLCOND = -7     /* connection route chosen explicitly and either its
                             growth exponent exceeds 25 or its 6M x 6M system
                             has a reciprocal condition number below 1e-13
                             (condition above 1e13) */
} scw_status;

typedef enum {
    SCW_FP64 = 0,         /* complex128 synthesis, complex128 output */
    SCW_FP32 = 1,         /* complex64 synthesis, complex64 output */
    SCW_BF16X3 = 2,       /* bf16 hi/lo split products, FP32 accumulate, complex64 out */
    SCW_FP16X3 = 3        /* fp16 hi/lo split products, FP32 accumulate, complex64 out */
} scw_precision;

typedef enum {
    /* Layer-by-layer elimination from the bottom up that only ever forms
       decaying exponentials; the default. Same solution as the full
       boundary-value system of Eqs. 24-26. */
    SCW_ROUTE_STABLE = 0,
    /* The paper's connection equations (Sec. 2.5.4, Eqs. 27-29): the product
       K of per-layer transfer matrices and a 6M x 6M solve. K holds growing
       evanescent exponentials up to exp(growth_exponent), so this route
       fails with SCW_EILLCOND when the growth exponent exceeds 25 or the
       system's reciprocal condition number is below 1e-13. */
    SCW_ROUTE_CONNECTION = 1,
    /* SCW_ROUTE_STABLE with its per-layer elimination on the GPU in FP64
       (rocSOLVER LU with partial pivoting, rocBLAS complex GEMM); the 4M x 4M
       top-surface system stays on the host. Same solution as
       SCW_ROUTE_STABLE to rounding. Needs about 2 L (2M)^2 x 16 bytes of
       device memory for the per-layer interface matrices. */
    SCW_ROUTE_STABLE_DEVICE = 2,
    /* SCW_ROUTE_CONNECTION with the layer matrices, the product K and the
       alpha recursion on the GPU in FP64 (rocSOLVER, rocBLAS); the 6M x 6M
       system stays on the host. Needs about 2 L (4M)^2 x 16 bytes of device
       memory. */
    SCW_ROUTE_CONNECTION_DEVICE = 3
} scw_route;

/* Where the per-layer eigendecompositions of A C run (Sec. 3.2, Sec. 4.2). */
typedef enum {
    /* LAPACK zgeev on the host, one layer per host thread (default). */
    SCW_EIG_HOST = 0,
    /* The library's batched FP64 eigensolver on the GPU (scw_eig_batched):
       every layer at once; agrees with the host route to rounding. Needs
       about 6 L (2M)^2 x 16 bytes of device memory during the solve and
       2M <= SCW_EIG_MAX_N. */
    SCW_EIG_DEVICE = 1
} scw_eig_where;

typedef struct scw_ctx scw_ctx;
typedef struct scw_solution scw_solution;

/* Problem description (Sec. 2.3, Sec. 3). All lengths use the unit of lambda.
 *
 *   nx, ny, nz   sample voxels; layer l covers z in [l*pz, (l+1)*pz], the top
 *                surface is z0 = 0 and the field propagates towards +z.
 *   px, py, pz   voxel pitch; the lateral period is X = nx*px, Y = ny*py and
 *                voxel (i, j) sits at (i*px, j*py).
 *   n            host complex128 [nz][ny][nx]: complex refractive index
 *                n + i*kappa (kappa > 0 absorbs).
 *   lambda       vacuum wavelength.
 *   n_top        real index of the upper half-space.
 *   n_bot_re/im  complex index of the lower half-space.
 *   U, V         odd numbers of spatial frequencies along x and y (Sec. 2.2);
 *                M = U*V.
 *   inc_ex, inc_ey
 *                host complex128 [inc_ny][inc_nx] images of the incident E_x
 *                and E_y at the top surface, spanning one lateral period
 *                (either may be NULL for zero). When both are NULL the
 *                incident field is the plane wave below.
 *   pw_u, pw_v   integer spatial frequency of the incident plane wave; must
 *                lie inside the U x V band.
 *   pw_ex, pw_ey complex (re, im) transverse amplitudes of the plane wave.
 *   route        scw_route of the boundary solve.
 *   eig          scw_eig_where of the eigendecompositions (0: host).
 */
typedef struct {
    int nx, ny, nz;
    double px, py, pz;
    const double* n;
    double lambda;
    double n_top;
    double n_bot_re, n_bot_im;
    int U, V;
    const double* inc_ex;
    const double* inc_ey;
    int inc_nx, inc_ny;
    int pw_u, pw_v;
    double pw_ex[2];
    double pw_ey[2];
    int route;
    int eig;
} scw_problem;

/* Output grid: fx*fy points per plane spanning one lateral period,
 * x_f = f*X/fx, y_g = g*Y/fy, and fz cell-centred planes
 * z_j = z_begin + (j + 1/2)(z_end - z_begin)/fz. Planes above the sample get
 * incident + reflected waves, planes below get the transmitted waves (Eq. 9),
 * planes inside get the modal field of their layer (Eqs. 30-34); a plane on
 * an interface belongs to the layer below. */
typedef struct {
    int fx, fy, fz;
    double z_begin, z_end;
} scw_grid;

/* Diagnostics of one solution. */
typedef struct {
    int M, L;
    double min_abs_sz;         /* min |s_z| over both half-spaces */
    double min_abs_gamma_rel;  /* min |gamma| / max |gamma| over layers */
    double growth_exponent;    /* k * d * sum_l max_j Im(gamma_lj): largest
                                  exponent a transfer-matrix product holds */
    double connection_rcond;   /* reciprocal condition (1-norm) of the 6M x 6M
                                  system for SCW_ROUTE_CONNECTION, else 0 */
    double setup_seconds;      /* wall time of scw_solve */
    double eig_seconds;        /* part spent in the eigensolves */
    double assembly_device_ms; /* GPU time of the band DFT + assembly kernels */
    double boundary_seconds;   /* wall time of the boundary solve (route) */
} scw_solution_info;

/* Thread-local description of the last failure on the calling thread. */
const char* scw_last_error(void);

/* Create a context on HIP device `hip_device`. It owns device workspaces and
 * a host thread pool of `host_threads` workers (<= 0: all hardware threads).
 * Calls that use one context, or one solution, must not overlap in time from
 * several host threads: they update its plans, tuning cache and profiling
 * state. Separate contexts are independent. */
int scw_create(scw_ctx** out, int hip_device, int host_threads);
void scw_destroy(scw_ctx* ctx);

/* FP64 setup (Sec. 3.1-3.4 and Sec. 3.6's alpha recovery):
 *   device  band Fourier coefficients of n^2 and 1/n^2 per layer (Eqs. 11-12)
 *           and the blocks of the property matrix D (Eq. 21);
 *   host    per-layer eigendecomposition (LAPACK zgeev on the 2M x 2M product
 *           of D's off-diagonal blocks, since D^2 is block diagonal),
 *           boundary solve by `route`, and the mode coefficients alpha of
 *           every layer;
 *   device  the per-layer synthesis matrix P = [Q_x; Q_y; Psi (S_y Q_bx -
 *           S_x Q_by)] of Sec. 4.1 (Eq. 34), its z rows by a band
 *           convolution with psi.
 * Blocks until done. On success *out is a library-owned solution. */
int scw_solve(scw_ctx* ctx, const scw_problem* prob, scw_solution** out);

/* n problems solved together (Sec. 3; the setup of a spectral sweep or of a
 * training set). Each is solved as scw_solve would solve it; the device
 * eigendecompositions (eig = SCW_EIG_DEVICE) of all problems with the same
 * truncation U*V share one batched launch of the eigensolver, in rounds of
 * up to about 24 GB of device workspace. On success out[i] (caller-provided
 * array of n pointers) receives problem i's solution, each freed by
 * scw_solution_free. On failure every out[i] is NULL and the message names
 * the problem. The solutions' eig_seconds all report the shared batch time
 * of their round (plus any host part). */
int scw_solve_batch(scw_ctx* ctx, const scw_problem* probs, int n, scw_solution** out);

/* Batched FP64 eigendecomposition on the GPU (the step of Sec. 3.2 and
 * Sec. 4.2 that the paper names its next bottleneck), as scw_solve runs it
 * for SCW_EIG_DEVICE: count independent n x n complex matrices, each reduced
 * to Hessenberg form by Householder reflections, to complex Schur form by the
 * shifted QR algorithm, and its eigenvectors found by back-substitution on
 * the Schur factor.
 *   n          matrix order, 1 <= n <= SCW_EIG_MAX_N;
 *   A_dev      device complex128 [count][n][n], column-major; overwritten;
 *   w_dev      device complex128 [count][n]: the eigenvalues;
 *   X_dev      device complex128 [count][n][n], column-major: column j is a
 *              unit-norm eigenvector of eigenvalue j.
 * Workspace (2 count n^2 x 16 bytes) is allocated and freed by the call,
 * which blocks until the result is ready. Errors: SCW_EINVAL for a bad size
 * or null pointer; SCW_ELAPACK when the QR iteration of a matrix does not
 * converge (the message names the matrix); SCW_ENOMEM, SCW_EHIP. */
#define SCW_EIG_MAX_N 2048
int scw_eig_batched(scw_ctx* ctx, int n, int count, double* A_dev, double* w_dev,
                    double* X_dev, void* hip_stream);
void scw_solution_free(scw_solution* sol);
int scw_solution_info_get(const scw_solution* sol, scw_solution_info* info);

/* Copy the exterior coefficients (host complex128 [3][M] each, component
 * major p_x, p_y, p_z, mode order m of Sec. 2.2) into caller buffers; any
 * pointer may be NULL. p_inc is at z0, p_ref at z0, p_trn at the bottom
 * surface (Eq. 9). */
int scw_solution_exterior(const scw_solution* sol, double* p_inc, double* p_ref,
                          double* p_trn);

/* One plane-wave illumination: integer spatial frequency (u, v) inside the
 * U x V band and complex (re, im) transverse amplitudes, as the problem's
 * pw_* fields. */
typedef struct {
    int u, v;
    double ex[2];
    double ey[2];
} scw_plane_wave;

/* Several illuminations of one sample (Sec. 2.3's incident field, one plane
 * wave each, e.g. the directions of a condenser aperture) sharing one setup:
 * the band coefficients, eigendecompositions, synthesis matrices P and the
 * factorisation of the boundary system are computed once; each illumination
 * adds only its right-hand side and mode coefficients. The problem's own
 * incident fields (inc_ex, inc_ey, pw_*) are ignored. `waves`: host array of
 * n_waves (1..4096) entries, read during the call. The solution behaves as a
 * scw_solve result for illumination 0 in every other entry point
 * (scw_synthesize, scw_solution_exterior, ...). Errors as scw_solve, and
 * SCW_EINVAL for a wave outside the band or a bad count. */
int scw_solve_illuminations(scw_ctx* ctx, const scw_problem* prob, int n_waves,
                            const scw_plane_wave* waves, scw_solution** out);

/* The fields of every illumination of a scw_solve_illuminations solution on
 * `grid`, as n_waves scw_synthesize calls would give them. The modal sum of
 * all illuminations reads each layer's P once, on the matrix cores (FP32
 * inputs, FP32 accumulation), then each illumination's exterior planes and
 * inverse transform follow. precision: SCW_FP32 only. E_dev: caller-owned
 * device complex64 [n_waves][3][fz][fy][fx]. Work is enqueued on hip_stream;
 * the first call for a grid builds its plan synchronously. Errors:
 * SCW_EINVAL for a null argument, another precision or a bad grid. */
int scw_synthesize_illuminations(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid,
                                 int precision, void* E_dev, void* hip_stream);

/* Field synthesis, the hot path (Eqs. 9, 10, 30-34):
 *   for every plane, p(m, z) = P_l (alpha_l o g(z)) inside layer l, or the
 *   exterior plane waves outside; then E(x, y, z) = sum_m p(m, z)
 *   exp(i k s_m . r) on the grid by a separable inverse transform.
 * E_dev: caller-owned device buffer [3][fz][fy][fx], complex128 for SCW_FP64,
 * complex64 otherwise. `hip_stream` is a hipStream_t (NULL = default stream).
 * The call enqueues work and returns; the first call for a new grid,
 * precision or kernel configuration builds a plan (device tables and
 * workspaces) synchronously. A plan is never rebuilt or freed before
 * scw_solution_free, so work already enqueued, or captured in a HIP graph,
 * stays valid while later calls use other grids, precisions or
 * configurations (or scw_tune_synthesis runs). Calls that use the same plan
 * share its workspaces: order them on one stream, or synchronise between
 * streams, so that they do not overlap in time. */
int scw_synthesize(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid,
                   int precision, void* E_dev, void* hip_stream);

/* Allocation-free form of scw_synthesize, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc. It computes the same field on the same kernels,
 * with the plan's tables (plane tasks, exterior planes, twiddles) built on
 * the device by a kernel and every workspace placed in one static device
 * array of SCW_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.
 * It allocates nothing, copies nothing from the host and never blocks: all
 * work is enqueued on hip_stream.
 *   precision  SCW_FP64 or SCW_FP32 (the split modes return SCW_EINVAL);
 *   E_dev      caller-owned device buffer as for scw_synthesize.
 * The transform is the one scw_synthesize would choose, except that a grid
 * on which it would choose the matrix-core form gets the factored form when
 * it applies and the direct sum otherwise. Every call on one GPU shares that
 * GPU's array: calls that overlap in time (two streams, two contexts, two
 * threads) race and give wrong fields; order them. Errors: SCW_EINVAL for a
 * null argument, a bad grid or precision, or a problem and grid whose tables
 * and workspaces need more than SCW_NOALLOC_SCRATCH_BYTES (the message gives
 * the size); SCW_EHIP if the array could not be attached at scw_create. */
#define SCW_NOALLOC_SCRATCH_BYTES (32u << 20)
int scw_synthesize_noalloc(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid,
                           int precision, void* E_dev, void* hip_stream);

/* Periodic display (Sec. 4.6: the field of one unit cell applied to the
 * whole periodic pattern): the field over tx x ty lateral periods. Every
 * plane wave of Eq. 10 has a lattice frequency, so the field repeats with the
 * period; one period is synthesised on `grid` and copied tx x ty times.
 * E_dev: caller-owned device buffer [3][fz][ty*fy][tx*fx] (complex128 for
 * SCW_FP64, complex64 otherwise); column tx'*fx + f of a row lies at
 * x = tx'*X + f*X/fx. Work is enqueued on hip_stream; the period is held in a
 * workspace of the solution's plan for this grid and precision, so calls on
 * one solution must be ordered. Errors: as scw_synthesize, and SCW_EINVAL
 * for tx or ty below 1. */
int scw_synthesize_tiled(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int tx,
                         int ty, int precision, void* E_dev, void* hip_stream);

/* A large sample composed of small patches in two dimensions (Sec. 1): px x
 * py solutions, patches[j*px + i] for the patch at lateral position (i, j),
 * each solved as its own periodic unit cell, each synthesised on `grid` over
 * its own period and written side by side: patch (i, j) fills columns
 * i*fx .. (i+1)*fx - 1 and rows j*fy .. (j+1)*fy - 1 of E_dev
 * [3][fz][py*fy][px*fx]. Coupling across patch borders is not modelled (each
 * patch sees its own periodic continuation); identical patches give exactly
 * the tiled field of one. Patches may differ in truncation and lateral
 * period. Errors: as scw_synthesize, SCW_EINVAL for a null patch or counts
 * below 1. */
int scw_synthesize_composed(scw_ctx* ctx, scw_solution* const* patches, int px, int py,
                            const scw_grid* grid, int precision, void* E_dev,
                            void* hip_stream);

/* Kernel configuration of scw_synthesize for one solution. Fields left 0
 * take the library's choice: a configuration found by scw_tune_synthesis for
 * the same shape on this context, else the built-in default.
 *   modal_rows  rows of the synthesis matrix per wavefront in the modal sum
 *               (FP32 and split modes): 2, 4, 8 or 16, lowered where needed
 *               so that rows x planes-per-task stays <= 32;
 *   transform   how Eq. 10 is evaluated: SCW_XFORM_FFT (Horner x pass and a
 *               factored y pass fy = R * P; FP64/FP32, fy a power of two,
 *               V <= 32), SCW_XFORM_MFMA (y pass as a GEMM on the matrix
 *               cores; the only transform of the split modes), or
 *               SCW_XFORM_DIRECT (Horner in x and y);
 *   fft_radix   P of the factored y pass (2 .. 32, a power of two);
 *   tiles       row tiles per plane (DIRECT), plane-components per block
 *               (MFMA) or columns per block, 32 or 64 (FFT); 0 = automatic.
 * A configuration the solution's shape or precision cannot run makes the
 * next scw_synthesize fail with SCW_EINVAL. cfg = NULL clears it. */
typedef enum {
  SCW_XFORM_AUTO = 0,
  SCW_XFORM_FFT = 1,
  SCW_XFORM_MFMA = 2,
  SCW_XFORM_DIRECT = 3
} scw_transform;

typedef struct {
  int modal_rows;
  int transform;  /* scw_transform */
  int fft_radix;
  int tiles;
} scw_synth_config;

int scw_synthesis_configure(scw_solution* sol, const scw_synth_config* cfg);

/* Autotuner result. Times are mean milliseconds per call, measured with HIP
 * events on the caller's stream. */
typedef struct {
  int n_candidates;          /* configurations timed */
  double default_ms;         /* the built-in default, same sweep */
  double best_ms;            /* the chosen configuration */
  scw_synth_config config;   /* chosen synthesis configuration */
  int batch_radix;           /* batched synthesis: chosen P of the y pass */
  int batch_blocks_per_cu;   /* batched synthesis: persistent blocks per CU */
  int batch_chunk;           /* batched synthesis: work items per queue grab */
} scw_tune_report;

/* Time the candidate kernel configurations of scw_synthesize for this
 * solution, grid and precision (modal-sum row blocking, then transform kind,
 * radix and tiling, each stage timed alone with `reps` calls after one
 * warm-up), keep the fastest in the context, keyed by problem shape, grid and
 * precision, and report it. Later calls of that shape and precision use it
 * wherever their solution's explicit configuration leaves a field 0; the
 * solution's own configuration is left as it was. E_dev is a caller-owned output
 * buffer as for scw_synthesize and holds the synthesized field on return.
 * Synchronises `hip_stream`. */
int scw_tune_synthesis(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                       void* E_dev, void* hip_stream, int reps, scw_tune_report* report);

/* The field on a lateral slice instead of a volume: Eq. 10 evaluated on an
 * x-z plane (axis SCW_SLICE_XZ: x_f = f X / n for f < n, at y = position)
 * or a y-z plane (SCW_SLICE_YZ: y_g = g Y / n, at x = position), for the fz
 * cell-centred planes z_j = z_begin + (j + 1/2)(z_end - z_begin)/fz, inside
 * or outside the sample as for scw_synthesize (X, Y: the lateral period;
 * position: any real value, in the units of lambda). Per plane and
 * component the spectrum is summed over the other lateral frequency with the
 * phase of `position`, then over the kept one on the n samples.
 * Precision SCW_FP64 (E_dev complex128) or SCW_FP32 (complex64); E_dev
 * receives [3][fz][n], caller-owned. Enqueued on hip_stream after the
 * solution's slice plan is built (the first call for a slice shape
 * synchronises the stream). Errors: SCW_EINVAL for a null argument, an
 * unknown axis, n < 1, fz < 1 or above 21845, z_end <= z_begin, or another
 * precision. */
enum { SCW_SLICE_XZ = 0, SCW_SLICE_YZ = 1 };
typedef struct {
    int axis;          /* SCW_SLICE_XZ or SCW_SLICE_YZ */
    double position;   /* y of an x-z slice, x of a y-z slice */
    int n;             /* samples along the kept lateral axis */
    int fz;
    double z_begin, z_end;
} scw_slice;
int scw_synthesize_slice(scw_ctx* ctx, scw_solution* sol, const scw_slice* slice, int precision,
                         void* E_dev, void* hip_stream);

/* Coherent imaging through an ideal objective (Sec. 1: an optical system
 * applied to the field's plane-wave spectrum): the field of scw_synthesize on
 * `grid`, with every mode whose direction sine |s_bar| = sqrt(s_x^2 + s_y^2)
 * exceeds `na` removed before Eq. 10 (the objective's coherent transfer
 * function, unit magnification), and its intensity |E_x|^2 + |E_y|^2 +
 * |E_z|^2. E_dev as for scw_synthesize (it receives the filtered field);
 * I_dev, when not null, receives [fz][fy][fx] float (double for SCW_FP64),
 * caller-owned. Errors as scw_synthesize, and SCW_EINVAL for na < 0 or not
 * finite. */
int scw_synthesize_image(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                         double na, void* E_dev, void* I_dev, void* hip_stream);

/* The field of scw_synthesize with a transfer function applied to the
 * plane-wave spectrum before Eq. 10 (Sec. 1: optical elements act linearly on
 * the spectrum): on every plane, each mode m's coefficients are multiplied by
 * H[m]. Examples: apodization or phase plates; an ideal objective,
 * H[m] = [|s_bar_m| <= NA] (as scw_synthesize_image); propagation by dz in a
 * half-space whose s_z is s_z,m, H[m] = exp(i k s_z,m dz). H_dev: device
 * complex128 [M] in mode order m = (v + V/2) U + (u + U/2), caller-owned,
 * read by the kernels enqueued on hip_stream. E_dev and I_dev as for
 * scw_synthesize_image. Errors as scw_synthesize, and SCW_EINVAL for a null
 * H_dev. */
int scw_synthesize_filtered(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                            const void* H_dev, void* E_dev, void* I_dev, void* hip_stream);

/* Convenience: scw_solve + scw_synthesize + scw_solution_free. */
int scw_field(scw_ctx* ctx, const scw_problem* prob, const scw_grid* grid,
              int precision, void* E_dev, void* hip_stream);

/* Batched synthesis: many solved problems (for example wavelengths x patches
 * with different truncation orders U x V) on one shared grid, in one
 * persistent kernel launch that is captured in a HIP graph and replayed.
 * Every plane of `grid` must lie outside every job's sample (above z0 or
 * below its bottom surface): the field there follows from the exterior
 * coefficients alone (Eq. 9, then Eq. 10). Requirements: precision
 * SCW_FP32; U, V <= 31; grid->fy a power of two >= 2 with
 * 256 * fy / 32 + 24 * max(U V) <= 48 KiB (the per-block tables of the
 * factored y pass and the spectra of one plane; fy <= 2048 always fits).
 * `jobs` are borrowed: they must outlive the batch. E_dev receives
 * [njobs][3][fz][fy][fx] complex64, jobs in the order given.
 * scw_batch_launch enqueues the graph on `hip_stream` (NULL = default
 * stream); the first launch with a given E_dev captures the graph. Launches of
 * one batch must not overlap (they share a work counter). */
typedef struct scw_batch scw_batch;
int scw_batch_plan(scw_ctx* ctx, scw_solution* const* jobs, int njobs, const scw_grid* grid,
                   int precision, scw_batch** out);
int scw_batch_launch(scw_batch* batch, void* E_dev, void* hip_stream);
void scw_batch_free(scw_batch* batch);
/* Time the batched kernel over its tunable shapes (P of the factored y
 * pass, persistent blocks per CU, work items per queue grab), keep the fastest for later launches of
 * this batch (the graph is captured again) and for batches of the same grid
 * on this context, and report it. E_dev as for scw_batch_launch; it holds
 * the batch's field on return. Synchronises `hip_stream`. */
int scw_batch_tune(scw_batch* batch, void* E_dev, void* hip_stream, int reps,
                   scw_tune_report* report);
/* Set the batched kernel's shape explicitly: radix P of the factored y pass
 * (a power of two in [2, min(32, fy)] whose per-block tables fit, see above),
 * persistent blocks per CU (1..64) and work items per queue grab (1..1024).
 * Later launches capture the graph again. Returns SCW_EINVAL (the batch
 * unchanged) for a shape outside these ranges. Host-only; no device work. */
int scw_batch_configure(scw_batch* batch, int radix, int blocks_per_cu, int chunk);

/* Spectral-convolution surrogate of the transmitted field (Eq. 9 below the
 * sample) for one patch family: 8 x 32 x 32 voxels at pitch lambda/4
 * (lambda = 1), index 1 above and below, normal x-polarised plane wave of unit
 * amplitude, 15 x 15 band (U = V = 15). Input patches are complex64
 * [B][8][32][32]; encoded inputs are float [B][16][32][32]; outputs are the
 * coefficients p_trn as complex64 [B][3][15][15] (component, then mode order
 * of Sec. 2.2). The network is a lift to 32 channels, four Fourier
 * layers (truncated DFT2 on |ky| <= 8, 0 <= kx <= 8, per-mode complex 32 x 32
 * mixing, real inverse DFT2, plus a pointwise 32 x 32 map and bias, GELU
 * between layers) and a per-mode complex head on the 15 x 15 band.
 * Parameters are one flat FP32 array of scw_sur_param_count() values. The
 * training loss is sum |out - target|^2 / sum |target|^2 over the batch.
 * Device pointers are caller-owned; every call may be enqueued on `stream`
 * except those that return host values, which synchronise it. */
typedef struct scw_sur scw_sur;
long long scw_sur_param_count(void);
int scw_sur_create(scw_ctx* ctx, int max_batch, unsigned long long seed, scw_sur** out);
void scw_sur_free(scw_sur* sur);
int scw_sur_get_params(scw_sur* sur, float* host);
int scw_sur_set_params(scw_sur* sur, const float* host);  /* also resets Adam state */
/* Arithmetic of the network's matrix products: bf16 = 0 (default) computes
 * them in FP32 on the vector units; bf16 = 1 rounds both operands of every
 * product to bf16 and runs it on the matrix cores with FP32 accumulation
 * (parameters, Adam state and the elementwise steps stay FP32). In that mode
 * inference (scw_sur_forward, scw_sur_infer_checked) also stores the
 * activations and spectra between its kernels in bf16: each is used only as
 * a rounded operand, so the outputs are those of the FP32-storage kernels up
 * to the order of the FP32 sums; training keeps FP32 storage. */
int scw_sur_set_compute(scw_sur* sur, int bf16);
int scw_sur_encode(scw_sur* sur, const void* n_dev, int batch, void* x_dev, void* stream);
int scw_sur_forward(scw_sur* sur, const void* x_dev, int batch, void* out_dev, void* stream);
/* loss and, when grad_host is not NULL, dL/dparams (complex entries as
 * dL/dRe + i dL/dIm) copied to the host */
int scw_sur_loss_grad(scw_sur* sur, const void* x_dev, const void* target_dev, int batch,
                      double* loss, float* grad_host, void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8); loss may be NULL */
int scw_sur_train_step(scw_sur* sur, const void* x_dev, const void* target_dev, int batch,
                       float lr, double* loss, void* stream);
/* Surrogate inference of host patches (complex128 [B][8][32][32]) with a CWT
 * check on n_check seeded patches, solved together by scw_solve_batch (device
 * eigensolver, SCW_ROUTE_STABLE_DEVICE). When their rel-L2 exceeds tol,
 * every patch is solved by CWT the same way instead and *fell_back = 1.
 * out_host receives complex128 [B][3][15][15]. Synchronous. */
int scw_sur_infer_checked(scw_ctx* ctx, scw_sur* sur, const double* n_host, int batch,
                          int n_check, unsigned long long seed, double tol, double* out_host,
                          int* fell_back, double* check_err);

/* The stages of scw_synthesize (Eq. 10 per plane after Eqs. 30-34 / Eq. 9),
 * selectable for timing single stages and for callers that keep one plane
 * spectrum and transform it more than once. */
enum scw_stage_mask {
    SCW_STAGE_MODAL = 1,      /* per-layer modal sum into the plan's spectra */
    SCW_STAGE_EXTERIOR = 2,   /* plane-wave spectra of planes outside the sample */
    SCW_STAGE_TRANSFORM = 4,  /* inverse transform of the plan's spectra into E */
    SCW_STAGE_ALL = 7
};
/* scw_synthesize restricted to the stages in `stages` (a non-zero mask of
 * scw_stage_mask). The spectra live in the workspace of the (solution, grid,
 * precision) plan, which the first call builds: a call without
 * SCW_STAGE_MODAL / SCW_STAGE_EXTERIOR transforms whatever the last call that
 * ran them left there (undefined before any). E_dev as for scw_synthesize;
 * it is written only with SCW_STAGE_TRANSFORM. SCW_STAGE_ALL is exactly
 * scw_synthesize. SCW_EINVAL for a mask outside 1..7. */
int scw_synthesize_stages(scw_ctx* ctx, scw_solution* sol, const scw_grid* grid, int precision,
                          int stages, void* E_dev, void* hip_stream);

/* Per-stage timing of scw_synthesize with HIP events recorded on the
 * synthesis stream between its kernels. scw_profile_begin enables recording
 * for up to `max_calls` following scw_synthesize calls on this context;
 * scw_profile_end waits for those events and writes the mean duration of each
 * stage in milliseconds to stage_ms[0 .. n_stages-1] (n_stages <= 8) and the
 * number of calls recorded to *calls; it then disables recording. Stage names
 * come from scw_stage_name. */
int scw_profile_begin(scw_ctx* ctx, int max_calls);
int scw_profile_end(scw_ctx* ctx, double* stage_ms, int n_stages, int* calls);
const char* scw_stage_name(int stage);

/* Bytes of HBM the synthesis of `grid` must move at `precision`: the
 * per-layer synthesis matrices of the layers the grid touches, once each, plus
 * the output field. Used for roofline reporting. */
double scw_synthesis_bytes(const scw_solution* sol, const scw_grid* grid,
                           int precision);

#ifdef __cplusplus
}
#endif
#endif /* SCW_H */

/*
 * pwf.h - C ABI of the preconditioned Wirtinger flow (PWF) hot path on AMD
 * Instinct MI355X (gfx950).
 *
 * The operations follow "Speckle-based X-ray microtomography via
 * preconditioned Wirtinger flow" (Lee, Hugonnet, Lim, Park, arXiv 2503.20146):
 * the forward model of Eq. 1 (PhysicalModel in Algorithm S2), the loss of
 * Eq. 2, the Wirtinger derivative, preconditioner and regulariser of
 * Algorithm S2, and the Nesterov-accelerated loop of Algorithm S1.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Fields are row-major [ny][nx] with x fastest.  Complex fields are
 *   interleaved single precision (re, im) pairs ("complex64"); intensities
 *   are float32.  Every data pointer is a device pointer unless stated.
 * - A call works on a batch of n independent instances (projections or
 *   regions of interest).  Per-instance arguments are arrays of n pointers
 *   that live in HOST memory and point to device buffers; problems are an
 *   array of n descriptors in host memory.  Instances may share a diffuser.
 * - Supported grids: nx, ny in {128, 256, 512, 1024, 2048} (independently).
 * - The caller owns every device buffer, including the workspace whose size
 *   pwf_workspace_size() returns.  The library allocates only its own
 *   immutable twiddle tables (once per device) and never on the hot path.
 * - Calls are asynchronous on `stream` (a hipStream_t; NULL is the default
 *   stream).  Host pointer arrays may be reused as soon as a call returns.
 * - Errors in arguments are reported synchronously through the return value
 *   before any work is queued.  A non-finite loss found on the GPU sets a
 *   device flag that pwf_sync_status() reports.  Nothing aborts or throws
 *   across this boundary.
 * - Calls that overlap on one workspace race; use one workspace per stream.
 */
#ifndef PWF_H_
#define PWF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PWF_OK = 0,
  PWF_ERR_ARG = -1,        /* NULL or non-finite argument, bad count */
  PWF_ERR_SIZE = -2,       /* grid side outside the supported set */
  PWF_ERR_EVANESCENT = -3, /* lambda / (2 p) >= 1/sqrt(2): evanescent bins */
  PWF_ERR_WORKSPACE = -4,  /* workspace NULL, misaligned or too small */
  PWF_ERR_HIP = -5,        /* a HIP runtime call failed */
  PWF_ERR_NONFINITE = -6,  /* the loss became NaN or Inf on the GPU */
  PWF_ERR_SCRATCH = -7     /* batch too large for the allocation-free variant */
} pwf_status;

/* Imaging geometry (Results, PWF subsection; Fig. 1a): grid, pixel pitch p at
 * the detector, X-ray wavelength lambda, sample-to-diffuser distance L1 and
 * diffuser-to-detector distance L2, all in SI units.  Distances may be 0
 * (identity propagation) but not negative. */
typedef struct {
  int32_t nx, ny;
  double pixel_m;
  double wavelength_m;
  double z1_m, z2_m;
} pwf_geometry;

/* Partial coherence of the source (Methods, "Intensity optical transfer
 * function (IOTF)", Eqs. 3-5), in one of three forms (`kind`):
 *   PWF_SRC_GAUSS      Gaussian intensity point spread function of standard
 *                      deviation sigma_x_px, sigma_y_px (pixels at the
 *                      detector), i.e. Eq. 4 with x_coh = 2 sqrt(pi) sigma p;
 *                      0 means a fully coherent source.
 *   PWF_SRC_COHERENCE  the coherence lengths x_coh_m, y_coh_m (metres) of
 *                      Eqs. 4-5, as pwf_fit_coherence returns them (Eq. 3);
 *                      0 means coherent along that axis.
 *   PWF_SRC_IOTF       the IOTF itself, separable and sampled on the DFT bins:
 *                      IOTF(kx, ky) = iotf_x[kx] iotf_y[ky], with iotf_x a
 *                      device float32 array of nx values and iotf_y of ny
 *                      (bin k > n/2 stands for frequency k - n).  Both arrays
 *                      must be even (iotf[k] == iotf[n - k]) and finite; the
 *                      library does not read device memory to check, and
 *                      non-finite values surface as PWF_ERR_NONFINITE.  The
 *                      arrays are read by every call that uses the problem.
 * Unused members are ignored.  The regulariser's sample transfer function
 * (Eq. 14) is STF = IOTF^(2 gamma) in every form, the relation Eqs. 5 and 14
 * give for the Gaussian model (negative IOTF samples count as 0 there). */
typedef enum { PWF_SRC_GAUSS = 0, PWF_SRC_COHERENCE = 1, PWF_SRC_IOTF = 2 } pwf_source_kind;

typedef struct {
  int32_t kind;
  double sigma_x_px, sigma_y_px;
  double x_coh_m, y_coh_m;
  const float* iotf_x;
  const float* iotf_y;
} pwf_source;

/* Solver parameters (Results, PWF subsection; Methods, Eqs. 11, 14-15).
 *   eta            step size of the gradient step (Algorithm S1)
 *   alpha_re/im    complex regularisation parameter alpha
 *   gamma          oversampling ratio of the sample transfer function
 *   precond_scale  s_P in P^-1_k = s_P / (u^2 + v^2), u, v in cycles/pixel
 *   precondition   0 skips the preconditioner (Im g is used unfiltered) */
typedef struct {
  double eta;
  double alpha_re, alpha_im;
  double gamma;
  double precond_scale;
  int32_t precondition;
} pwf_params;

/* One instance: geometry, source, parameters and the diffuser transmission
 * t (device, complex64 [ny][nx]; Methods, "Diffuser transmission function"). */
typedef struct {
  pwf_geometry geom;
  pwf_source source;
  pwf_params params;
  const void* diffuser;
} pwf_problem;

/* Iterate of Algorithm S1 for pwf_step, in caller memory (all device,
 * complex64 [ny][nx]):
 *   psi      extrapolated iterate psi in real space (read/written)
 *   psi_hat, z_hat
 *            spectra of the last two gradient-step iterates z_k and z_{k-1}
 *            in the library's frequency layout: z_k is in psi_hat for even k
 *            and in z_hat for odd k, and pwf_step overwrites z_{k-1} with
 *            z_{k+1}.  The spectrum of psi_k, z_k + beta_{k-1} (z_k - z_{k-1}),
 *            is formed from them when needed; pwf_state_init sets both to the
 *            spectrum of psi_0 (z_{-1} = z_0 = psi_0).
 *   y_hat    spectrum of the measured speckle y in half form: y is real, so
 *            row ky keeps kx = 1 .. nx/2 - 1 at position kx and the real
 *            x-spectra at kx = 0 and nx/2, packed as one complex column, at
 *            position 0 (transformed along y together); positions nx/2 .. nx-1
 *            of each row are unused
 *   k        iterations done so far (host value, advanced by pwf_step)
 * The frequency layout is row-major [r][s]: column kx of the 2-D DFT sits at
 * s = 2 kx for 0 < kx < nx/2, at s = 2 (nx - kx) + 1 for nx/2 < kx < nx, at
 * s = 0 for kx = 0 and at s = 1 for kx = nx/2, so that kx and -kx are
 * neighbours.  Row r holds ky = r for ny < 512; for ny >= 512 the column
 * transform is split into its even and odd frequencies (one radix-2 stage in
 * the row sweeps, two ny/2-point halves in the column sweeps), and row
 * r = p ny/2 + j holds ky = 2 j + p (p = 0, 1). */
typedef struct {
  void* psi;
  void* psi_hat;
  void* z_hat;
  void* y_hat;
  int32_t k;
} pwf_state;

/* Human-readable text of a status code (static storage). */
const char* pwf_status_string(int32_t status);

/* Library version as 10000*major + 100*minor + patch. */
int32_t pwf_version(void);

/* Bytes of workspace that any call below needs for this batch; 0 if the
 * problems are invalid.  The workspace must be 256-byte aligned. */
size_t pwf_workspace_size(const pwf_problem* problems, int32_t n);

/* Forward model, Eq. 1 / PhysicalModel: f = |P2{t P1{exp(psi)}}|^2 * IPSF.
 *   psi[i]   device complex64 [ny][nx], the complex phase -mu + i phi
 *   f_out[i] device float32 [ny][nx] */
pwf_status pwf_forward(const pwf_problem* problems, int32_t n, const void* const* psi, float* const* f_out,
                       void* workspace, size_t workspace_bytes, void* stream);

/* RMSE image of the retrieved fields (Methods, "Reconstruction procedure"):
 * out[i] = 100 |y_i - f(psi_i)| / ref_mean[i], the misfit of the forward model
 * in percent of the reference speckle's mean intensity (one measurement, so
 * the root-mean-square over measurements is the absolute value).  y: device
 * float32 [ny][nx]; ref_mean: host float64 [n] (> 0); out: device float32. */
pwf_status pwf_rmse_image(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                          const double* ref_mean, float* const* out, void* workspace, size_t workspace_bytes,
                          void* stream);

/* Loss (Eq. 2), Wirtinger derivative g (WirtingerDerivative of Algorithm S2,
 * normalised by max|t|^2) and update direction d = Preconditioner(g) +
 * Regularizer(psi) at psi.  The real gradient of the loss is
 * dL/dRe psi + i dL/dIm psi = 4 max|t|^2 g.
 *   y[i]        device float32 [ny][nx], measured speckle
 *   g_out[i]    device complex64 or NULL (array itself may be NULL)
 *   d_out[i]    device complex64 or NULL (array itself may be NULL)
 *   loss_out    device float64 [n] or NULL
 * With neither g nor d requested only the forward model and the loss run. */
pwf_status pwf_gradient(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                        void* const* g_out, void* const* d_out, double* loss_out, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Loss (Eq. 2) and its real gradient dL/dRe psi + i dL/dIm psi = 4 max|t|^2 g
 * at psi, for automatic-differentiation wrappers (the forward fields are
 * recomputed, nothing is kept between calls).
 *   grad_out[i]  device complex64 [ny][nx]
 *   loss_out     device float64 [n] or NULL */
pwf_status pwf_loss_grad(const pwf_problem* problems, int32_t n, const void* const* psi, const float* const* y,
                         void* const* grad_out, double* loss_out, void* workspace, size_t workspace_bytes,
                         void* stream);

/* pwf_loss_grad for callers that cannot allocate device memory (code under
 * stream or graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, bit for bit, with the workspace in a static
 * buffer of the library instead of caller memory, so there are no workspace
 * arguments and nothing is allocated.  The buffer is a fixed 64 MiB per GPU
 * (the first 1 MiB holds the twiddle tables), held from the library's load
 * until the process ends; a batch needs 4 fields per instance plus small
 * tables (one 1024^2 instance takes ~32 MiB), at most 64 instances:
 * pwf_loss_grad_noalloc_limit() returns the bytes available, and larger
 * batches get PWF_ERR_SCRATCH before any work is queued.  The first call on a
 * device resolves the buffer's address there and copies the tables in
 * (synchronously).  Every call on a GPU uses that GPU's one buffer: calls that
 * overlap on one GPU (on different streams or threads without ordering)
 * race; calls in one stream are ordered. */
size_t pwf_loss_grad_noalloc_limit(void);
pwf_status pwf_loss_grad_noalloc(const pwf_problem* problems, int32_t n, const void* const* psi,
                                 const float* const* y, void* const* grad_out, double* loss_out, void* stream);

/* Prepare states for pwf_step: psi = psi0 (or 0 when psi0 or psi0[i] is NULL),
 * z = 0, momentum scalar 1, k = 0 (Algorithm S1 initialisation), and the
 * spectrum of y.  states is a host array of n pwf_state. */
pwf_status pwf_state_init(const pwf_problem* problems, int32_t n, pwf_state* states, const void* const* psi0,
                          const float* const* y, void* workspace, size_t workspace_bytes, void* stream);

/* One iteration of Algorithm S1 on every instance: loss at the entering psi,
 * gradient, direction, z = psi - eta d, Nesterov extrapolation.  Advances
 * states[i].k.  loss_out: device float64 [n] or NULL. */
pwf_status pwf_step(const pwf_problem* problems, int32_t n, pwf_state* states, double* loss_out,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Algorithm S1 from psi = 0 for `iters` iterations per instance.
 *   psi_out[i]  device complex64 [ny][nx]: psi after the last iteration
 *   loss_hist   device float64 [n * iters] or NULL: loss at the psi entering
 *               each iteration, instance-major
 *   corr_tol    <= 0: fixed iteration count.  In (0, 1): stopping rule of the
 *               Methods section ("Reconstruction procedure"; the paper uses
 *               10^-0.00001): an instance stops after the first iteration whose
 *               new exp(psi) has normalised correlation |<x_k, x_k-1>| /
 *               (|x_k| |x_k-1|) above corr_tol with the previous one (FP64
 *               sums); its later sweeps are skipped, psi_out holds that iterate
 *               and loss_hist entries past its stop are left untouched.  The
 *               call then synchronises on `stream` to fill iters_done.
 *   iters_done  host int32 [n] or NULL: iterations done per instance
 * With graph mode on (the default) the whole loop is one hipGraph launch. */
pwf_status pwf_solve(const pwf_problem* problems, int32_t n, const float* const* y, void* const* psi_out,
                     int32_t iters, double corr_tol, double* loss_hist, int32_t* iters_done, void* workspace,
                     size_t workspace_bytes, void* stream);

/* Workspace bytes for pwf_solve_joint (pwf_workspace_size plus one field per
 * instance and the diffuser-step reductions); 0 if the batch is invalid. */
size_t pwf_joint_workspace_size(const pwf_problem* problems, int32_t n);

/* Joint diffuser refinement (Results, "Diffuser transmission function";
 * Fig. S12): Algorithm S1 on every instance, as pwf_solve with a fixed
 * iteration count, and after each iteration a gradient step on the shared
 * diffuser t:
 *   t <- t - eta_t sum_j conj(u1_j) a2_j / sum_j max|u1_j|^2
 * where u1_j is instance j's field incident on the diffuser and a2_j its
 * misfit back-propagated to the diffuser plane (conj(u1) a2 = dL/dt*; the
 * paper gives no rule, this is the library's reading).  All instances must
 * share one diffuser pointer and one grid shape (else PWF_ERR_ARG); that
 * device array is READ AND WRITTEN in place and holds the refined t on
 * return.  eta_t >= 0 (0: t unchanged, the result equals pwf_solve's).
 * Sums over instances run in instance order in FP64 (deterministic).
 * workspace: pwf_joint_workspace_size bytes. */
pwf_status pwf_solve_joint(const pwf_problem* problems, int32_t n, const float* const* y, void* const* psi_out,
                           int32_t iters, double eta_t, double* loss_hist, void* workspace, size_t workspace_bytes,
                           void* stream);

/* Reference GPU path for speed comparisons: the literal Algorithm S1/S2 on
 * ONE instance, one kernel per operation (16 two-dimensional FFTs plus
 * element-wise kernels per iteration), no fusion, no batching, no graph.
 * Same arguments and results as pwf_solve with n = 1. */
pwf_status pwf_solve_plain(const pwf_problem* problem, const float* y, void* psi_out, int32_t iters,
                           double* loss_hist, void* workspace, size_t workspace_bytes, void* stream);

/* Timing aid: launch sweep `sweep` (0..11, the steps of one fused iteration
 * in order: S0 psi update, S1 x Q_L1, S2 x t, S3 x Q_L2, S4 |v|^2, S5 blur and
 * loss, S6 back-blur, S7 x conj Q_L2, S8 x conj t, S9 x conj Q_L1, S10
 * gradient, S11 direction and Nesterov step) `reps` times over the batch.  It
 * reuses the fields that a previous pwf_solve with the same problems left in
 * `workspace`; the fields it rewrites are meaningless afterwards.  Returns
 * PWF_ERR_ARG for a sweep outside 0..11 or reps < 1. */
pwf_status pwf_bench_sweep(const pwf_problem* problems, int32_t n, int32_t sweep, int32_t reps, void* workspace,
                           size_t workspace_bytes, void* stream);

/* Tile width (columns per workgroup) of the column sweep S`sweep` of the
 * iteration (sweep = 1, 3, 5, 7, 9 or 11; -1: every column sweep, including
 * those of pwf_forward / pwf_gradient) for grid side n.  Two widths are
 * compiled per side (128: 32/16, 256: 16/32, and over one half of the split
 * column transform of the larger sides (see the state layout above) 512:
 * 16/32, 1024: 16/8, 2048: 8/16); 0 restores the default.  PWF_ERR_SIZE / PWF_ERR_ARG for an
 * unsupported side, sweep or width.  Process-wide; applies to calls issued
 * afterwards. */
pwf_status pwf_set_column_tile(int32_t n, int32_t sweep, int32_t width);

/* Current tile width of column sweep S`sweep` for side n (0 if unsupported). */
int32_t pwf_column_tile(int32_t n, int32_t sweep);

/* FFT plan of the row sweep S`sweep` of the iteration (sweep = 0, 2, 4, 6, 8
 * or 10) for grid side n: plan 0 is the side's default radix plan, 1 its
 * alternative plan with fewer elements per lane (e.g. 32x32 and 16x16x4 at
 * 1024), 2 (sides 1024 and 2048 only) the alternative's radices with the
 * small radix first (4x16x16 at 1024, 8x16x16 at 2048); -1 restores the
 * built-in choice.  PWF_ERR_SIZE / PWF_ERR_ARG for an unsupported side,
 * sweep or plan.  Process-wide; applies to calls issued afterwards. */
pwf_status pwf_set_row_plan(int32_t n, int32_t sweep, int32_t plan);

/* Current plan (0, 1 or 2) of row sweep S`sweep` for side n; -1 if unsupported. */
int32_t pwf_row_plan(int32_t n, int32_t sweep);

/* Autotuner: for each grid shape in the batch, time each of the twelve
 * sweeps of the iteration with every compiled tile width (column sweeps) or
 * radix plan (row sweeps), `reps` launches each, HIP events on `stream`,
 * synchronous, and keep the fastest per sweep, as pwf_set_column_tile /
 * pwf_set_row_plan would.  Clobbers
 * the workspace contents. */
pwf_status pwf_autotune(const pwf_problem* problems, int32_t n, int32_t reps, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Autotuner with a persistent cache: a text file at cache_path (host path,
 * created when missing) keyed by the device's architecture with the library
 * version (e.g. "gfx950/v10301": entries timed on other kernels are not
 * reused), the batch's class mix (its grid shapes and instance counts,
 * marked "/merged" when pwf_set_merged_launch(1) makes the batch launch
 * merged: the tuner then picks among what the merged kernels hold) and the
 * grid side, holding
 * that side's column-tile widths (S1..S11) and row plans (S0..S10).  When
 * every side of the batch has an entry for this architecture and mix, the
 * stored choices are applied and nothing is timed (*tuned = 0, tuned may be
 * NULL); otherwise, or with force != 0, pwf_autotune runs (same arguments)
 * and its choices replace this batch's entries in the file (*tuned = 1).
 * PWF_ERR_ARG when the file cannot be written. */
pwf_status pwf_autotune_cached(const pwf_problem* problems, int32_t n, int32_t reps, const char* cache_path,
                               int32_t force, int32_t* tuned, void* workspace, size_t workspace_bytes,
                               void* stream);

/* Capture pwf_solve's loop in a hipGraph (1, default) or launch eagerly (0). */
void pwf_set_graph_mode(int32_t on);

/* Batches of several grid shapes (pwf_solve): 1 launches each sweep of the
 * iteration once over every size class, each workgroup running the sweep
 * body of its class's side (sides 512, 1024 and 2048; at most 4 classes; a
 * class whose row plan or column tile width the merged kernels do not hold
 * gets a launch of its own in that sweep, and the autotuner, tuning such a
 * batch, keeps to the plans and widths they hold); 0 (default) launches
 * every class separately, the classes' iterations on parallel streams.
 * Results are identical bit for bit.  Process-wide. */
void pwf_set_merged_launch(int32_t on);

/* Wait for `stream` and report PWF_ERR_NONFINITE if a loss computed by the
 * last call that used `workspace` was NaN or Inf, PWF_ERR_HIP on a runtime
 * error, else PWF_OK.  Every loss-computing call clears the flag when it
 * starts. */
pwf_status pwf_sync_status(void* workspace, void* stream);

/* ---------------------------------------------------------------- calibration
 * The steps before the iteration, run once per dataset (Methods, "Intensity
 * optical transfer function (IOTF)", Eq. 3; Results, "Diffuser transmission
 * function"). */

/* Device workspace bytes for pwf_speckle_g2 (independent of the image). */
size_t pwf_speckle_workspace_size(void);

/* Normalised circular autocorrelations of the reference speckle `ref`
 * (device float32 [ny][nx]) along x and along y, each averaged over the other
 * axis: g2x[d] = <I(x,y) I(x+d,y)> / <I>^2 and likewise g2y, d = 0..max_shift
 * (0 <= max_shift <= 32, < nx, ny).  Sums in FP64 in a fixed order
 * (deterministic).  g2x, g2y: HOST float64 [max_shift + 1]; the call
 * synchronises on `stream`.  PWF_ERR_ARG for bad sizes or a non-positive
 * mean, PWF_ERR_WORKSPACE for a missing / misaligned / short workspace. */
pwf_status pwf_speckle_g2(const float* ref, int32_t nx, int32_t ny, int32_t max_shift, double* g2x, double* g2y,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Coherence length from g2 (host arrays, count >= 3 shifts from d = 0) by the
 * Siegert relation and the Gaussian model of Eq. 3 with a free contrast c:
 * least squares of ln(g2(d) - 1) = ln c - pi (d p)^2 / coh^2 over d = 1..K,
 * K the last shift before g2 - 1 first drops below 2% of g2(1) - 1 (d = 0
 * holds the noise variance).  coh_m: metres; contrast may be NULL.  Host-only;
 * PWF_ERR_ARG when fewer than two shifts qualify or the fit does not decay.
 * The fitted lengths go to the iteration as a PWF_SRC_COHERENCE source. */
pwf_status pwf_fit_coherence(const double* g2, int32_t count, double pixel_m, double* coh_m, double* contrast);

/* Diffuser estimate from the reference speckle `ref` (device float32):
 *   t = FreePropagation( sqrt(max(Re F^-1{F{ref} IOTF / (IOTF^2 + eps)}, 0)), -L2 )
 * i.e. Wiener deconvolution by the problem's IOTF, zero phase (the paper
 * fixes the unknown phase of the reference to zero) and back-propagation
 * over L2.  problem->diffuser is not read; t_out: device complex64 [ny][nx].
 * workspace: pwf_workspace_size(problem, 1) bytes.  eps >= 0. */
pwf_status pwf_diffuser_from_reference(const pwf_problem* problem, const float* ref, double eps, void* t_out,
                                       void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- tomography
 * The step after the iteration (Methods, "Reconstruction procedure"). */

/* Workspace bytes for pwf_fbp; 0 when unsupported (1 <= n_proj <= 4096,
 * 64 <= nx <= 1024, ny a positive multiple of 32). */
size_t pwf_fbp_workspace_size(int32_t n_proj, int32_t nx, int32_t ny);

/* Filtered back-projection of n_proj retrieved projections psi[j] (device
 * complex64 [ny][nx], psi = -mu + i phi) taken at angles_rad[j] (host) about
 * the detector's y axis, slice by slice (every detector row y is one
 * parallel-beam sinogram):
 *   vol[y][Z][X] = scale (pi / n_proj) sum_j q_j,y(X cos th_j - Z sin th_j)
 * q: each row zero-padded to the next power of two of 2 nx (at least 64) and
 * circularly convolved with the band-limited (Ram-Lak) ramp h(0) = 1/4,
 * h(odd n) = -1/(pi^2 n^2); detector pixel i at u = i + 1/2 - nx/2, voxel
 * centres X, Z = k + 1/2 - n_out/2 (pixel units), linear interpolation, 0
 * outside the detector.  With scale = lambda / (2 pi p), vol = -beta + i delta.
 * vol_out: device complex64 [ny][n_out][n_out], n_out a multiple of 16.
 * Angles should be equally spaced over [0, pi) for the pi / n_proj weight.
 * FP32 sums.  PWF_ERR_SIZE for unsupported shapes, PWF_ERR_ARG for null or
 * non-finite arguments, PWF_ERR_WORKSPACE for a missing / short workspace. */
pwf_status pwf_fbp(const void* const* psi, int32_t n_proj, int32_t nx, int32_t ny, const double* angles_rad,
                   int32_t n_out, double scale, void* vol_out, void* workspace, size_t workspace_bytes,
                   void* stream);

/* Workspace bytes for pwf_background_quadratic; 0 when unsupported (n a
 * multiple of 16 in [16, 8192], n_slices >= 1). */
size_t pwf_background_workspace_size(int32_t n_slices, int32_t n);

/* Quadratic background removal after tomography (Methods, "Reconstruction
 * procedure"; slow phase variations are weakly constrained by the speckle
 * data, which leaves a smooth per-slice background in the tomogram).
 * vol: device complex64 [n_slices][n][n] (e.g. a pwf_fbp volume, slice-major
 * [y][Z][X]), modified in
 * place.  For every slice, the background area is the set of voxels whose
 * centre lies at distance >= r_bg (voxels) from the rotation axis (the slice
 * centre); the real and imaginary parts are fitted separately by least
 * squares with b = c0 + c1 x + c2 z + c3 x^2 + c4 x z + c5 z^2, where x, z are
 * the voxel-centre coordinates divided by n/2, and b is subtracted from the
 * whole slice.  Sums and coefficients in FP64, in a fixed order (the result is
 * reproducible).  coef_out: optional HOST float64 [n_slices][2][6] (real part,
 * then imaginary part); when given the call synchronises on `stream`.
 * PWF_ERR_ARG when r_bg is negative or not finite or leaves too few background
 * voxels to determine the six coefficients. */
pwf_status pwf_background_quadratic(void* vol, int32_t n_slices, int32_t n, double r_bg, double* coef_out,
                                    void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes for pwf_shell_correlation; 0 when unsupported (n = 128,
 * 256, 512, 1024 or 2048; dims 2 or 3). */
size_t pwf_shell_correlation_workspace_size(int32_t n, int32_t dims);

/* Fourier shell (dims = 3) or ring (dims = 2) correlation of Eq. 16 between
 * the real (part = 0) or imaginary (part = 1) parts of two device complex64
 * arrays g1, g2 of n^dims elements (e.g. two pwf_fbp volumes of n slices):
 *   fsc[kappa] = Re sum G1* G2 / sqrt(sum |G1|^2 sum |G2|^2) over the shell
 *   kappa = round(|k|) of signed index frequencies, kappa = 0 .. n/2.
 * The resolution criterion of the paper is fsc = 1/4 (Eqs. 17-18).  The two
 * real fields, each scaled to unit RMS (which leaves fsc unchanged), are
 * transformed together as one complex field (FP32): a shell where one input's
 * amplitude is a fraction r of the other's carries an absolute error of about
 * 1e-7 / r.  Shell sums in FP64 in a fixed order (bit-reproducible from call
 * to call).  fsc_out: HOST float64 [n/2 + 1]; the call synchronises on
 * `stream`. */
pwf_status pwf_shell_correlation(const void* g1, const void* g2, int32_t n, int32_t dims, int32_t part,
                                 double* fsc_out, void* workspace, size_t workspace_bytes, void* stream);

/* Release the library's twiddle tables and cached graphs. */
void pwf_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* PWF_H_ */

/*
 * qbvm.h - C interface of the MI355X (gfx950) PinT quasi-boundary value solver.
 *
 * Method: J. Liu, "Fast parallel-in-time quasi-boundary value methods for
 * backward heat conduction problems" (arXiv 2107.06381).  Given the noisy final
 * state g_delta of the heat equation z_t = Lap z on Omega=(0,L)^d (d = 1, 2, 3,
 * homogeneous Dirichlet data, Section 1), the library solves the regularised
 * all-at-once system of Section 3:
 *
 *   PinT-QBVM  (Section 3.1, QBVM_PQ): omega = -1/alpha,   f0 = g_delta/(tau alpha)
 *   PinT-MQBVM (Section 3.2, QBVM_PM): omega = -tau/alpha, f0 = g_delta/alpha
 *     (1/tau) y^0 - Lap_h y^0 - (omega/tau) y^N = f0
 *     (1/tau) y^t - Lap_h y^t - (1/tau) y^{t-1} = 0,  t = 1..N
 *
 * with the (2d+1)-point Dirichlet Laplacian Lap_h on m interior points per
 * dimension (h = L/(m+1)), backward Euler with tau = T/n, N = n and
 * N_t = n+1 time levels.  The solve follows the diagonalisation of Section 3.3
 * (eq. "3step"): omega-power scaling and a DFT along time (Step a), N_t
 * independent complex-shifted spatial solves (Step b), and the inverse DFT with
 * the inverse scaling (Step c).
 *
 * Conventions shared by every call:
 *  - All solve data are IEEE double.  Grid functions are stored in C order with
 *    x_1 fastest: index (x_d, ..., x_1); full solutions are y[t][x_d]..[x_1],
 *    t = 0..n, i.e. (n+1) * m^d doubles.
 *  - Pointers documented as DEVICE point to memory on the GPU the plan was made
 *    on; HOST pointers are ordinary CPU memory.  The caller owns every buffer it
 *    passes; the library owns only what a plan allocates.
 *  - Return value 0 (QBVM_OK) on success, a negative QBVM_E* code otherwise.  No
 *    C++ exception crosses this interface.  After QBVM_EHIP the HIP error text is
 *    available from qbvm_last_error().
 *  - A plan is bound to one HIP stream and is not thread safe.  Solves are
 *    enqueued asynchronously on that stream unless stated otherwise.
 *  - Input and output buffers must not alias.
 */
#ifndef QBVM_H
#define QBVM_H

#ifdef __cplusplus
extern "C" {
#endif

#define QBVM_OK            0
#define QBVM_EINVAL       -1  /* invalid argument (sizes, alpha <= 0, NaN, null) */
#define QBVM_ENOMEM       -2  /* device or host allocation failed */
#define QBVM_EHIP         -3  /* a HIP runtime call failed */
#define QBVM_ENOROOT      -4  /* discrepancy principle has no root in the bracket */
#define QBVM_EUNSUPPORTED -5  /* size outside what the kernels support */
#define QBVM_ENOMODEL     -6  /* learned alpha requested but no model was set */
#define QBVM_ENOCONV      -7  /* an iterative Step (b) stopped short of its tolerance */

/* Regularisation variant: PinT-QBVM (Section 3.1) or PinT-MQBVM (Section 3.2). */
#define QBVM_PQ 0
#define QBVM_PM 1

/* What qbvm_solve writes to y. */
#define QBVM_OUT_ALL 0 /* every level: (n+1) * m^d doubles, y[t][x_d]..[x_1]  */
#define QBVM_OUT_Y0  1 /* the reconstruction y^0 only: m^d doubles (Section 5) */
#define QBVM_OUT_YN  2 /* the final level y^N only: m^d doubles              */

/* Size limits of this build.  Within them, a time length n+1 whose FFT core (Rader on n,
 * or Bluestein on a 7-smooth length >= 2(n+1)-1, for lengths with a prime factor above 47)
 * would exceed 4096 points is refused with QBVM_EUNSUPPORTED at plan creation.  Every
 * sine length 2(m+1) within the limits has a transform (its Bluestein form needs a
 * power-of-two core >= 2m+1 only). */
#define QBVM_MAX_NT      4096  /* n + 1, d = 1 */
#define QBVM_MAX_NT_MD   2048  /* n + 1, d = 2, 3 (one time signal and its tables fit in LDS) */
#define QBVM_MAX_M_1D    2047  /* the sine transform of g (length 2(m+1)) serves 1D too */
#define QBVM_MAX_M_2D    2047
#define QBVM_MAX_M_3D    511

/* Number of floats in a learned-alpha model blob (see qbvm_set_alpha_model). */
#define QBVM_MLP_PARAMS   6401
#define QBVM_MODEL_FLOATS 6469
#define QBVM_NFEAT        33

/* A plan holds what one grid fixes (Section 2 discretisation, Section 3.3 factorisation):
 * the stencil eigenvalues, the FFT factorisations and tables of the time length n+1
 * (Steps a and c) and of the sine length 2(m+1) (the Step (b) diagonalisation in
 * 2D/3D), and the solve workspace.  Opaque; created by qbvm_plan. */
typedef struct qbvm_plan_s* qbvm_plan_t;

/* Discretisation (Section 2): d in {1,2,3}; m >= 1 interior points per
 * dimension; n >= 1 backward-Euler steps; domain length L > 0; final time T > 0. */
typedef struct {
  int d;
  int m;
  int n;
  double L;
  double T;
} qbvm_grid;

/* Options of qbvm_choose_alpha (an addition; the paper fixes alpha a priori). */
typedef struct {
  double tau_dp;    /* discrepancy factor: seek D(alpha) = tau_dp * delta (e.g. 1.1) */
  double log10_lo;  /* bisection bracket on log10(alpha), e.g. -20 */
  double log10_hi;  /* e.g. 0 */
  int steps;        /* bisection halvings, e.g. 30 */
  int use_learned;  /* 1: try the plan's network first, bisection on a window miss */
  double win_lo;    /* accept the predicted alpha if win_lo <= D/delta <= win_hi */
  double win_hi;
} qbvm_alpha_opts;

typedef struct {
  double discrepancy;    /* D(alpha_out) in the h^{d/2}-weighted 2-norm */
  double alpha_learned;  /* network prediction (0 if not used) */
  int iterations;        /* discrepancy evaluations performed */
  int used_fallback;     /* 1 if the prediction missed the window and bisection ran */
  int bracket_hit;       /* 1 if the root lies outside the bracket (end returned) */
} qbvm_alpha_info;

/* ---------------------------------------------------------------- plans ---- */

/* Create a plan for one grid (the discretisation of Section 2), bound to hip_stream
 * (a hipStream_t; NULL = the default stream) on the current HIP device.  Builds the
 * FFT factorisations along time (length n+1, the diagonalisation of the
 * omega-circulant time matrix in Section 3.3) and for the sine transforms (length
 * 2(m+1), the eigenbasis of the Dirichlet stencil used in Step (b)), uploads
 * twiddle, Rader/Bluestein and eigenvalue tables, and allocates the workspace.
 * *out receives the plan; on error *out is NULL. */
int qbvm_plan(qbvm_plan_t* out, const qbvm_grid* grid, void* hip_stream);

/* Release a plan and its device memory (waits for its stream).  NULL is a no-op. */
void qbvm_plan_destroy(qbvm_plan_t p);

/* Re-bind a plan to another stream. */
int qbvm_plan_set_stream(qbvm_plan_t p, void* hip_stream);

/* Device bytes held by the plan (tables + workspace). */
long long qbvm_plan_workspace_bytes(qbvm_plan_t p);

/* Autotuner (an addition): for the power-of-two kernels of this plan's shape, time
 * every kernel variant (complex values per lane, signals per workgroup) of the
 * sine passes over the levels, of the time transform and of the general
 * right-hand side's time transform on a scratch array of the full solution size,
 * and keep the fastest in the plan.  Results are also
 * cached per (device, kernel role, transform length) and used as the defaults of
 * later plans.  The plan's current variant is kept unless another is more than 3%
 * faster.  Synchronous; allocates and frees (n+1) m^d doubles of scratch.
 * ms_out (HOST, may be NULL) receives 30 timings in milliseconds (-1 where not
 * applicable): rows variants 0, 1, 3, 4, 5, 6, 7; columns variants 0, 1, 3, 4, 5,
 * 6, 7; time variants 0..5; general right-hand-side time variants 0..5; the x_2 and x_1
 * passes that the plane pass replaces (sum); plane-pass variants 0..2. */
int qbvm_plan_autotune(qbvm_plan_t p, double* ms_out);

/* The kernel variants a plan uses (HOST outputs, each may be NULL): sine rows, sine
 * columns, time, general right-hand-side time. */
int qbvm_plan_get_variants(qbvm_plan_t p, int* var_rows, int* var_cols, int* var_time, int* var_general);

/* Select kernel variants by hand (an addition, for tests and tuning outside the
 * autotuner): -1 keeps the current one.  A variant must exist for the plan's
 * transform lengths (sine variants 0..7 for a power-of-two sine length, time
 * variants 0..5 for a power-of-two or Rader length and 0..3 for Good-Thomas (2 and 3
 * with Rader's algorithm for the prime rows),
 * general variants 0..5 where the padded general pipeline runs), else QBVM_EINVAL and
 * nothing changes.  Shapes that use the generic kernels accept only -1. */
int qbvm_plan_set_variants(qbvm_plan_t p, int var_rows, int var_cols, int var_time, int var_general);

/* Plane pass (an addition to the output schedule of Step (c)): for d >= 2 with m = 127 the
 * x_2 and x_1 sine transforms of each level (and x_3 position) run in one kernel on the
 * whole plane, which moves 16 bytes per unknown less than a columns pass followed by a
 * rows pass.  On by default (variant 0) where the shape allows it; qbvm_plan_autotune
 * times its variants (0: 16 values per lane, 512 lanes; 1: 8 values per lane, 1024 lanes;
 * 2: as 0, loads issued earlier) against the separate passes and keeps the fastest.
 * variant < 0 selects the separate passes.  A variant >= 0 where the shape does not allow
 * the plane pass: QBVM_EUNSUPPORTED; an unknown variant: QBVM_EINVAL; nothing changes. */
int qbvm_plan_set_plane(qbvm_plan_t p, int variant);

/* *variant (HOST) receives the plane-pass variant qbvm_solve uses, or -1 (separate passes). */
int qbvm_plan_get_plane(qbvm_plan_t p, int* variant);

/* -------------------------------------------------------------- solving ---- */

/* Solve one PinT system (Sections 3.1-3.3).  g_delta: DEVICE, m^d doubles.
 * y: DEVICE, (n+1) * m^d doubles for QBVM_OUT_ALL, m^d for QBVM_OUT_Y0/YN.
 * alpha > 0; variant QBVM_PQ or QBVM_PM.  Asynchronous on the plan's stream. */
int qbvm_solve(qbvm_plan_t p, double alpha, int variant, const double* g_delta,
               double* y, int output);

/* Another spatial operator (1D plans; Section 3.3 notes that the operator enters only
 * Step (b)): every later qbvm_solve on this plan uses the tridiagonal matrix A in
 * place of -Lap_h, A[i][i-1] = lower[i-1], A[i][i] = diag[i], A[i][i+1] = upper[i]
 * (HOST arrays of m-1, m, m-1 doubles, copied; lower/upper may be NULL when m = 1),
 * e.g. -(kappa u')' with variable kappa.  Step (b) is then the partitioned tridiagonal
 * elimination (cyclic reduction between chunks) per shift d_j/tau, without pivoting:
 * d_j/tau I + A must not need pivoting (A diagonally dominant with positive diagonal,
 * as diffusion operators are).  diag == NULL restores
 * the Dirichlet stencil.  Synchronous (waits for the plan's stream).  While an
 * operator is set, qbvm_solve_general, qbvm_discrepancy, qbvm_choose_alpha and
 * qbvm_bisect_batched return QBVM_EUNSUPPORTED (they work in the sine basis).
 * QBVM_EINVAL for d > 1 or non-finite entries. */
int qbvm_plan_set_operator_1d(qbvm_plan_t p, const double* lower, const double* diag, const double* upper);

/* Another spatial operator in 2D (Section 3.3: the operator enters only Step (b)):
 * every later qbvm_solve on this (d = 2) plan uses A = -div(kappa grad u) in place of
 * -Lap_h, in conservative five-point form with kappa at the cell faces and zero
 * Dirichlet data:
 *   (A u)_{j,i} = [kx[j][i] (u_{j,i} - u_{j,i-1}) + kx[j][i+1] (u_{j,i} - u_{j,i+1})
 *                + ky[j][i] (u_{j,i} - u_{j-1,i}) + ky[j+1][i] (u_{j,i} - u_{j+1,i})] / h^2,
 * node (j, i) at x_1 = (i+1) h, x_2 = (j+1) h, u = 0 outside the grid.  kx: HOST, m rows
 * of m+1 faces between x_1 neighbours; ky: HOST, m+1 rows of m faces between x_2
 * neighbours; both row-major, positive and finite, copied.  kappa = 1 is -Lap_h.
 * Step (b) then solves the shifted systems (d_j/tau I + A) w_j = f0 for
 * j < ceil(N_t/2) (the rest are their complex conjugates) by batched conjugate
 * orthogonal conjugate gradients preconditioned with d_j/tau I + kbar (-Lap_h), kbar =
 * (min + max)/2 of kappa, which the sine transform diagonalises; a system stops when
 * its residual falls to tol |f0| (0 < tol < 1), all stop after max_iter iterations
 * (>= 1).  Such solves are synchronous on the plan's stream (the host checks
 * convergence once per iteration) and return QBVM_ENOCONV, with y written, if some
 * system did not converge; qbvm_plan_operator_stats reports the last one.  The
 * plan allocates 12 (ceil(N_t/2)) m^2 doubles of workspace here.  kx == NULL restores
 * the Dirichlet stencil.  While the operator is set, qbvm_solve_general,
 * qbvm_discrepancy, qbvm_choose_alpha and qbvm_bisect_batched return
 * QBVM_EUNSUPPORTED.  QBVM_EINVAL for d != 2, NULL ky, a non-positive or
 * non-finite coefficient, tol or max_iter out of range; QBVM_EUNSUPPORTED for m > 4480
 * (the operator kernel keeps a workgroup's 1024 points and a grid row either side in LDS). */
int qbvm_plan_set_operator_2d(qbvm_plan_t p, const double* kx, const double* ky, double tol, int max_iter);

/* The same in 3D (d = 3 plans): A = -div(kappa grad u) in conservative seven-point form,
 *   (A u)_{k,j,i} = sum over the six faces of the cell of kappa_face (u_{k,j,i} - u_neighbour) / h^2,
 * node (k, j, i) at x_1 = (i+1) h, x_2 = (j+1) h, x_3 = (k+1) h, u = 0 outside the grid.
 * kx: HOST [m][m][m+1] faces between x_1 neighbours; ky: HOST [m][m+1][m] between x_2
 * neighbours; kz: HOST [m+1][m][m] between x_3 neighbours; row-major, positive, finite,
 * copied.  Everything else (method, preconditioner, tolerance, workspace of
 * 12 ceil(N_t/2) m^3 doubles, errors, the entry points it disables) as for 2D;
 * QBVM_EINVAL for d != 3. */
int qbvm_plan_set_operator_3d(qbvm_plan_t p, const double* kx, const double* ky, const double* kz, double tol,
                              int max_iter);

/* Statistics of the last 2D/3D-operator solve (HOST outputs, each may be NULL): iterations
 * taken, the largest relative residual |r_j|/|f0| over the systems, and the number of
 * systems that stopped on a breakdown (a zero bilinear form) before converging. */
int qbvm_plan_operator_stats(qbvm_plan_t p, int* iterations, double* max_rel_residual, int* breakdowns);

/* Solve the all-at-once system of Sections 3.1/3.2 for a general right-hand side (an
 * addition beyond the paper's data: source terms, or one application of the PinT
 * system as a preconditioner).  f: DEVICE, (n+1) m^d doubles, one block per level,
 * for the rows (I/tau - Lap_h) y^0 - (omega/tau) y^N = f^0 and
 * (I/tau - Lap_h) y^t - y^{t-1}/tau = f^t (t >= 1); y: DEVICE, (n+1) m^d doubles, may
 * equal f.  Step (a) becomes a Gamma_omega-scaled DFT along time of every mode.
 * qbvm_solve is the case f = (f0, 0, ..., 0).  f is not modified unless y == f.
 * Asynchronous on the plan's stream; uses the plan's workspace and tables, so calls
 * on one plan are ordered by its stream.  QBVM_EUNSUPPORTED when one time signal and
 * its working copy exceed a workgroup's LDS, while a 1D operator is set, or on a 1D
 * plan whose sine length exceeds the FFT core (see the size limits). */
int qbvm_solve_general(qbvm_plan_t p, double alpha, int variant, const double* f, double* y);

/* Solve `count` independent instances of possibly different grids in one
 * batched launch sequence (an addition; not in the paper).  All arrays of
 * length `count` are HOST arrays; g_deltas[i] and ys[i] are DEVICE pointers
 * with the sizes qbvm_solve documents for grids[i] and outputs[i] (every output mode is
 * supported).  The launch sequence is one HIP graph per set of (grid, variant, output):
 * the 1D instances with every level run as two persistent launches over device tables
 * of their argument blocks (uploaded with every call), every other instance as its own
 * chain of kernels; alpha is read from a device table uploaded with every call.  A later
 * call with the same set reuses the graph, for new buffers too (their addresses are
 * written into the recorded launches).  At most 8 sets are kept (least recently used
 * dropped); plans are cached per grid.  Asynchronous on hip_stream (the uploads are
 * ordered on it).  A single-level output of a 1D grid whose sine transform exceeds the
 * FFT core: QBVM_EUNSUPPORTED. */
int qbvm_solve_batched(int count, const qbvm_grid* grids, const double* alphas,
                       const int* variants, const double* const* g_deltas,
                       double* const* ys, const int* outputs, void* hip_stream);

/* Free every cached batched plan and graph. */
void qbvm_batched_cache_clear(void);

/* ---------------------------------------------- regularisation parameter ---- */

/* D(alpha) = ||y^N(alpha) - g_delta||_h, ||v||_h = h^{d/2} ||v||_2 (the discrete
 * L2 norm of Section 5), with y^N computed by Step (c) at the last level only.
 * g_delta: DEVICE.  *D_out: HOST.  Returns once the result is on the host (the
 * last kernel posts it to host memory the plan owns; g_delta has been read by
 * then); later work on the plan's stream stays ordered after it. */
int qbvm_discrepancy(qbvm_plan_t p, double alpha, int variant, const double* g_delta,
                     double* D_out);

/* Choose alpha by the discrepancy principle D(alpha) = tau_dp * delta (an
 * addition; the paper uses alpha = delta or tau*delta a priori, Section 5).
 * With opts->use_learned the plan's network predicts log10 alpha from the sine
 * spectrum of g_delta and delta; the prediction is accepted if
 * win_lo <= D/delta <= win_hi, otherwise the device-side bisection on log10 alpha
 * runs and its result is returned.  g_delta: DEVICE; delta > 0 (weighted norm).
 * alpha_out, info: HOST (info may be NULL).  Returns once the result is on the
 * host, as qbvm_discrepancy.  Returns QBVM_ENOROOT
 * (with *alpha_out = the nearer bracket end and info->bracket_hit = 1) when the
 * root is outside the bracket. */
int qbvm_choose_alpha(qbvm_plan_t p, int variant, const double* g_delta, double delta,
                      const qbvm_alpha_opts* opts, double* alpha_out, qbvm_alpha_info* info);

/* qbvm_choose_alpha for `count` instances one after another (batch size 1 each), with
 * the latency of every call measured on the host (steady clock around the call, which
 * returns once its result is on the host) and no interpreter between calls: the
 * per-instance latency of the alpha choice, learned or bisection.  g_deltas: DEVICE,
 * count * m^d doubles; deltas: HOST, count doubles; alphas_out: HOST, count;
 * infos_out, seconds_out: HOST, count each, may be NULL.  An instance whose root lies
 * outside the bracket is recorded (info.bracket_hit = 1) and the loop goes on; any
 * other error stops it and is returned. */
int qbvm_choose_alpha_each(qbvm_plan_t p, int variant, int count, const double* g_deltas,
                           const double* deltas, const qbvm_alpha_opts* opts, double* alphas_out,
                           qbvm_alpha_info* infos_out, double* seconds_out);

/* Batched bisection for `count` instances on the plan's grid (label generation).
 * g_deltas: DEVICE, count * m^d doubles; deltas: DEVICE, count doubles;
 * alphas_out: DEVICE, count doubles; hits_out: DEVICE, count ints (may be NULL).
 * Asynchronous on the plan's stream. */
int qbvm_bisect_batched(qbvm_plan_t p, int variant, int count, const double* g_deltas,
                        const double* deltas, const qbvm_alpha_opts* opts,
                        double* alphas_out, int* hits_out);

/* Learned-alpha input features for `count` instances on the plan's grid:
 * 32 bins of log10(h^d * sum of squared orthonormal-DST coefficients) over
 * rho = |k|_2 in [sqrt(d), m sqrt(d)], then log10(delta).  g_deltas: DEVICE,
 * count * m^d; deltas: DEVICE, count; feats: DEVICE, count * 33 floats (FP32 of
 * the FP64 values).  Asynchronous on the plan's stream. */
int qbvm_features(qbvm_plan_t p, int count, const double* g_deltas, const double* deltas,
                  float* feats);

/* Attach a learned-alpha model to the plan (copied to the device).  model: HOST,
 * QBVM_MODEL_FLOATS floats = network parameters (QBVM_MLP_PARAMS, layout of
 * qbvm_mlp_forward) | feature mean[33] | feature std[33] | label mean | label std.
 * The network maps standardised features to the standardised label log10 alpha. */
int qbvm_set_alpha_model(qbvm_plan_t p, const float* model);

/* ------------------------------------------------------- network (FP32) ---- */
/* 33 -> 64 -> 64 -> 1 perceptron, GELU (erf form) after both hidden layers.
 * Parameter layout (QBVM_MLP_PARAMS floats): W1[64][33] | b1[64] | W2[64][64] |
 * b2[64] | W3[64] | b3.  All pointers DEVICE; asynchronous on hip_stream. */

/* out[b] = net(X[b, :]) for b < B.  X: B x 33 row-major. */
int qbvm_mlp_forward(const float* params, int B, const float* X, float* out, void* hip_stream);

/* Mean-squared-error loss over the batch and its gradient (backpropagation).
 * grad: QBVM_MLP_PARAMS floats (overwritten); loss: 1 float (overwritten). */
int qbvm_mlp_loss_grad(const float* params, int B, const float* X, const float* y,
                       float* grad, float* loss, void* hip_stream);

/* Largest batch of qbvm_mlp_loss_grad_noalloc. */
#define QBVM_NOALLOC_MAX_BATCH 16384

/* qbvm_mlp_loss_grad without any allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc).  Same kernels, arguments and results as qbvm_mlp_loss_grad; the
 * per-sample activations go to a fixed array of QBVM_NOALLOC_MAX_BATCH * 193 floats
 * (12.1 MiB) that every GPU the library runs on holds until the process ends.  The
 * first call on a device looks up that device's copy.  B > QBVM_NOALLOC_MAX_BATCH
 * returns QBVM_EINVAL and enqueues nothing.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (other streams, other threads) race and must be
 * ordered by the caller, e.g. by issuing them on one stream.  Nothing in the array needs
 * to start at zero (each call writes every entry it reads). */
int qbvm_mlp_loss_grad_noalloc(const float* params, int B, const float* X, const float* y,
                               float* grad, float* loss, void* hip_stream);

/* One Adam step (bias-corrected, step >= 1) on n parameters. */
int qbvm_adam_step(float* params, const float* grad, float* m, float* v, int n, int step,
                   float lr, float beta1, float beta2, float eps, void* hip_stream);

/* ------------------------------------------------------ kernel timing ---- */
/* For benchmarks: while enabled, every kernel that a plan launches directly on
 * its stream is bracketed by two HIP events recorded on that stream (kernels
 * inside captured graphs are not).  Aggregates are kept per kernel kind. */
void qbvm_profile_enable(int on);
void qbvm_profile_reset(void);
/* Waits for the recorded events, folds them into the aggregates and returns the
 * number of kernel kinds seen so far. */
int qbvm_profile_count(void);
/* Kernel kind i (0 <= i < qbvm_profile_count()): its name (copied into name_buf,
 * HOST, buf_len bytes), number of launches, summed duration in milliseconds and
 * the summed algorithmic bytes (compulsory reads and writes of the kernel's
 * design) and FLOPs (5 n log2 n per complex FFT of length n plus the pointwise
 * work).  All outputs are HOST pointers. */
int qbvm_profile_get(int i, char* name_buf, int buf_len, long long* launches, double* total_ms,
                     double* bytes, double* flops);

/* ------------------------------------------------------------- errors ---- */
const char* qbvm_strerror(int code);
const char* qbvm_last_error(void);
int qbvm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QBVM_H */

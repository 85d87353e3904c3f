/*
 * mlba.h -- C ABI of the MI355X (gfx950) library for preconditioned
 * modified linearized Bregman (MLBA) frame-based deblurring.
 *
 * Method: Cai, Donatelli, Bianchi, Huang, "Regularization preconditioners for
 * frame-based image deblurring with reduced boundary artifacts"
 * (arXiv:1504.07234).  One iteration is eq. (MLBA2) of section 3:
 *
 *     x^k     = delta_k S_mu(z^k)                      (eq. soft)
 *     r^k     = g - A W^T x^k                           (eqs. modeld, wavecoeff)
 *     z^{k+1} = z^k + W A^T P_{alpha_k} r^k             (eq. MLBA2)
 *
 * with A the blur of section 2, W the linear B-spline framelet of section
 * 6.1 and P the spectral Tikhonov preconditioner of Algorithm 1 (BCCB/FFT,
 * eq. Alg1) or Algorithm 3 (symmetrised PSF, DCT, eq. Alg3).
 *
 * Conventions shared by every entry point
 *   - Images are row-major float32 arrays, element (y, x) at y*side + x.
 *     Observed images are n x n.  The unknown image is N x N with
 *     N = n + p - 1 for MLBA_BC_RECT (section 2.1) and N = n otherwise.
 *   - Frame coefficients are band-planar float32 [bands][N][N] with
 *     bands = 8*levels + 1: band 0 is the final low-pass image, then for each
 *     level l = 1..levels the eight pairs (i,j) = (0,1),(0,2),(1,0),(1,1),
 *     (1,2),(2,0),(2,1),(2,2), where (i,j) applies mask b_i along x and b_j
 *     along y (section 6.1; level l uses dilation 2^(l-1)).
 *   - The PSF is p x p float32 (p odd), centre (c, c), c = (p-1)/2.
 *   - Every pointer named as "device" must point to device memory of the
 *     current HIP device; "host" pointers are read before the call returns.
 *     The caller owns every buffer it passes; the library never frees them.
 *   - Work is enqueued on `stream` and is asynchronous unless stated.  A plan
 *     owns its workspace (allocated by mlba_plan_create), so one plan must
 *     not be used by two streams at the same time.  Entry points other than
 *     mlba_plan_create / mlba_plan_destroy / mlba_batch_create /
 *     mlba_batch_destroy / mlba_unrolled_create / mlba_unrolled_destroy
 *     allocate no device memory (graph instantiation aside, see
 *     mlba_batch_restore).  Each object records a completion event on the
 *     stream of every call that enqueues work on its buffers; its destroy
 *     call waits for that event (not for the whole device), then frees.
 *   - Errors: every call returns an int status.  Negative values are
 *     errors (nothing was enqueued), MLBA_WARN_DIVERGED is a warning.
 *     No C++ exception crosses this interface.
 */
#ifndef MLBA_H
#define MLBA_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define MLBA_OK              0
#define MLBA_WARN_DIVERGED   1   /* residual became non-finite or grew 1e3-fold */
#define MLBA_EINVAL         -1   /* bad argument (null, size, odd/even rules)    */
#define MLBA_EUNSUPPORTED   -2   /* size outside the supported transforms        */
#define MLBA_EHIP           -3   /* a HIP runtime call failed (mlba_last_hip_error) */
#define MLBA_ENOMEM         -4   /* device allocation failed                     */

/* ---- boundary models (section 2) ------------------------------------ */
#define MLBA_BC_RECT      0  /* rectangular n^2 x m^2 A = M A_big, eq. (Arect) */
#define MLBA_BC_REFLECT   1  /* reflective (half-sample symmetric) pad, Table 1 */
#define MLBA_BC_PERIODIC  2  /* periodic pad, Table 1                          */
#define MLBA_BC_ZERO      3  /* zero pad, Table 1                              */
#define MLBA_BC_ANTIREFLECT 4  /* antireflective pad, section 2.2: position -i holds
                                  2 f[0] - f[i] along each axis, corners antireflected
                                  along one axis then the other; A^T is replaced by the
                                  reblurring A' (the same pad, PSF rotated 180 degrees)
                                  everywhere the method uses it                    */

/* ---- preconditioners (section 4) ------------------------------------ */
#define MLBA_PRECOND_BCCB 0  /* P = (C C^T + alpha I)^-1 by 2-D FFT, Algorithm 1 */
#define MLBA_PRECOND_DCT  1  /* P = (Q Q^T + alpha I)^-1 by 2-D DCT of the
                                symmetrised PSF, Algorithm 3                  */
#define MLBA_PRECOND_NONE 2  /* P = I: plain linearized Bregman, eq. (iterLinBreg) */
#define MLBA_PRECOND_AR   3  /* P = (Q Q' + alpha I)^-1, Q the antireflective blur of the
                                symmetrised PSF, by the 2-D antireflective transform
                                (sections 2.2, 4.3: Algorithm 3 for MLBA_BC_ANTIREFLECT) */

/* ---- alpha schedules ------------------------------------------------- */
#define MLBA_ALPHA_CONST      0  /* alpha_k = alpha0                              */
#define MLBA_ALPHA_GEOMETRIC  1  /* alpha_k = max(alpha0 * ratio^k, alpha_floor)  */
#define MLBA_ALPHA_TABLE      2  /* alpha_k = table[k] (host, >= k0+iters values) */
#define MLBA_ALPHA_NS         3  /* Algorithm 4-NS (MLBA_METHOD_ALG4, BCCB or DCT plan): alpha_n solves
                                    alpha_n ||(C C^T + alpha_n I)^{-1} r^n|| = q_n ||r^n||,
                                    q_n = max{ns_q, 2 ns_rho + (1 + ns_rho) / tau_n},
                                    tau_n = ||r^n|| / noise (eq. Alg4_rev_7); the run stops at
                                    the first n with ||r^n|| <= tau noise, tau = (1 + 2 ns_rho) /
                                    (1 - 2 ns_rho) (eq. Alg4_rev_12); noise = stop->noise_norm
                                    (required); alpha0 is the first Newton start.  alpha_n
                                    is found on the device (at most 12 Newton steps in log
                                    alpha inside a shrinking bracket, stopping once a step
                                    moves log alpha by < 2^-22: the FP32 sums resolve no
                                    finer); alpha_out reports it */

typedef struct mlba_alpha_schedule {
    int kind;
    double alpha0;
    double ratio;
    double alpha_floor;
    const double* table;  /* host; used when kind == MLBA_ALPHA_TABLE */
    int table_len;
    double ns_q;          /* MLBA_ALPHA_NS: q in (2 rho, 1) (the paper's runs: 0.5)  */
    double ns_rho;        /* MLBA_ALPHA_NS: rho in (0, 1/2) (the paper's runs: 1e-4) */
} mlba_alpha_schedule;

/* Update direction (section 5).  MLBA: eq. (MLBA2), z += W A^T P_alpha r with
 * the preconditioner of the plan (periodic model, BCCB plan, MLBA_BLUR_FFT:
 * computed as ALG4's direction, since A = C there).  ALG4: eq. (Alg4), z += W C^T (C C^T +
 * alpha I)^{-1} r, C the periodic (BCCB plan) or reflective-of-the-symmetrised-
 * PSF (DCT plan) blur: no A^T product; square boundary models only (plans
 * with MLBA_BC_RECT return MLBA_EUNSUPPORTED), preconditioner BCCB or DCT. */
#define MLBA_METHOD_MLBA 0
#define MLBA_METHOD_ALG4 1
/* ALG2: eq. (Alg2), z += W A^T t with t ~ (A A^T + alpha I)^{-1} r from
 * beta_n = min{pcg_max, beta_tol} steps of CG preconditioned by the plan's
 * (C C^T + alpha I)^{-1} (BCCB or DCT), started from zero; beta_tol is the first
 * step whose preconditioned relative residual sqrt(res^T M^-1 res / r^T M^-1 r)
 * is at most pcg_tol (eq. bet; the paper: 5 and 1e-3).  The stopping test
 * runs on the device: every iteration enqueues pcg_max CG steps and the steps
 * after the stop leave t unchanged (no host round trip; iters <= 65536).  With
 * MLBA_BC_RECT and MLBA_BLUR_FFT each (A A^T + alpha I) d is one transform
 * pair of the grid with |H|^2. */
#define MLBA_METHOD_ALG2 2

/* Discrepancy-principle stop, eq. (discrpr): stop at the first k with
 * ||r^k|| <= gamma * noise_norm.  Checked every `check_every` iterations
 * (one device->host copy of a scalar per check). */
typedef struct mlba_stop {
    double noise_norm;
    double gamma;
    int check_every;
} mlba_stop;

/* Parameters of a restoration run. */
typedef struct mlba_params {
    mlba_alpha_schedule alpha;
    const double* mu;          /* host, n_mu values: 1 (all bands) or `bands`  */
    int n_mu;
    double delta;              /* > 0: step delta_k = delta;
                                  <= 0: delta_k = 0.9 / max(||A^T P_{alpha_k} A||, 0.9)
                                  (section 3, convergence theorem for MLBA), the norm
                                  computed once per distinct alpha_k by Lanczos
                                  (up to 1000 steps, converged to 1e-9 relative;
                                  antireflective model: 50 power steps, see
                                  mlba_plan_opnorm); the algorithm 4 methods use 1 */
    const double* delta_table; /* host, optional: delta_k = delta_table[k] for
                                  k = 0 .. k0+iters (k0+iters+1 values); the
                                  last value scales the returned image; its
                                  length is delta_table_len                   */
    int iters;                 /* iterations to run                           */
    int k0;                    /* global index of the first iteration (resume) */
    const mlba_stop* stop;     /* optional discrepancy stop (NULL: fixed iters) */
    int state;                 /* MLBA_STATE_EXPLICIT or MLBA_STATE_IMPLICIT    */
    int method;                /* MLBA_METHOD_MLBA or MLBA_METHOD_ALG4          */
    double* alpha_out;         /* host, optional: the alpha_k of each iteration run
                                  (iters values; synchronous copy at the end)   */
    int pcg_max;               /* MLBA_METHOD_ALG2: step cap (0: 5)            */
    double pcg_tol;            /* MLBA_METHOD_ALG2: tolerance (0: 1e-3)         */
    int* pcg_steps_out;        /* host, optional: beta_n of each iteration run  */
    double* delta_out;         /* host, optional: the delta_k used, one per
                                  iteration run plus the one scaling the
                                  returned image (iters_done + 1 values, at most
                                  iters + 1)                                   */
    int delta_table_len;       /* values in delta_table; MLBA_EINVAL when
                                  delta_table is given with fewer than
                                  k0 + iters + 1                               */
} mlba_params;

/* State kept between iterations.  Explicit: the frame coefficients z
 * ([bands][N][N]), updated by z += W A^T t.  Implicit: since z^0 = 0 and every
 * update of eq. (MLBA2) is W applied to A^T t, z^k = W omega^k with
 * omega^{k+1} = omega^k + A^T t_k; only omega (N x N) is kept and the
 * synthesis recomputes W omega level by level.  Both compute the same
 * iteration (they differ by floating-point rounding only); the implicit state
 * moves about 6x fewer bytes per iteration.  An explicit state can be made from
 * an implicit one with mlba_framelet_analysis (z = W omega). */
#define MLBA_STATE_EXPLICIT 0
#define MLBA_STATE_IMPLICIT 1

typedef struct mlba_plan_s* mlba_plan_t;

/* ---- library --------------------------------------------------------- */
const char* mlba_status_string(int status);
int mlba_last_hip_error(void);   /* hipError_t of the last MLBA_EHIP on this thread */
int mlba_version(void);

/* ---- plans ------------------------------------------------------------
 * mlba_plan_create: n observed side, p odd PSF side (1 <= p <= n, p <= 49), bc one of
 * MLBA_BC_*, precond one of MLBA_PRECOND_*, levels in [1, 4] with
 * 2^(levels-1) < N.  The transforms of P have length L = n (BCCB and DCT:
 * n even, n >= 8) or L = 2(n - 1) (MLBA_PRECOND_AR, which also needs
 * MLBA_BC_ANTIREFLECT; n >= 4).  L = 2^a 3^b 5^c runs as mixed-radix
 * Stockham passes up to L = 2048; any other L runs in Bluestein's chirp
 * form over the smallest 2^a 3^b 5^c length m >= 2L - 1, which must be at
 * most 2048 (L <= 1024; e.g. the 196 x 196 field of view of section 6's
 * third example: n = 196 for BCCB and DCT, L = 390 for the antireflective
 * transform).  MLBA_EUNSUPPORTED otherwise.  psf: device p x p.
 * Allocates the workspace, copies the PSF and computes the spectrum of
 * (C C^T) or (Q Q^T) on `stream` (section 4.1 / 4.3).  The plan keeps no
 * reference to `psf`.  With MLBA_BC_ANTIREFLECT every A^T below (operators,
 * iterations, the norm of mlba_plan_opnorm) is the reblurring A'. */
int mlba_plan_create(mlba_plan_t* plan, int n, int p, int bc, int precond, int levels,
                     const float* psf, hipStream_t stream);
/* Replace the PSF (same p) and recompute the spectrum. psf: device p x p. */
int mlba_plan_set_psf(mlba_plan_t plan, const float* psf, hipStream_t stream);
int mlba_plan_destroy(mlba_plan_t plan);
/* How the blur A and its transpose (or, antireflective model, its reblur
 * A') are computed:
 * MLBA_BLUR_DIRECT (default): LDS-tiled direct convolution, p^2 taps per
 * output; MLBA_BLUR_FFT: circular convolution on an M x M grid, M >= m =
 * n + p - 1, M = 2^a 3^b (section 2.1's FFT evaluation), three passes per
 * product: row transforms, a column pass, inverse row transforms.  For
 * p = 5, 9, 17 and 31 the column pass is the p-tap convolution along y with
 * the PSF's rows transformed the same way (the same values as the column
 * transform pair with F(pad H) on every output that does not wrap around;
 * the taps, (M/2 + 1) p complex, are kept with the spectrum); otherwise it is
 * that transform pair.  The square models place the n x n image with its pad
 * (Table 1, section 2.2) on the grid, m x m; A^T folds the correlation back
 * by the pad's transpose.  With the periodic model and MLBA_PRECOND_BCCB,
 * MLBA_BLUR_FFT also selects for eq. (MLBA2) the spectral residual of
 * Algorithm 4 (A = C there): one 2-D transform pair per iteration.
 * mlba_plan_set_blur: MLBA_BLUR_FFT allocates the grid's workspace and PSF
 * spectrum on first use (synchronous) and returns MLBA_EUNSUPPORTED when M
 * would exceed 3072.  mlba_plan_autotune:
 * times both on the plan's own scratch buffers (`reps` calls each, HIP events,
 * synchronous), keeps the faster pair, writes the mean ms per call to ms_out
 * (host, optional: direct A, direct A^T, FFT A, FFT A^T; -1 where unavailable)
 * and returns the chosen mode (>= 0) or an error. */
#define MLBA_BLUR_DIRECT 0
#define MLBA_BLUR_FFT    1
int mlba_plan_set_blur(mlba_plan_t plan, int mode, hipStream_t stream);
int mlba_plan_autotune(mlba_plan_t plan, int reps, double* ms_out, hipStream_t stream);
/* Sizes: observed side n, PSF side p, unknown side N, number of bands. */
int mlba_plan_dims(mlba_plan_t plan, int* n, int* p, int* N, int* bands);
/* ||A^T P_alpha A||, the largest eigenvalue of the symmetric positive
 * semidefinite A^T P_alpha A (section 3, convergence theorem), by Lanczos from a
 * fixed pseudo-random start: at most `iters` steps (and at most 32768), stopping
 * once the largest Ritz value has changed by at most 1e-9 (relative) over 8
 * steps; the tridiagonal coefficients are read back every 8 steps.  With
 * MLBA_BC_ANTIREFLECT the operator A' P_alpha A is not symmetric and the
 * result is ||M v|| / ||v|| after `iters` power steps (an estimate of its
 * largest eigenvalue modulus).  Synchronous; result on host; uses the plan's
 * scratch buffers. */
int mlba_plan_opnorm(mlba_plan_t plan, double alpha, int iters, double* out, hipStream_t stream);

/* ---- operators (asynchronous) ---------------------------------------------- */
/* y = A u.   u: device N x N, y: device n x n (section 2, eq. Arect / Table 1). */
int mlba_apply_A(mlba_plan_t plan, const float* u, float* y, hipStream_t stream);
/* r = g - A u.  g, r: device n x n, u: device N x N. */
int mlba_residual(mlba_plan_t plan, const float* g, const float* u, float* r, hipStream_t stream);
/* w = A^T y.  y: device n x n, w: device N x N (section 2.1: A^T = A_big^T M^T;
 * for imposed boundaries the exact transpose of the padding). */
int mlba_apply_At(mlba_plan_t plan, const float* y, float* w, hipStream_t stream);
/* t = P_alpha r.  r, t: device n x n, may alias (section 4, Algorithms 1 / 3). */
int mlba_apply_P(mlba_plan_t plan, const float* r, float* t, double alpha, hipStream_t stream);
/* t = C^T (C C^T + alpha I)^{-1} r: the direction of eq. (Alg4) before W, with
 * C the periodic-boundary blur of the PSF (BCCB plan) or the reflective blur of
 * the symmetrised PSF (DCT plan).  r, t: device n x n, must not alias.  Square
 * models only (MLBA_EUNSUPPORTED for MLBA_BC_RECT or MLBA_PRECOND_NONE). */
int mlba_apply_CtP(mlba_plan_t plan, const float* r, float* t, double alpha, hipStream_t stream);
/* z = W f.  f: device N x N, z: device [bands][N][N] (section 6.1). */
int mlba_framelet_analysis(mlba_plan_t plan, const float* f, float* z, hipStream_t stream);
/* z += W w: the Bregman update of eq. (MLBA2).  w: device N x N. */
int mlba_analysis_update(mlba_plan_t plan, const float* w, float* z, hipStream_t stream);
/* f = W^T z.  z: device [bands][N][N], f: device N x N. */
int mlba_framelet_synthesis(mlba_plan_t plan, const float* z, float* f, hipStream_t stream);
/* f = W^T (delta S_mu(z)): threshold fused into synthesis (eqs. soft, MLBA2).
 * mu: host, n_mu = 1 or bands values. */
int mlba_threshold_synthesis(mlba_plan_t plan, const float* z, const double* mu, int n_mu,
                             double delta, float* f, hipStream_t stream);
/* x = delta S_mu(z) over `bands` planes of `band_elems` elements (eq. soft).
 * z, x: device, may alias.  mu: host, n_mu = 1 or `bands` values (<= 64). */
int mlba_soft_threshold(const float* z, float* x, int bands, size_t band_elems,
                        const double* mu, int n_mu, double delta, hipStream_t stream);

/* f = W^T(delta S_mu(W omega)): the synthesis step of the implicit state, one
 * launch per level plus levels - 1 low-pass launches.  omega, f: device N x N
 * (must not alias).  mu: host, n_mu = 1 or bands values. */
int mlba_shrink_synthesis(mlba_plan_t plan, const float* omega, const double* mu, int n_mu, double delta,
                          float* f, hipStream_t stream);

/* ---- preconditioner without a plan and without allocation ---------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): t = P_alpha r
 * exactly as mlba_apply_P computes it for a plan with this PSF, n and
 * preconditioner (MLBA_PRECOND_BCCB, section 4.1, or MLBA_PRECOND_DCT,
 * section 4.3), with no plan.  psf: device p x p (p odd, p <= n); r, t: device
 * n x n (may alias); alpha > 0.  n even, 8 <= n <= MLBA_STATIC_MAX_N,
 * n = 2^a 3^b 5^c; MLBA_EUNSUPPORTED for larger or other n and for the other
 * preconditioners, MLBA_EINVAL for bad arguments.  Each call rebuilds the
 * transform tables and the spectrum of the PSF, then runs the three transform
 * passes (asynchronous, on `stream`).  Working memory: one static device array
 * of about 50.5 MB per device, kept from the first call on that device until
 * the process ends (its address is looked up once per device); the call
 * allocates nothing.  Every call on a device shares that array, so calls that
 * overlap on one device (two streams, two host threads) race; calls in order
 * on one stream do not. */
#define MLBA_STATIC_MAX_N 2048
int mlba_apply_P_static(const float* psf, int n, int p, int precond, const float* r, float* t, double alpha,
                        hipStream_t stream);

/* ---- restoration --------------------------------------------------------
 * Runs params->iters iterations of eq. (MLBA2) from the state z_state
 * (device, in/out: [bands][N][N] for the explicit state, N x N omega for the
 * implicit one; pass NULL to start from zero in the plan's own state buffer)
 * and writes f_out = W^T(delta_K S_mu(z^K)) (device N x N).
 * g: device n x n.  rnorm_out: optional host array receiving ||r^k|| for each
 * iteration run (synchronous copy at the end).  iters_done: optional host
 * int receiving the number of iterations run (smaller than iters only when
 * the discrepancy stop fired).  Returns MLBA_WARN_DIVERGED when a residual
 * norm was non-finite or exceeded 1e3 times the first one (rnorm is then
 * always computed); otherwise the call is asynchronous unless rnorm_out,
 * iters_done, params->stop or an automatic delta is requested. */
int mlba_restore(mlba_plan_t plan, const float* g, const mlba_params* params,
                 float* f_out, float* z_state, double* rnorm_out, int* iters_done,
                 hipStream_t stream);

/* ---- batched restoration ------------------------------------------------
 * A batch advances many images of uneven sizes, each with its own plan (PSF,
 * boundary model, sizes), alpha, mu and step, through eq. (MLBA2) together:
 * every phase of an iteration is one launch covering the tiles of all images,
 * and each image follows exactly the arithmetic of its own plan.
 *
 * mlba_batch_create: count plans (host array of distinct plans sharing
 * `levels` and the preconditioner kind); the batch uses each plan's workspace
 * and state buffer, so those plans must not run other work while the batch
 * runs.  max_iters bounds the iteration count of one call.  Allocates the
 * batch's descriptor table, norm buffers and tile maps, the maps sized for
 * the tile choice with the most workgroups, so that mlba_batch_autotune and
 * mlba_batch_set_tiles allocate nothing (synchronous).
 *
 * mlba_batch_restore: g, f_out: host arrays of `count` device pointers
 * (image i: n_i x n_i input, N_i x N_i output).  alpha, delta: host arrays of
 * `count` values (delta <= 0: automatic step per image, see mlba_params).
 * mu: host array of count * n_mu values (n_mu = 1 or bands).  state:
 * MLBA_STATE_EXPLICIT (the frame coefficients z) or MLBA_STATE_IMPLICIT (omega
 * with z = W omega: per iteration the low-pass chain, one shrink-synthesis
 * launch per level, the blur, the preconditioner and omega += A^T t in the
 * A^T launch; no analysis).  z_state: NULL to start every image from zero in
 * its plan's state buffer, or a host array of `count` device pointers
 * ([bands][N_i][N_i] explicit, [N_i][N_i] implicit; in/out).  rnorm_out:
 * optional host array of count * iters residual norms (synchronous; returns
 * MLBA_WARN_DIVERGED as mlba_restore does).  use_graph != 0: the whole
 * sequence for this iteration count is captured once into a hipGraph on a
 * private stream (first call; instantiation allocates) and replayed on
 * `stream`; later calls with the same iteration count, state mode and
 * z_state presence only update the descriptor table and replay. */
typedef struct mlba_batch_s* mlba_batch_t;
int mlba_batch_create(mlba_batch_t* batch, int count, const mlba_plan_t* plans, int max_iters,
                      hipStream_t stream);
int mlba_batch_destroy(mlba_batch_t batch);
int mlba_batch_restore(mlba_batch_t batch, const float* const* g, const double* alpha, const double* mu,
                       int n_mu, const double* delta, int iters, float* const* f_out, float* const* z_state,
                       double* rnorm_out, int state, int use_graph, hipStream_t stream);

/* Autotuner of the batch's tile shapes.  Times every candidate of each
 * tunable phase on the batch's own images, `reps` launches each after one
 * untimed launch (HIP events on `stream`, synchronous), and keeps the fastest:
 *   - the blur A and the adjoint blur A^T: one or two output rows per thread
 *     (32- or 64-row tiles; PSFs with p > 33 always use 64-row tiles);
 *   - the preconditioner's row passes: at most 1, 2 or 4 row pairs per
 *     workgroup, or the built-in choice per size (cap 0);
 *   - its column pass: at most 1, 2, 4, 8 or 16 columns per workgroup, or
 *     the built-in choice (cap 0).
 * The timed launches only write the plans' scratch buffers (residual,
 * spectral workspace, A^T output), never a state.  A captured graph is
 * dropped and re-captured by the next graph restore.  Results do not depend on
 * the tile shapes: every choice computes each output with the same
 * arithmetic.  out (host, optional) receives the choices and the timings. */
#define MLBA_TUNE_ROWS 4
#define MLBA_TUNE_COLS 6
typedef struct mlba_batch_tuning {
    int conv_rows[2];                 /* chosen rows per thread: A, A^T          */
    int fft_rows_cap, fft_cols_cap;   /* chosen caps (0: built-in choice)        */
    double conv_ms[2][2];             /* [A / A^T][1 / 2 rows] mean ms per launch */
    double rows_ms[MLBA_TUNE_ROWS];   /* caps 0, 1, 2, 4: both row passes        */
    double cols_ms[MLBA_TUNE_COLS];   /* caps 0, 1, 2, 4, 8, 16                  */
} mlba_batch_tuning;
int mlba_batch_autotune(mlba_batch_t batch, int reps, mlba_batch_tuning* out, hipStream_t stream);
/* Sets the tile shapes directly from choice->conv_rows (each 1 or 2),
 * choice->fft_rows_cap and choice->fft_cols_cap (>= 0; a cap is rounded down
 * to a valid power of two per image size); the timings are ignored.  Lets a
 * caller reuse tuned choices for another batch of the same shapes
 * (synchronous). */
int mlba_batch_set_tiles(mlba_batch_t batch, const mlba_batch_tuning* choice, hipStream_t stream);

/* ---- differentiable unrolled MLBA -----------------------------------------
 * K iterations of eq. (MLBA2) from z = 0, f = W^T(delta S_mu(z^K)), for a
 * batch of images with the rectangular blur (section 2.1) and the BCCB
 * preconditioner (Algorithm 1), and the exact reverse-mode gradient of a loss
 * l(f) with respect to the per-band thresholds mu (eq. soft), alpha
 * (Algorithm 1), the PSF entries and the observations g.  The soft threshold
 * is differentiated almost everywhere: dS/dz = 1{|z| > mu} and
 * dS/dmu = -sgn(z) 1{|z| > mu}, taken as 0 at the kink |z| = mu.  delta is a
 * constant.  All images share alpha, mu, delta and the PSF side p; the
 * gradients returned are sums over the images, i.e. the gradient with respect
 * to parameters shared by the batch.
 *
 * mlba_unrolled_create: count distinct plans (MLBA_BC_RECT, MLBA_PRECOND_BCCB,
 * otherwise MLBA_EUNSUPPORTED; equal levels and p, otherwise MLBA_EINVAL),
 * iters = K >= 1, 1 <= ckpt_every <= K.  The object uses each plan's
 * workspace and PSF/spectrum (so those plans must not run other work
 * meanwhile) and allocates its own segment storage: per image
 * (ckpt_every + 2) states of bands*N*N floats plus ckpt_every images of each
 * of u, t and the half spectrum (synchronous).
 * mlba_unrolled_dims: number of checkpoint segments J = ceil(K / ckpt_every)
 * and, per image (host array of count values, optional), the checkpoint
 * buffer length J * bands * N_i * N_i in floats.
 *
 * mlba_unrolled_forward: g, f: host arrays of count device pointers (n_i x n_i
 * in, N_i x N_i out).  ckpt: host array of count device pointers to caller
 * buffers of the length above; slot j receives z^{j*ckpt_every}.  alpha > 0,
 * delta > 0; mu: host, n_mu = 1 or bands values >= 0.  Asynchronous.
 *
 * mlba_unrolled_backward: the same g, alpha, mu, delta and the checkpoints
 * written by the forward call (read only); df: host array of count device
 * pointers to dl/df (N_i x N_i).  Writes dmu (device, bands doubles), dalpha
 * (device, one double), dpsf (device, p*p doubles, row-major like the PSF)
 * and, when dg is not NULL, dg[i] = dl/dg_i (device n_i x n_i floats).  Each
 * checkpoint segment is recomputed once.  Results are deterministic (fixed
 * reduction order).  Asynchronous.  One object must not run two calls at
 * the same time. */
typedef struct mlba_unrolled_s* mlba_unrolled_t;
int mlba_unrolled_create(mlba_unrolled_t* unrolled, int count, const mlba_plan_t* plans, int iters,
                         int ckpt_every, hipStream_t stream);
int mlba_unrolled_destroy(mlba_unrolled_t unrolled);
int mlba_unrolled_dims(mlba_unrolled_t unrolled, int* segments, size_t* ckpt_elems_per_image);
int mlba_unrolled_forward(mlba_unrolled_t unrolled, const float* const* g, double alpha, const double* mu,
                          int n_mu, double delta, float* const* ckpt, float* const* f, hipStream_t stream);
int mlba_unrolled_backward(mlba_unrolled_t unrolled, const float* const* g, double alpha, const double* mu,
                           int n_mu, double delta, float* const* ckpt, const float* const* df, double* dmu,
                           double* dalpha, double* dpsf, float* const* dg, hipStream_t stream);

/* ---- phase and kernel timing (profiling aid) -----------------------------
 * Phases of one iteration of eq. (MLBA2) as the library runs them. */
#define MLBA_PHASE_SYNTHESIS 0  /* x = delta S_mu(z), u = W^T x                        */
#define MLBA_PHASE_BLUR      1  /* r = g - A u and ||r||^2 (with the FFT blur and the
                                   BCCB or DCT preconditioner also the
                                   preconditioner's forward row pass, fused with
                                   the residual's)                                  */
#define MLBA_PHASE_PRECOND   2  /* t = P_alpha r (the transform passes)              */
#define MLBA_PHASE_BLUR_T    3  /* w = A^T t (fused FFT path: from the
                                   preconditioner's inverse row pass on)            */
#define MLBA_PHASE_ANALYSIS  4  /* z += W w                                          */
#define MLBA_NPHASES         5
/* Kernels (one launch each unless noted). */
#define MLBA_KERNEL_SYNTHESIS_LEVEL   0  /* thresholded synthesis of one level (z state) */
#define MLBA_KERNEL_LOWPASS_LEVEL     1  /* low-pass of one level (omega state)          */
#define MLBA_KERNEL_SHRINK_SYNTHESIS  2  /* bands, threshold, synthesis of one level     */
#define MLBA_KERNEL_CONV_BLUR         3  /* direct r = g - A u                           */
#define MLBA_KERNEL_CONV_BLUR_T       4  /* direct A^T t (accumulating for omega)        */
#define MLBA_KERNEL_FOLD_REFLECT      5  /* fold of the reflective padding               */
#define MLBA_KERNEL_REDUCE            6  /* sum of the ||r||^2 partials                  */
#define MLBA_KERNEL_FFT_ROWS_FWD      7  /* preconditioner: forward row pass             */
#define MLBA_KERNEL_FFT_COLS          8  /* preconditioner: column pass with the filter  */
#define MLBA_KERNEL_FFT_ROWS_INV      9  /* preconditioner: inverse row pass             */
#define MLBA_KERNEL_FC_ROWS_FWD      10  /* FFT blur: forward row pass                   */
#define MLBA_KERNEL_FC_COLS          11  /* FFT blur: column pass (p-tap convolution
                                            along y, or the transform pair)       */
#define MLBA_KERNEL_FC_ROWS_INV      12  /* FFT blur: inverse row pass                   */
#define MLBA_KERNEL_FC_RESIDUAL_PRECOND_ROWS 13  /* fused residual rows + preconditioner
                                                    forward rows                        */
#define MLBA_KERNEL_PRECOND_ROWS_FC_FWD      14  /* fused preconditioner inverse rows +
                                                    A^T forward rows                    */
#define MLBA_KERNEL_ANALYSIS_LEVEL   15  /* analysis + Bregman update of one level       */
#define MLBA_KERNEL_OTHER            16  /* launch sequences timed as one: the 4-NS
                                            Newton steps, the PCG of Algorithm 2, copies */
#define MLBA_NKERNELS                17
/* mlba_profile_begin: the following mlba_restore calls on this plan record HIP
 * events on their stream (one at the start of an iteration and one after each
 * launch or launch sequence of the table above) for at most max_iters
 * iterations in total (host-side event objects, no device memory).
 * mlba_profile_end: waits for those events and writes, per phase, the summed
 * milliseconds (ms[MLBA_NPHASES], host) and the number of kernel launches
 * (launches[MLBA_NPHASES], host, optional), plus the number of iterations
 * recorded (iters, optional); keeps the per-kernel sums for
 * mlba_profile_kernels and releases the events.
 * mlba_profile_kernels: the per-kernel milliseconds (ms[MLBA_NKERNELS]) and
 * launch counts (launches[MLBA_NKERNELS], optional) of the last
 * mlba_profile_end (zero before one). */
int mlba_profile_begin(mlba_plan_t plan, int max_iters);
/* mlba_profile_every: after mlba_profile_begin, record only every stride-th
 * iteration (stride >= 1; the default 1 records every one), counting from the
 * first iteration after this call.  The recorded iterations still count
 * against max_iters. */
int mlba_profile_every(mlba_plan_t plan, int stride);
int mlba_profile_end(mlba_plan_t plan, double* ms, int* launches, int* iters);
int mlba_profile_kernels(mlba_plan_t plan, double* ms, int* launches);

#ifdef __cplusplus
}
#endif

#endif /* MLBA_H */

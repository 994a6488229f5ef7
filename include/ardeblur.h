/*
 * ardeblur.h -- C ABI of the MI355X (gfx950) library for preconditioned
 * Landweber deblurring under Anti-Reflective (AR) boundary conditions.
 *
 * Method: Dell'Acqua, Serra-Capizzano, Tablino-Possio, "Optimal
 * preconditioning for image deblurring with Anti-Reflective boundary
 * conditions" (arXiv 1211.0393).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Images are n1 x n2, row-major: i1 (row) is the slow axis, i2 (column)
 *    the fast, contiguous one (Sec. 1: row-wise ordering from the top-left
 *    corner).  Element (i1, i2) sits at offset i1 * n2 + i2.
 *  - Image buffers are DEVICE pointers on the plan's device, owned by the
 *    caller; the library never frees them.  Their element type is the plan's
 *    storage type (double for AR_F64, float for the other dtypes) unless
 *    stated otherwise.
 *  - The PSF is a HOST array of (2 q1 + 1) x (2 q2 + 1) doubles, row-major,
 *    psf[(q1 + s1) * (2 q2 + 1) + (q2 + s2)] = h_{s1,s2} (eq.
 *    (coefficienti_psf)).  It must be finite, nonnegative, sum to 1 within
 *    1e-12 * (number of taps), and satisfy the support condition of Sec. 2.2
 *    (q_j <= n_j - 3; n_j >= 3).  It is copied at plan creation.
 *  - The blur is a true convolution g_i = sum_s h_s f_{i-s}
 *    (eq. (modello_discreto)) of the AR-extended image (Sec. 2.2).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Every call is stream-ordered and asynchronous unless it returns host
 *    scalars (then it synchronizes that stream before returning).
 *  - Every function returns AR_OK (0) or a negative ar_status; on failure
 *    ar_last_error() gives a message (thread-local).  No call aborts.
 *  - A plan may be used by one host thread at a time; its scratch buffers
 *    are shared by all calls on it, so calls on one plan must not overlap
 *    on different streams.  Distinct plans are independent.
 */
#ifndef ARDEBLUR_H
#define ARDEBLUR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ar_plan_s *ar_plan_t;

/* Precision of a plan.
 *  AR_F32       : float images, float arithmetic in blur and transforms.
 *  AR_F64       : double images and arithmetic.
 *  AR_F32_ACC64 : float images; blur accumulation, boundary extension and
 *                 transforms computed in double (full rate on gfx950 when
 *                 packed FP32 is not used), intermediates stored as float.
 *  AR_F32_BF16X3: float images and blur; each axis of the AR transform is
 *                 applied as one dense m x m matrix product on the matrix
 *                 cores, operands split into two BF16 terms (hi + lo, three
 *                 products hi*hi + hi*lo + lo*hi), FP32 accumulation; about
 *                 1e-5 relative error per transform pass.
 * Eigenvalues, the filter division and all norms are FP64 in every mode. */
enum ar_dtype { AR_F32 = 0, AR_F64 = 1, AR_F32_ACC64 = 2, AR_F32_BF16X3 = 3 };

/* Transpose used by the iteration: the reblurring A' = A(PSF rotated by
 * 180 degrees) that the paper's experiments use (Sec. 4), or the exact
 * transpose A^T written in eq. (LandweberMeth). */
enum ar_tmode { AR_REBLUR = 0, AR_ADJOINT = 1 };

/* Eigenvalue filter giving the spectrum d of the preconditioner D.
 *  TIKHONOV : d = 1 / (lambda^2 + param)          (eq. (TikFilter))
 *  THRESHOLD: d = 1 / lambda^2 if |lambda| >= param, else 1
 *             (truncated-spectrum filter; not in the paper)
 *  GAINS    : learned per-radial-bin gains phi (set by ar_precond_set_gains)
 *  IDENTITY : d = 1 (D = I, plain Landweber)                           */
enum ar_filter { AR_FILTER_TIKHONOV = 0, AR_FILTER_THRESHOLD = 1, AR_FILTER_GAINS = 2,
                 AR_FILTER_IDENTITY = 3 };

enum ar_status {
  AR_OK = 0,
  AR_EINVAL = -1,       /* bad argument (null pointer, unknown enum, iters < 0, ...) */
  AR_ESHAPE = -2,       /* n_j < 3 or q_j > n_j - 3 or sizes too large */
  AR_EPSF = -3,         /* PSF entry negative / non-finite, or sum != 1 */
  AR_EALIAS = -4,       /* input and output buffers alias where forbidden */
  AR_EDEVICE = -5,      /* HIP runtime error (message has the HIP string) */
  AR_ENOMEM = -6,       /* device allocation failed */
  AR_ENONFINITE = -7,   /* a residual norm became NaN or Inf during iteration */
  AR_EUNSUPPORTED = -8  /* valid request this build does not implement */
};

/* Boundary conditions of a plan.  AR_BC_ANTIREFLECTIVE is the method of
 * this library (Sec. 2.2, Theorem 1); the other two are the comparators of
 * the paper's experiments (Sec. 4, Tables 1-2):
 *  AR_BC_REFLECTIVE: f_{1-i} = f_i, f_{n+i} = f_{n+1-i} (Sec. 2.1); the
 *      preconditioner is R diag(d) R^T with R^T the orthonormal 2-D DCT-II
 *      (eq. (Rn)) and lambda the symbol of the symmetrized PSF at
 *      x_k = k pi / n, k = 0..n-1 (natural order);
 *  AR_BC_PERIODIC: wrap-around extension; the preconditioner is
 *      F^{-1} diag(d) F with F the 2-D DFT and lambda the DFT of the PSF
 *      itself (not symmetrized, natural FFT order); d = 1/(|lambda|^2 + alpha).
 * The reblurring A' (PSF rotated by 180 degrees) is the transpose of every
 * iteration (for periodic BCs it equals A^T). */
enum ar_bc { AR_BC_ANTIREFLECTIVE = 0, AR_BC_REFLECTIVE = 1, AR_BC_PERIODIC = 2 };

/* Create a plan for n1 x n2 images and one PSF (S0-S2 of the path):
 * validates the arguments, copies the PSF to the device, and on the device
 * builds the blur weights, the symmetrized PSF
 *   s_{+-i1,+-i2} = (h_{-i1,-i2} + h_{-i1,i2} + h_{i1,-i2} + h_{i1,i2}) / 4
 * (Theorem 4, eq. (simmetrizzata2d-bis)), its eigenvalues lambda in FP64
 * on the extended grid of Theorem 2 (column order of T_{n1} (x) T_{n2}),
 * and the default Tikhonov filter with param = 1e-2.  Device scratch for
 * the iteration is allocated here and owned by the plan.
 *   out    : receives the plan (set to NULL on failure)
 *   dtype  : an ar_dtype
 *   device : HIP device ordinal the plan lives on
 * Errors: AR_EINVAL, AR_ESHAPE, AR_EPSF, AR_EDEVICE, AR_ENOMEM. */
int ar_plan_create(ar_plan_t *out, int n1, int n2, const double *psf_host,
                   int q1, int q2, int dtype, int device);

/* ar_plan_create under boundary conditions `bc` (an ar_bc; ar_plan_create is
 * this call with AR_BC_ANTIREFLECTIVE).  For Reflective and Periodic plans:
 * the blur extends the image by the plan's rule; ar_blur_apply_T supports
 * AR_REBLUR only (AR_ADJOINT: AR_EUNSUPPORTED); ar_transform and
 * ar_transform_inv apply R^T and R for Reflective plans (AR_EUNSUPPORTED for
 * Periodic plans, whose coefficients are complex); ar_eigenvalues gives
 * lambda for Reflective plans and |lambda| for Periodic plans;
 * ar_precond_set takes the Tikhonov, threshold and identity filters;
 * ar_precond_solve, ar_deblur_iterate (AR_REBLUR) and, for Reflective plans
 * with a strongly symmetric PSF, ar_tikhonov_solve work as documented.
 * ar_iterate_profile times the same five phases (AR_REBLUR).  dtype
 * AR_F32_BF16X3, batches, the learned filter (ar_features, the gains filter)
 * and ar_plan_tune / ar_plan_autotune are Anti-Reflective only
 * (AR_EUNSUPPORTED).  n_j >= 3, q_j <= n_j - 3.
 * Errors: as ar_plan_create; AR_EINVAL for an unknown bc. */
int ar_plan_create_bc(ar_plan_t *out, int n1, int n2, const double *psf_host, int q1, int q2,
                      int dtype, int bc, int device);

/* Release a plan and its device memory (waits for the device).  NULL is a
 * no-op returning AR_OK. */
int ar_plan_destroy(ar_plan_t p);

/* y = A_n x: AR extension of x (edges f_{1-i} = 2 f_1 - f_{1+i},
 * f_{n+i} = 2 f_n - f_{n-i}; corners by double anti-reflection, Sec. 2.2)
 * followed by the convolution of eq. (modello_discreto).
 * x, y: device, n1*n2, plan dtype; x == y is rejected (AR_EALIAS). */
int ar_blur_apply(ar_plan_t p, const void *x, void *y, void *stream);

/* y = A' r (tmode AR_REBLUR: the blur with the PSF rotated by 180 degrees,
 * Sec. 4) or y = A_n^T r (tmode AR_ADJOINT: exact transpose, i.e. the
 * correlation with h scattered to the extended grid and folded back with
 * the transposed AR weights +2 / -1 per axis).
 * r, y: device, n1*n2, plan dtype; r == y is rejected (AR_EALIAS). */
int ar_blur_apply_T(ar_plan_t p, const void *r, void *y, int tmode, void *stream);

/* c = T~ x with T~ = T~_{n1} (x) T~_{n2}, the inverse of the AR transform
 * of Theorem 1: per axis of length m, c_1 = alpha_m x_1, c_m = alpha_m x_m,
 * c_mid = Q_{m-2} (x_mid - x_1 p - x_m J p), p_j = 1 - j/(m-1), Q the DST-I
 * matrix of eq. (Qn), alpha_m = sqrt(m (2m-1) / (6 (m-1))).
 * Coefficients are stored n1 x n2 in the column order of T.
 * x, c: device, plan dtype; x == c (in place) is allowed. */
int ar_transform(ar_plan_t p, const void *x, void *c, void *stream);

/* x = T c, the AR transform of Theorem 1 (inverse of ar_transform):
 * x_1 = c_1 / alpha, x_m = c_m / alpha, x_mid = Q c_mid + x_1 p + x_m J p.
 * c, x: device, plan dtype; in place allowed. */
int ar_transform_inv(ar_plan_t p, const void *c, void *x, void *stream);

/* Set the preconditioner spectrum d from lambda (Sec. 4): filter is an
 * ar_filter, param its parameter (Tikhonov alpha > 0, threshold t > 0,
 * ignored for IDENTITY and GAINS).  For AR_FILTER_GAINS, gains_dev is a
 * DEVICE array of AR_FNET_BINS floats in [0, 1] (the learned filter below;
 * the same as ar_precond_set_gains); for the other filters it is ignored
 * and may be NULL.  Computed in FP64 on the device; stored in FP64 and in
 * the plan dtype.  Stream-ordered.  Errors: AR_EINVAL (unknown filter,
 * parameter not finite and > 0, GAINS without gains). */
int ar_precond_set(ar_plan_t p, int filter, double param, const float *gains_dev, void *stream);

/* Host helper (no device work): divide a HOST PSF of (2 q1 + 1) x (2 q2 + 1)
 * doubles by its sum in place, so that it satisfies the normalisation
 * sum h = 1 that the plan functions check (Sec. 2, the PSF is nonnegative
 * and sums to one).  The library never renormalises a PSF silently.
 * Errors: AR_EINVAL (NULL), AR_ESHAPE (negative half-width), AR_EPSF (an
 * entry negative or not finite, or a sum that is not positive and finite;
 * the array is left unchanged). */
int ar_psf_normalize(double *psf_host, int q1, int q2);

/* Copy the FP64 eigenvalues lambda (n1*n2, coefficient layout) of the
 * symmetrized PSF's AR matrix into the device buffer lambda_dev. */
int ar_eigenvalues(ar_plan_t p, double *lambda_dev, void *stream);

/* Copy the FP64 filter spectrum d (n1*n2) into the device buffer d_dev. */
int ar_filter_values(ar_plan_t p, double *d_dev, void *stream);

/* z = D y with D = T diag(d) T~ (Sec. 4; for the Tikhonov filter this is
 * (P(s)^2 + alpha I)^{-1} y, P(s) the AR matrix of the symmetrized PSF).
 * y, z: device, plan dtype; y == z allowed. */
int ar_precond_solve(ar_plan_t p, const void *y, void *z, void *stream);

/* Direct Tikhonov restoration for a strongly symmetric PSF
 * (h_{-s1,s2} = h_{s1,-s2} = h_{s1,s2}, eq. (strong_simmetry_condition)):
 * then A = T diag(lambda) T~ with lambda the eigenvalues of Theorem 2, the
 * reblurring A' equals A, and the Tikhonov solution
 * x = (A'A + alpha I)^{-1} A' g is T diag(lambda / (lambda^2 + alpha)) T~ g
 * (Theorems 1-2 with eq. (TikFilter)); the factor is formed in FP64.
 * g, x: device, n1*n2, plan dtype; x == g (in place) is allowed.
 * Symmetry is checked on the host PSF (plan creation or ar_plan_set_psf)
 * to 1e-14 of its largest entry.  Stream-ordered.
 * Errors: AR_EINVAL (NULL, alpha not finite and > 0), AR_EPSF (the plan's
 * PSF is not strongly symmetric). */
int ar_tikhonov_solve(ar_plan_t p, const void *g, void *x, double alpha, void *stream);

/* Run `iters` steps of (D-)Landweber (eqs. (LandweberMeth) and
 * (DLandweberMeth)):  x_{k+1} = x_k + tau D A'(g - A x_k)  with A' chosen
 * by tmode and D = I when precondition == 0.
 *   g       : device, n1*n2, plan dtype (observed image)
 *   x       : device, n1*n2, plan dtype; in: x_0, out: x_iters
 *   f_true  : device or NULL; when given, RRE_k = ||x_k - f||_F / ||f||_F
 *             is accumulated in FP64 for k = 1..iters
 *   resnorm_host : host array of iters doubles or NULL:
 *             resnorm[k] = ||g - A x_k||_F (FP64 accumulation), k = 0..iters-1
 *   rre_host     : host array of iters doubles or NULL: rre[k] = RRE(x_{k+1})
 *   best_it_host : host int or NULL: first k >= 1 minimising RRE(x_k)
 *                  (needs f_true)
 * Host outputs imply one synchronization at the end.  If a requested
 * residual norm is not finite the call returns AR_ENONFINITE (x holds the
 * last iterate).  g, x, f_true must not alias. */
int ar_deblur_iterate(ar_plan_t p, const void *g, void *x, int iters, double tau,
                      int tmode, int precondition, const void *f_true,
                      double *resnorm_host, double *rre_host, int *best_it_host,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * iteration and outputs as ar_deblur_iterate (the same kernels, so x and
 * the scalars are bitwise equal), with no hipMalloc, hipFree or other
 * allocation in the call.  Its partial sums and reduced scalars live in a
 * static device buffer of 2 MiB (262144 doubles) that each GPU the library
 * runs on holds until the process ends; a run with scalars requested needs
 * iters * (residual + update partials) + 2 iters + 1 doubles of it (at
 * 1024 x 1024 about 770 per iteration, so up to ~340 iterations per call).
 * Differences from ar_deblur_iterate: best_it_host needs rre_host (the call
 * keeps no host buffer of its own); sizes beyond the buffer return
 * AR_EINVAL before any device work.  Calls that overlap on one GPU share the
 * buffer and race: order them on one stream.  The plan's own scratch (r, y,
 * c) is allocated by ar_plan_create, as for every entry point. */
int ar_deblur_iterate_noalloc(ar_plan_t p, const void *g, void *x, int iters, double tau,
                              int tmode, int precondition, const void *f_true,
                              double *resnorm_host, double *rre_host, int *best_it_host,
                              void *stream);

/* Launch tunables of a plan (they change speed; where they change the
 * arithmetic, results agree to rounding, as stated below).
 *  AR_TUNE_ROW_WAVES / AR_TUNE_COL_WAVES : rows (columns) transformed per
 *      workgroup by the wave-per-sequence transform, 1, 2 or 4 (0 = auto);
 *      on an axis of length 1024, the FP64-arithmetic passes of a workgroup
 *      with an even count take its rows (columns) in pairs, two per complex
 *      FFT (a pre-weighted DST-I form with a running sum for the odd
 *      outputs), equal to the one-per-FFT form up to rounding
 *  AR_TUNE_ROW_EXCL / AR_TUNE_COL_EXCL   : 1 = reserve a whole CU per
 *      workgroup of that pass (spreads few workgroups over all CUs)
 *  AR_TUNE_ROW_ALGO / AR_TUNE_COL_ALGO   : FFT of the DST-I, 1 = mixed
 *      radix (only when every prime factor of n - 1 is <= 31), 2 = Bluestein
 *      chirp-z with a power-of-two FFT (any length); 0 = auto
 *  AR_TUNE_ROW_LANES / AR_TUNE_COL_LANES : wavefronts per sequence, 1, 2
 *      or 4 (0 = auto: 2 for an axis of length 1024, else 1); with G of
 *      them, a row's (column's) butterflies and elements are dealt to 64 G
 *      lanes; an axis of length 1024 with G = 2 or 4 runs the length-1024
 *      kernels, which deal the output pairs of the radix-31 (and, G = 4,
 *      radix-11) butterflies to the G wavefronts
 *  AR_TUNE_BLUR : engine of the FP32 blur of A x and A' r: 0 = automatic
 *      (the matrix cores when q1 <= 10 and q2 <= 8 at plan creation; the
 *      autotuner leaves it alone), 1 = vector ALU, 2 = matrix cores (FP16 hi/lo operands, three products,
 *      FP32 accumulation, exact power-of-two scaling; about 2^-21 relative
 *      per product against FP32's 2^-24).  This one changes results in the
 *      last bits; the batched executor always uses the vector-ALU blur.
 *  AR_TUNE_FUSE : with the matrix-core blur and the reblurring transpose, 1 =
 *      one kernel computes r = g - A x on the reblur's halo and y = A' r
 *      (Anti-Reflective and Reflective plans), 0 = two kernels (default).
 *      Same products; the residual's scale comes from a wider halo, so
 *      results can differ in the last bits of the smallest values. */
enum ar_tune_key { AR_TUNE_ROW_WAVES = 0, AR_TUNE_COL_WAVES = 1, AR_TUNE_ROW_EXCL = 2,
                   AR_TUNE_COL_EXCL = 3, AR_TUNE_ROW_ALGO = 4, AR_TUNE_COL_ALGO = 5,
                   AR_TUNE_ROW_LANES = 6, AR_TUNE_COL_LANES = 7, AR_TUNE_BLUR = 8,
                   AR_TUNE_FUSE = 9 };

/* Set one tunable (value 0 restores the automatic choice).  Errors:
 * AR_EINVAL for an unknown key or value. */
int ar_plan_tune(ar_plan_t p, int key, int value);

/* Read a tunable's current value into *value. */
int ar_plan_get_tune(ar_plan_t p, int key, int *value);

/* Autotuner: times every candidate setting of the transform tunables with
 * HIP events on `stream`, one axis after the other, on short runs of whole
 * preconditioned iterations (reblur transpose) over zero images in buffers
 * it allocates and frees, keeps the fastest, and returns the best measured
 * time of one iteration in *best_us (may be NULL).  Uses and overwrites the
 * plan's scratch; synchronizes `stream`.  Errors: AR_ENOMEM when the
 * temporary buffers cannot be allocated, AR_EDEVICE on other HIP errors. */
int ar_plan_autotune(ar_plan_t p, double *best_us, void *stream);

/* Phase profiler of one (D-)Landweber iteration: after one untimed
 * iteration (on a private copy of x; x and g are only read), each phase's
 * kernel is launched `reps` times back to back between two HIP events on
 * `stream`; phase_us[0..4] receives the average duration per launch in
 * microseconds:
 *   0: r = g - A x (residual blur with FP64 norm partials); with the fused
 *      residual and reblur (AR_TUNE_FUSE = 1), y = A' (g - A x) in one kernel
 *   1: y = A' r or A^T r (transpose blur; correlation + fold for A^T); 0
 *      with the fused kernel
 *   2: row pass of T~ (0 when precondition == 0)
 *   3: column pass T~ / d / T (0 when precondition == 0)
 *   4: row pass of T fused with x += tau w (the plain update when
 *      precondition == 0)
 * x, g: device, plan dtype; reps >= 1. */
int ar_iterate_profile(ar_plan_t p, const void *g, const void *x, int tmode, int precondition,
                       int reps, double *phase_us, void *stream);

/* ------------------------------------------------------------------
 * Batched executor: many independent deblurring problems of uneven sizes,
 * each with its own plan (PSF, eigenvalues, filter), iterated together.
 * Problems are grouped by PSF column half-width (one blur launch per group)
 * and by image shape (one transform launch per group, sharing the FFT
 * tables); every launch covers all problems of its group, and the whole
 * run of `iters` iterations is captured once into a HIP graph that
 * ar_batch_iterate replays with a single graph launch.
 * ------------------------------------------------------------------ */
typedef struct ar_batch_s *ar_batch_t;

/* Create a batch over `count` plans (host array).  The plans must be
 * distinct, share one dtype (not AR_F32_BF16X3) and device, and outlive the batch; the batch
 * runs on their scratch buffers, so a plan must not be used on its own
 * while a batch call that includes it is in flight.  Every image shape of
 * the batch must fit the wave-per-sequence transform (n <= 2048 for
 * AR_F32, n <= 1024 for the double-arithmetic dtypes).  `stream` is used
 * for set-up copies and synchronized.
 * Errors: AR_EINVAL (null, count < 1, repeated plan, mixed dtype/device),
 * AR_EUNSUPPORTED, AR_EDEVICE, AR_ENOMEM. */
int ar_batch_create(ar_batch_t *out, int count, const ar_plan_t *plans, void *stream);

/* Autotuner of a batch: for every shape group, times each candidate
 * transform setting (FFT form, waves per workgroup, CU-exclusive
 * workgroups) on the batched launches themselves and stores the fastest
 * in every plan of the group (batched launches use the settings of the
 * group's first plan).
 * *best_us (may be NULL) receives the tuned time of one batched
 * preconditioner application.  Uses the plans' scratch; synchronizes. */
int ar_batch_autotune(ar_batch_t b, double *best_us, void *stream);

/* Run `iters` (D-)Landweber steps on every problem of the batch, exactly
 * the recurrence of ar_deblur_iterate applied to each problem with its
 * plan's filter.
 *   g, x      : host arrays of `count` device pointers (problem i has its
 *               plan's shape and dtype); x is in/out
 *   f_true    : NULL or a host array of `count` device pointers
 *   resnorm_host : NULL or count*iters doubles, [i * iters + k] = ||r_k|| of problem i
 *   rre_host     : NULL or count*iters doubles (needs f_true)
 *   best_it_host : NULL or count ints (needs f_true)
 * The first call for a given (iters, tau, tmode, precondition, outputs,
 * launch settings) captures the graph; later calls only update the
 * device-side job tables and replay it.  Calls on one batch must be
 * ordered (same stream, or synchronized between).
 * Errors as ar_deblur_iterate; AR_ENONFINITE if any requested residual
 * norm is not finite; AR_ESHAPE if a plan's PSF half-widths changed (via
 * ar_plan_set_psf) since ar_batch_create (the batch's blur groups, LDS
 * sizes and tile tables were laid out for the old ones). */
int ar_batch_iterate(ar_batch_t b, const void *const *g, void *const *x, int iters, double tau,
                     int tmode, int precondition, const void *const *f_true,
                     double *resnorm_host, double *rre_host, int *best_it_host, void *stream);

/* Release a batch (not its plans).  NULL is a no-op returning AR_OK. */
int ar_batch_destroy(ar_batch_t b);

/* Replace the PSF of a plan (S0-S2 again: weights, symmetrized PSF,
 * eigenvalues, and the current filter re-applied) without reallocating.
 * The new half-widths must not exceed those the plan was created with;
 * the PSF rules of ar_plan_create apply.  Synchronizes `stream`.  A batch
 * that includes the plan must be re-created if q1 or q2 changes.
 * Errors: AR_EINVAL, AR_ESHAPE (q larger than at creation), AR_EPSF. */
int ar_plan_set_psf(ar_plan_t p, const double *psf_host, int q1, int q2, void *stream);

/* ------------------------------------------------------------------
 * Learned preconditioner filter (not part of the paper's method: the
 * paper's filter is Tikhonov, eq. (TikFilter)).  A small network maps
 * per-problem features to 64 gains g_b in [0, 1] that set a Tikhonov
 * parameter per eigenvalue-magnitude bin:
 *   d = 1 / (lambda^2 + a_b),  a_b = 10^(-6 + 6 g_b),
 *   b = ebin(lambda) = #{j in 1..63 : |lambda| >= 10^(-4 + j/16)}.
 * Radial bins of the features: coefficient (k1, k2) has x_j = r_j pi /
 * (n_j - 1) with r_j = k_j on interior columns of T and 0 on the first and
 * last one (the grid of Theorem 2); rho = sqrt((x1/pi)^2 + (x2/pi)^2) /
 * sqrt(2) and rbin = min(floor(64 rho), 63), decided exactly in integers.
 * ------------------------------------------------------------------ */
enum { AR_FNET_BINS = 64, AR_FNET_IN = 65, AR_FNET_HIDDEN = 128, AR_FNET_NPARAM = 33216 };

/* Features of one problem into feat_dev (device, 65 floats):
 *  [0, 64): mean FP64 eigenvalue lambda of the plan per radial bin (0 for
 *           an empty bin);
 *  64     : log(nu_hat), the noise estimate of g: L = 5-point Laplacian
 *           (0 1 0 / 1 -4 1 / 0 1 0) on the interior pixels, sigma =
 *           lmed(|L - lmed(L)|) / 0.6745 / sqrt(20) with lmed the lower
 *           median (rank floor((N-1)/2)), nu_hat = sigma sqrt(n1 n2) / ||g||_F.
 * g: device, n1*n2, plan dtype.  Uses the plan's scratch.  Errors: AR_EINVAL. */
int ar_features(ar_plan_t p, const void *g, float *feat_dev, void *stream);

/* Set the spectrum from gains (device, 64 floats in [0, 1]) as above, in
 * FP64; the filter becomes AR_FILTER_GAINS and is kept across
 * ar_plan_set_psf.  Errors: AR_EINVAL. */
int ar_precond_set_gains(ar_plan_t p, const float *gains_dev, void *stream);

/* Training label of the plan's current filter (64 floats, device): with
 * the bin centre c_b = 10^(-4 + (b + 1/2)/16) and a_b = 1/d(c_b) - c_b^2
 * (Tikhonov: alpha; threshold: 0 above t, 1 - c_b^2 below; identity:
 * 1 - c_b^2), label_b = (log10(clip(a_b, 1e-6, 1)) + 6) / 6. */
int ar_gains_label(ar_plan_t p, float *label_dev, void *stream);

/* Filter network 65 -> 128 -> 128 -> 64 (ReLU, ReLU, logistic sigmoid).
 * Parameters (AR_FNET_NPARAM floats, host, in this order): W1 (128 x 65),
 * b1 (128), W2 (128 x 128), b2 (128), W3 (64 x 128), b3 (64); each W is
 * (out, in) row-major.  The network keeps FP32 master weights and Adam
 * moments; its forward pass uses the weights rounded to BF16 (round to
 * nearest even) on MFMA with FP32 accumulation, activations entering a
 * layer split into two BF16 terms (hi + lo); biases stay FP32. */
typedef struct ar_fnet_s *ar_fnet_t;

/* Create a network on `device` from initial parameters (host); the random
 * initialisation is the caller's.  Errors: AR_EINVAL, AR_EDEVICE, AR_ENOMEM. */
int ar_fnet_create(ar_fnet_t *out, const float *params_host, int device);

/* Create a network on `device` from a weights file: a NumPy .npy file
 * (format 1.0-3.0) holding one C-order little-endian float32 vector of
 * AR_FNET_NPARAM parameters in the layout above (the trained weights ship
 * as paper_1211_0393_amd/fnet_weights.npy).  Errors: AR_EINVAL (NULL, file
 * missing or not such a vector, non-finite parameter), AR_EDEVICE,
 * AR_ENOMEM. */
int ar_fnet_load(ar_fnet_t *out, const char *weights_path, int device);

/* Release a network.  NULL is a no-op. */
int ar_fnet_destroy(ar_fnet_t net);

/* Copy the FP32 master parameters to the host (synchronizes the device). */
int ar_fnet_get_params(ar_fnet_t net, float *params_host);

/* y (batch x 64) = network(x (batch x 65)); device FP32 buffers, batch >= 1. */
int ar_fnet_infer(ar_fnet_t net, const float *x_dev, float *y_dev, int batch, void *stream);

/* Gradient of the loss mean((y - t)^2) over batch x 64 with respect to the
 * parameters (layout above) at the current BF16 weights, into grad_dev
 * (device, AR_FNET_NPARAM floats); the loss into loss_dev (device float,
 * may be NULL).  x: batch x 65, t: batch x 64, device FP32. */
int ar_fnet_grad(ar_fnet_t net, const float *x_dev, const float *t_dev, int batch,
                 float *grad_dev, float *loss_dev, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * counter kept by the network) on the gradient above with learning rate
 * lr; refreshes the BF16 weights.  loss_dev as in ar_fnet_grad. */
int ar_fnet_train_step(ar_fnet_t net, const float *x_dev, const float *t_dev, int batch,
                       float lr, float *loss_dev, void *stream);

/* Thread-local message describing the last failure ("" if none). */
const char *ar_last_error(void);

/* Library version string. */
const char *ar_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ARDEBLUR_H */

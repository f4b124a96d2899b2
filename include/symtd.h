/*
 * symtd: implicit symmetric CP decomposition of moment tensors on AMD MI355X.
 *
 * The method is that of Sherman & Kolda, "Estimating higher-order moments
 * using symmetric tensor decomposition" (arXiv 1911.03813).  The data tensor
 * is the d-th empirical moment X = sum_l nu_l v_l^{(x)d} (eq. (tensorX)),
 * given only by its weights nu (p) and observations V (n x p, one column per
 * observation).  The model is M = sum_j lambda_j a_j^{(x)d} with weights
 * lambda (r) and factors A (n x r) (eq. (cp_element)).  The objective is
 * f(lambda, A) = ||X - M||^2 (eq. (optFunc)); X is never formed.
 *
 * Conventions for every call:
 *   - Matrices are column-major with a leading dimension (ldv, lda, ldg >= n).
 *   - Array arguments are DEVICE pointers unless stated otherwise; the caller
 *     owns them; the library keeps no caller pointer after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Evaluation calls are stream-ordered and asynchronous: they return
 *     before the GPU has finished, and results are valid once the stream
 *     reaches that point.
 *   - Errors found while checking arguments return a negative status and
 *     launch nothing; symtd_last_error() then describes the problem.  HIP
 *     errors are returned as SYMTD_EDEVICE with the HIP message attached.
 *   - Errors found on the device during an asynchronous call (a split
 *     product's bounded wait for a neighbouring block that gave up, which
 *     leaves that call's results invalid) are recorded in the context and
 *     returned as SYMTD_EDEVICE by the next call on the context made after
 *     the device recorded them, or by symtd_check; the record is then
 *     cleared, and later calls run normally.
 *   - A context is not thread-safe and serves one stream at a time: use one
 *     per host thread, and do not let calls on different streams overlap.
 */
#ifndef SYMTD_H
#define SYMTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum symtd_status {
  SYMTD_OK = 0,
  SYMTD_EINVAL = -1,       /* bad size, order, leading dimension, null pointer or dtype/precision pair */
  SYMTD_EALIGN = -2,       /* pointer not aligned to its element size */
  SYMTD_ENOMEM = -3,       /* device workspace could not be allocated */
  SYMTD_EDEVICE = -4,      /* a HIP call failed; the message carries HIP's error string */
  SYMTD_EUNSUPPORTED = -5, /* the device is not a gfx950 (MI355X-class) GPU */
  SYMTD_ENONFINITE = -6,   /* a non-finite value was found where the call checks for one */
  SYMTD_EREJECTED = -7     /* a request exceeds the configured device-memory budget */
} symtd_status;

/* Storage type of V, A and G_A. nu, lambda, g_lambda, f and alpha are always fp64. */
typedef enum symtd_dtype { SYMTD_F64 = 0, SYMTD_F32 = 1 } symtd_dtype;

/* Arithmetic used for the two products V'A and V*W of eq. (Y).
 *   SYMTD_PREC_FP64: fp64 matrix-core products (needs SYMTD_F64 storage).
 *   SYMTD_PREC_FP32: fp32 matrix-core products (needs SYMTD_F32 storage).
 *   SYMTD_PREC_FP16: fp16 operands (V, A and W = nu z^{d-1}, the latter times a
 *                    power of two that keeps it in fp16's normal range), fp32
 *                    accumulation; through a data handle (symtd_data_create).
 *   SYMTD_PREC_BF16X3: every operand split as hi + lo with hi = bf16(x),
 *                    lo = bf16(x - hi); products hi hi + hi lo + lo hi with fp32
 *                    accumulation; through a data handle.
 * In every precision the column sums w_j, the split reductions, B = A'A,
 * u, f and g_lambda are accumulated in fp64.  Stated bounds (errors relative
 * to the cancelling terms, d = 3): fp64 1e-12, fp32 1e-5, and worst cases
 * bf16x3 2 (d+1) 3 2^-16 = 3.7e-4, fp16 2 (d+1) 2 2^-11 = 7.8e-3; the
 * measured 16-bit errors sit far below these (bf16x3 about 1e-2 of what
 * plain bf16 products make, fp16 within a few times a model of its own
 * roundings), and the tests check those tighter per-shape bounds. */
typedef enum symtd_prec {
  SYMTD_PREC_FP64 = 0, SYMTD_PREC_FP32 = 1, SYMTD_PREC_FP16 = 2, SYMTD_PREC_BF16X3 = 3
} symtd_prec;

typedef struct symtd_ctx symtd_ctx;

/* Create a context on HIP device `device`. The context owns a device
 * workspace that grows on demand (growing synchronises the device).
 * Returns SYMTD_EUNSUPPORTED if the device is not gfx950. */
symtd_status symtd_create(int device, symtd_ctx** out);

/* Destroy a context and free its workspace. NULL is ignored. */
void symtd_destroy(symtd_ctx* ctx);

/* Message describing the last error on this context ("" if none). The
 * string stays valid until the next call on the context. */
const char* symtd_last_error(const symtd_ctx* ctx);

/* Static name of a status code. */
const char* symtd_status_string(symtd_status s);

/* Wait for `stream` and return SYMTD_EDEVICE if a call on this context
 * recorded a device-side error (see the conventions above), clearing the
 * record; SYMTD_OK otherwise. */
symtd_status symtd_check(symtd_ctx* ctx, void* stream);

/*
 * Objective and gradient, Algorithm 2 (fg_implicit) of the paper:
 *   Y   = V D_nu [V'A]^{d-1}                       eq. (Y), Lemma 3.3
 *   w_j = a_j' y_j = sum_l nu_l <v_l, a_j>^d       Lemma 3.5
 *   B = A'A, C = B^{d-1}, u = (B * C) lambda       (elementwise powers)
 *   f   = alpha + lambda'u - 2 w'lambda            (lambda'u = ||M||^2, Lemma 3.4)
 *   g_lambda = -2 (w - u)                          eq. (gradl)
 *   G_A = -2 d (Y - A D_lambda C) D_lambda         eq. (gradb)
 *
 * dt       storage type of V, A and G_A.
 * V        n x p, leading dimension ldv >= n (column l = observation l).
 * nu       p weights (fp64). Any finite values are accepted.
 * A        n x r, leading dimension lda >= n.
 * lambda   r weights (fp64).
 * d        tensor order, 2 <= d <= 16.
 * alpha    the constant ||X||^2 term (host value); 0 gives the shifted f.
 * prec     product precision (see symtd_prec).
 * f        1 fp64 value (device), g_lambda r fp64 values (device).
 * G_A      n x r of type dt, leading dimension ldg >= n (device).
 * All outputs are fully overwritten. V, nu, A and lambda are read only.
 * Sizes: n, p, r >= 1. Pointers must be aligned to their element size.
 */
symtd_status symtd_fg(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                      const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                      const void* A, int64_t lda, const double* lambda, int64_t r, int d,
                      double alpha, symtd_prec prec,
                      double* f, double* g_lambda, void* G_A, int64_t ldg);

/*
 * symtd_fg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * arguments, results and kernels are those of symtd_fg (the results are the
 * same bits), but the call allocates nothing: its workspace is a fixed
 * array of SYMTD_NOALLOC_SCRATCH_BYTES in device memory, one per GPU that
 * the library runs on, held until the process ends (its address is looked
 * up by symtd_create).  Returns SYMTD_EINVAL if the evaluation's workspace
 * does not fit (it grows with p r + p_splits n r; d = 4, n = 100, p = 5000,
 * r = 20 in fp64 needs about 16 MB, the n = 1000, p = 1e5, r = 100 fp32
 * evaluation 81 MB and does not fit).  Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU, from any context or stream,
 * race; calls in stream order are safe (nothing in the array needs to start
 * at zero).  Per-kernel timing (symtd_profile_*) does not apply to it.
 */
#define SYMTD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
symtd_status symtd_fg_noalloc(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                              const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                              const void* A, int64_t lda, const double* lambda, int64_t r, int d,
                              double alpha, symtd_prec prec,
                              double* f, double* g_lambda, void* G_A, int64_t ldg);

/*
 * Data handles: a data set (V, nu) prepared once for repeated evaluations.
 * For SYMTD_PREC_FP16 and SYMTD_PREC_BF16X3 (fp32 storage) the handle holds
 * one 16-bit copy of V (covariate-contiguous, padded; two bf16 planes for
 * BF16X3) that both products read, converted on `stream`; the call returns
 * after the conversion.  Its device memory is about 2 (fp16) or 4 (bf16x3)
 * bytes per element of V.  For SYMTD_PREC_FP32 / FP64 it only records the
 * pointers.  The caller must keep V and nu unchanged while the handle lives
 * (nu is read at every evaluation).  symtd_fg_data is symtd_fg on the
 * handle's data with the handle's precision; A and G_A have the storage type.
 */
typedef struct symtd_data symtd_data;
symtd_status symtd_data_create(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                               const double* nu, int64_t n, int64_t p, symtd_prec prec, symtd_data** out);
void symtd_data_destroy(symtd_data* data);
symtd_status symtd_fg_data(symtd_ctx* ctx, void* stream, const symtd_data* data, const void* A, int64_t lda,
                           const double* lambda, int64_t r, int d, double alpha, double* f, double* g_lambda,
                           void* G_A, int64_t ldg);

/*
 * Algorithm 2 for several models sharing one data tensor: model m (0 <= m <
 * models) has factors = columns m*r .. m*r + r - 1 of A and weights
 * lambda[m*r .. m*r + r - 1]; its f is f[m] and its gradients occupy the same
 * columns of g_lambda and G_A.  The two products read V once for all models
 * (their columns side by side); the model terms B, C, u are formed per model.
 * 1 <= models <= 1024.  symtd_fg is this call with models = 1.  Other
 * arguments as in symtd_fg.
 *
 * An evaluation is four kernels in order on `stream` (no other stream is
 * used): the factor copy with the Gram matrices A'A, the two products, and a
 * closing kernel for G_A, g_lambda and f.  Calls that overlap on one context
 * race (they share its workspace and counters).
 */
symtd_status symtd_fg_multi(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                            const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                            const void* A, int64_t lda, const double* lambda, int64_t r, int64_t models,
                            int d, double alpha, symtd_prec prec,
                            double* f, double* g_lambda, void* G_A, int64_t ldg);

/*
 * The constant term alpha = ||X||^2 = nu' [V'V]^d nu (elementwise power),
 * which is Lemma 3.4 applied to X (Section 3.3). O(n p^2) work: the p x p
 * Gram matrix is formed tile by tile on fp64 matrix cores from the values of
 * V exactly as stored (fp32 storage is widened exactly) and never stored.
 * alpha: 1 fp64 value (device). Other arguments as in symtd_fg.
 */
symtd_status symtd_normX(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                         const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                         int d, double* alpha);

/* ------------------------------------------------------------------------
 * Solve: minimise f over (lambda, A) with L-BFGS and restarts (Section 4: an
 * L-BFGS method with memory m = 5 and limits on iterations and evaluations;
 * Section 4.2: several starts, the best final f is kept).
 *
 * Starts (Section 4.2): lambda_0 = 1 and A_0 with unit columns drawn either
 * from N(0,1) (SYMTD_INIT_GAUSS) or as V Omega with Omega ~ N(0,1)^{p x r}
 * (SYMTD_INIT_RRF, the randomized range finder of eq. (rrf)).  The normals
 * are Philox-4x32-10 / Box-Muller draws keyed by (seed, restart): element e
 * (column-major) of the start matrix of restart k is normal e mod 4 of the
 * Philox block with counter (e/4 low word, e/4 high word, k, s) and key
 * (seed low word, seed high word), with s = 1 for the Gaussian A_0 and s = 2
 * for Omega; words (x0, x1) give normals 0, 1 and (x2, x3) normals 2, 3,
 * through u = (x + 1/2) 2^-32, sqrt(-2 ln u_a) (cos, sin)(2 pi u_b).
 *
 * The method minimises phi = f / s with s = alpha when alpha is used (known
 * or computed) and s = 1 otherwise.  Each iteration takes the L-BFGS
 * direction (memory m, H0 = gamma I with gamma = s'y/y'y of the newest pair;
 * a pair is kept only if s'y > 1e-10 y'y; a non-descent direction clears the
 * memory and uses -g) and a strong-Wolfe line search (c1 = 1e-3, c2 = 0.9;
 * first trial min(1, 1/||g||_2) along -g, else 1; bracketing doubles the
 * trial; zoom uses the safeguarded cubic minimiser; at most 20 evaluations).
 * Stopping: ||grad phi||_inf <= pgtol; phi_k - phi_{k+1} <= ftol
 * max(|phi_k|, |phi_{k+1}|, 1); iterations >= max_iters; evaluations >=
 * max_evals; a failed line search; a non-finite value at the start.
 *
 * All restarts run together: every evaluation step evaluates all of them in
 * one symtd_fg_multi-style pass (V read once), and the L-BFGS state of every
 * restart lives on the device; the host only polls stop flags.  The call is
 * synchronous with respect to `stream` (it returns after the solve).
 * ------------------------------------------------------------------------ */
typedef enum symtd_init { SYMTD_INIT_GAUSS = 0, SYMTD_INIT_RRF = 1 } symtd_init;

typedef enum symtd_alpha_mode {
  SYMTD_ALPHA_COMPUTE = 0,   /* alpha = ||X||^2 by symtd_normX, then used as s */
  SYMTD_ALPHA_GIVEN = 1,     /* use opts.alpha (> 0) */
  SYMTD_ALPHA_NONE = 2       /* shifted objective (alpha = 0), s = 1 */
} symtd_alpha_mode;

typedef enum symtd_exit {
  SYMTD_EXIT_RUNNING = 0, SYMTD_EXIT_PGTOL = 1, SYMTD_EXIT_FTOL = 2, SYMTD_EXIT_MAX_ITERS = 3,
  SYMTD_EXIT_MAX_EVALS = 4, SYMTD_EXIT_LINESEARCH = 5, SYMTD_EXIT_NONFINITE = 6
} symtd_exit;

/* The data of one decomposition problem (device pointers as in symtd_fg). */
typedef struct symtd_problem {
  symtd_dtype dt;
  const void* V; int64_t ldv;
  const double* nu;
  int64_t n, p;
  int d;
  int64_t r;
} symtd_problem;

typedef struct symtd_solve_opts {
  symtd_prec prec;
  int m;                    /* L-BFGS memory, 1..8 (paper: 5) */
  double pgtol;             /* >= 0 */
  double ftol;              /* >= 0 (L-BFGS-B's default factr 1e7 times eps is 2.22e-9) */
  int64_t max_iters;        /* >= 1 */
  int64_t max_evals;        /* >= 1 */
  int restarts;             /* >= 1 */
  uint64_t seed;
  symtd_init init;
  symtd_alpha_mode alpha_mode;
  double alpha;             /* used with SYMTD_ALPHA_GIVEN */
  const void* A0;           /* optional device starts, n x (restarts r) of type dt, leading
                               dimension n (restart k = columns k r ..); NULL = draw them */
  int check_every;          /* evaluation steps between polls of the stop flags (0 = automatic) */
  double sigma;             /* > 0: minimise the objective of the moment corrected for spherical
                               Gaussian noise of this level, ||X - Delta - M||^2 (d = 3 or 4,
                               n <= 4096; see symtd_fg_corrected); alpha then stands for
                               ||X - Delta||^2 (computed, given or 0).  0 = the plain objective.
                               symtd_solve only (the batched and served forms refuse it) */
  /* Checkpoint and resume (symtd_solve only; the batched and served forms
   * refuse them).  The state of a solve between two evaluation steps is its
   * restarts' L-BFGS vectors x, g, d, S, Y, their next trial points, their
   * line-search and counter state, the stop counter and the f traces; it is
   * written to and read from caller-owned host memory as one opaque block
   * of symtd_solve_state_bytes bytes. */
  int64_t pause_after;      /* > 0: once this many evaluation steps have run (counting those of
                               the solve it resumes) while some restart is still running, write
                               the state to state_out and return SYMTD_OK with exit_reason
                               SYMTD_EXIT_RUNNING and steps = pause_after; A, lambda and the
                               other figures of the result are not written.  0 = run to the end */
  void* state_out;          /* host, symtd_solve_state_bytes bytes, written when the solve pauses;
                               NULL = pause without saving */
  const void* state_in;     /* host: a state written by a paused solve of the same problem and the
                               same options (pause_after, state_out, state_in, A0 and check_every
                               aside) and trace_len; the solve continues from it, taking its
                               starts and alpha from it, and ends with the same results as an
                               uninterrupted solve, bit for bit (steps aside: the steps that run
                               after every restart has stopped depend on check_every).  A state
                               of another problem or other options is refused with SYMTD_EINVAL
                               (V and nu themselves are not checked).  NULL = start afresh */
} symtd_solve_opts;

typedef struct symtd_solve_result {
  /* caller-owned outputs */
  void* A; int64_t lda;     /* device, n x r of type dt: factors of the best restart */
  double* lambda;           /* device, r values */
  double* f_restarts;       /* host, `restarts` final f values (working precision), or NULL */
  int64_t* iters_restarts;  /* host, `restarts` values, or NULL */
  int64_t* evals_restarts;  /* host, `restarts` values, or NULL */
  int* exit_restarts;       /* host, `restarts` symtd_exit values, or NULL */
  double* f_trace;          /* host, restarts x trace_len: f at the start and after every
                               accepted step (NaN past the end), or NULL */
  int64_t trace_len;
  /* written by the call */
  double f;                 /* f (alpha included) at the best restart's final point, evaluated
                               with fp64 products whatever the working precision; the best
                               restart is the one with the lowest final f in working precision */
  double alpha;             /* the alpha used (0 with SYMTD_ALPHA_NONE) */
  double rel_err;           /* sqrt(max(f, 0) / alpha), NaN without alpha */
  int64_t iters, evals;     /* of the best restart */
  int exit_reason;          /* of the best restart */
  int best_restart;         /* lowest final f, lowest index on ties */
  int64_t steps;            /* evaluation steps run (all restarts together) */
} symtd_solve_result;

/* Fill `opts` with defaults: fp32 products, m = 5, pgtol = 1e-4, ftol =
 * 2.22e-9, max_iters = 10000, max_evals = 50000 (Section 4), 1 restart,
 * seed 0, RRF starts, alpha computed, no noise correction, no pause and
 * no saved state. */
symtd_status symtd_solve_opts_default(symtd_solve_opts* opts);

symtd_status symtd_solve(symtd_ctx* ctx, void* stream, const symtd_problem* pb,
                         const symtd_solve_opts* opts, symtd_solve_result* out);

/* Size in bytes of the state that symtd_solve writes when it pauses, for
 * this problem, these options and a result with this trace_len (0 without
 * a trace).  Host-only: needs no device.  SYMTD_EINVAL on a null argument,
 * r < 1, restarts or m out of range, a negative trace_len or an unknown
 * storage type. */
symtd_status symtd_solve_state_bytes(const symtd_problem* pb, const symtd_solve_opts* opts, int64_t trace_len,
                                     size_t* bytes);

/* ------------------------------------------------------------------------
 * Moments corrected for spherical Gaussian noise (the lower-order terms that
 * keep X from being exactly of rank r, Section 4.2; the paper leaves their
 * removal to future work).  For v = mu + sigma g with g ~ N(0, I), Isserlis'
 * theorem gives E[v^{(x)d}] = E[mu^{(x)d}] + Delta with
 *   d = 3:  Delta = sigma^2 sym3(m (x) I)
 *   d = 4:  Delta = sigma^2 sym6(S (x) I) + sigma^4 sym3(I (x) I)
 * where m = sum_l nu_l v_l, S = sum_l nu_l v_l v_l' - sigma^2 I and symK sums
 * the K placements of the factors over the d index positions.  The corrected
 * objective ||X - Delta - M||^2 = f + 2 sum_j lambda_j Delta a_j^d + constant.
 * ------------------------------------------------------------------------ */

/* m = sum_l nu_l v_l (n fp64 values) and, when M2 is not NULL, M2 = sum_l
 * nu_l v_l v_l' (n x n fp64, column-major), device pointers, summed in fp64.
 * Asynchronous. */
symtd_status symtd_moment_stats(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                                const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                                double* m, double* M2);

/* symtd_fg, then the correction of the noise level sigma >= 0 (d = 3 or 4,
 * n <= 4096; m and, for d = 4, M2 from symtd_moment_stats):
 *   f += 2 sum_j lambda_j Delta a_j^d, g_lambda_j += 2 Delta a_j^d,
 *   column j of G_A += 2 d lambda_j Delta a_j^{d-1},
 * so that with alpha = alpha_c (symtd_alpha_corrected) f = ||X - Delta - M||^2.
 * The correction terms are formed in fp64.  Asynchronous. */
symtd_status symtd_fg_corrected(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                                const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                                const void* A, int64_t lda, const double* lambda, int64_t r, int d,
                                double alpha, symtd_prec prec, double sigma, const double* m, const double* M2,
                                double* f, double* g_lambda, void* G_A, int64_t ldg);

/* alpha_c = ||X - Delta||^2 = alpha - 2 <X, Delta> + ||Delta||^2 for alpha =
 * ||X||^2 (symtd_normX): <X, Delta> = sum_l nu_l Delta v_l^d on the device,
 * ||Delta||^2 in closed form.  *alpha_c is a HOST value; synchronous. */
symtd_status symtd_alpha_corrected(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                                   const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                                   int d, double sigma, const double* m, const double* M2, double alpha,
                                   double* alpha_c);

/* ------------------------------------------------------------------------
 * The explicit route (Algorithm 1, fg_explicit): the data tensor stored as a
 * dense n^d array, for the comparison of Section 4.1 (Table 1).  X must be
 * symmetric; entry (i_1, .., i_d) is at i_1 + n i_2 + .. + n^{d-1} i_d.
 * ------------------------------------------------------------------------ */

/* X = sum_l nu_l v_l^{(x)d} (eq. (tensorX)), every entry summed in fp64
 * over the observations and stored in the type dt.  X: n^d values (device),
 * fully overwritten; n^{d-1} < 2^31.  Asynchronous. */
symtd_status symtd_form_moment(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                               const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                               int d, void* X);

/* Algorithm 1: y_j = X a_j^{d-1} (eq. (ExpXbdd)), w_j = a_j'y_j, and f,
 * g_lambda, G_A as in symtd_fg (same closing kernel, same precisions:
 * SYMTD_PREC_FP64 for fp64 storage, SYMTD_PREC_FP32 for fp32).  The first
 * of the d - 1 contracted modes runs on the matrix cores (the first product
 * of symtd_fg, with X's mode-1 unfolding as n^{d-1} unit-weight columns),
 * the others in a second kernel.  O(r n^d) work.  n^{d-1} < 2^31.
 * Asynchronous; the context's workspace is used. */
symtd_status symtd_fg_explicit(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* X, int64_t n, int d,
                               const void* A, int64_t lda, const double* lambda, int64_t r, double alpha,
                               symtd_prec prec, double* f, double* g_lambda, void* G_A, int64_t ldg);

/* ------------------------------------------------------------------------
 * Stochastic objective and Adam (Section 5).
 *
 * For very many observations, the objective and gradient are estimated from
 * s columns of V drawn uniformly with replacement (Lemma 5.1): Algorithm 2
 * on the sampled columns with weights p nu_i / s (= 1/s for nu = 1/p) gives
 * unbiased estimates of X a^{d-1}, and so of the shifted objective (alpha
 * = 0) and its gradient, which are linear in X.
 *
 * Draws: sample k of draw t under `seed` is word k mod 4 of the
 * Philox-4x32-10 block with counter (k / 4, t low word, t high word, 3) and
 * key (seed low word, seed high word), mapped to column floor(x p / 2^32).
 * ------------------------------------------------------------------------ */

/* Shifted objective and gradient (alpha = 0) on draw `draw` of s samples.
 * Arguments as in symtd_fg, plus s >= 1, seed, draw >= 0 and idx: NULL, or
 * s int64 device values that receive the sampled column indices.  Uses the
 * context's solver workspace for the gathered columns.  Asynchronous. */
symtd_status symtd_fg_sampled(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                              const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                              int64_t s, uint64_t seed, int64_t draw,
                              const void* A, int64_t lda, const double* lambda, int64_t r, int d,
                              symtd_prec prec, double* f, double* g_lambda, void* G_A, int64_t ldg,
                              int64_t* idx);

/* Adam (Kingma & Ba, 2015) on the sampled shifted objective with the
 * paper's schedule: epochs of epoch_len steps, each step on a fresh draw
 * (draw t = steps taken before it; all restarts step together on the same
 * draw); after every epoch the shifted objective is estimated on a fixed
 * set of est_samples columns (draw 0 of Philox stream 4, same map).  If the
 * estimate did not decrease, the state saved at the previous accepted epoch
 * (x, the moments and the step count) is restored and the learning rate
 * drops from lr0 to lr1; the second time the restart stops on that saved
 * state.  Starts as in symtd_solve (seed, init, A0).  max_epochs caps the
 * epochs. */
typedef struct symtd_adam_opts {
  symtd_prec prec;          /* SYMTD_PREC_FP64 or SYMTD_PREC_FP32, matching the storage */
  int64_t samples;          /* s, columns per step (paper: 10, 100, 1000) */
  int64_t est_samples;      /* columns of the fixed estimation set (paper: 1000) */
  int epoch_len;            /* steps per epoch (paper: 100) */
  int64_t max_epochs;
  double lr0, lr1;          /* learning rates (paper: 0.01, then 0.001) */
  double beta1, beta2, eps; /* Adam's constants (0.9, 0.999, 1e-8) */
  int restarts;             /* 1 .. 1024 */
  uint64_t seed;            /* starts and draws */
  symtd_init init;
  const void* A0;           /* optional starts, as in symtd_solve_opts */
} symtd_adam_opts;

/* Defaults: fp32, s = 100, 1000 estimation samples, epochs of 100, at most
 * 1000 epochs, lr 0.01 then 0.001, beta 0.9 / 0.999, eps 1e-8, 1 restart,
 * seed 0, RRF starts. */
symtd_status symtd_adam_opts_default(symtd_adam_opts* opts);

/* Result as in symtd_solve, with: f = the shifted objective (alpha = 0) of
 * the best restart's final point on the whole data set (fp64 products); the
 * best restart has the lowest shifted objective in working precision; alpha
 * = 0, rel_err = NaN; iters = gradient steps, evals = epochs;
 * exit_reason SYMTD_EXIT_FTOL (second epoch without decrease) or
 * SYMTD_EXIT_MAX_ITERS (max_epochs); f_restarts the shifted objectives;
 * f_trace the estimates (at the start, then after every epoch).
 * Synchronous. */
symtd_status symtd_solve_adam(symtd_ctx* ctx, void* stream, const symtd_problem* pb, const symtd_adam_opts* opts,
                              symtd_solve_result* out);

/* ------------------------------------------------------------------------
 * Batched forms: many independent problems of uneven shape at once.
 *
 * Every problem is one instance of the grouped kernels: each evaluation step
 * runs four launches for all instances (first product with its epilogue, fp64
 * model terms, split second product, G_A assembly), driven by tables of work
 * items (instance, tile, column group ...), so the device is filled by many
 * small products.  An instance's tiles, splits and summation orders depend
 * only on its own shape: its results are the same bits whatever else is in
 * the batch.  (These kernels differ from the single-instance ones, so the
 * batched and single forms agree to the stated tolerances, not bitwise.)
 * ------------------------------------------------------------------------ */
typedef struct symtd_fg_item {
  const void* V; int64_t ldv; const double* nu; int64_t n, p; int d;
  const void* A; int64_t lda; const double* lambda; int64_t r; int64_t models;
  double alpha;
  double* f;                /* models values */
  double* g_lambda;         /* models * r values */
  void* G_A; int64_t ldg;   /* n x (models r); rows n .. ldg-1 are not written */
} symtd_fg_item;

/* symtd_fg_multi for every item (all items share dt and prec).  Device
 * pointers as in symtd_fg; the call synchronises `stream` before returning. */
symtd_status symtd_fg_batched(symtd_ctx* ctx, void* stream, symtd_dtype dt, symtd_prec prec,
                              int64_t count, const symtd_fg_item* items);

/* symtd_solve for every problem (problem i with options opts[i], results in
 * outs[i]; all problems share dt), all advanced together on the grouped
 * engine: each problem's restarts are lanes of the device L-BFGS, one
 * evaluation step evaluates every live lane, finished problems leave the
 * step tables.  The starts are drawn as in symtd_solve.  Synchronous. */
symtd_status symtd_solve_batched(symtd_ctx* ctx, void* stream, int64_t count, const symtd_problem* pbs,
                                 const symtd_solve_opts* opts, symtd_solve_result* outs);

/* ------------------------------------------------------------------------
 * Served form: a request loop over the grouped engine (continuous batching).
 *
 * A server owns its own context on `device`, a device memory budget
 * (`memory_bytes`, the arena that admitted requests live in) and a host
 * thread that runs the engine.  symtd_server_submit copies the request's V
 * and nu (device pointers) into a private staging copy before it returns, so
 * the caller may reuse them at once, and queues it.  The server thread admits
 * queued requests in arrival order while their footprint (padded V, the
 * evaluation buffers and the L-BFGS state of their restarts) fits into the
 * free memory, runs evaluation steps for every admitted request together,
 * and moves finished requests to the completion queue; requests that arrive
 * while others run join at the next step boundary.  Each result is the same
 * bits as the same request solved alone on the grouped engine
 * (symtd_solve_batched with one problem).  All requests of a server share
 * its dtype and precision.  submit, poll, cancel and stats may be called
 * from any host thread.
 * ------------------------------------------------------------------------ */
typedef struct symtd_server symtd_server;

typedef struct symtd_server_opts {
  int device;
  symtd_dtype dt;
  symtd_prec prec;
  size_t memory_bytes;      /* device memory for admitted requests */
  int check_every;          /* evaluation steps between polls (0 = automatic) */
  int use_graph;            /* replay captured steps (1) or launch eagerly (0) */
} symtd_server_opts;

typedef struct symtd_server_result {
  uint64_t id;
  symtd_status status;      /* SYMTD_OK, or the error that ended this request */
  double f, alpha, rel_err;
  int64_t iters, evals;     /* of the best restart */
  int exit_reason, best_restart;
  int64_t n, r;
  double* A;                /* host, n x r column-major, owned by the result */
  double* lambda;           /* host, r values, owned by the result */
  double t_submit, t_admit, t_done;   /* seconds since the server started */
} symtd_server_result;

typedef struct symtd_server_stats {
  int64_t submitted, admitted, completed, cancelled, queued, running;
  int64_t steps;            /* evaluation steps run */
  size_t memory_used, memory_bytes;
} symtd_server_stats;

symtd_status symtd_server_create(const symtd_server_opts* opts, symtd_server** out);
/* Queue one request (opts->A0 must be NULL; trace outputs are not kept).
 * SYMTD_EREJECTED if its footprint exceeds the whole memory budget. */
symtd_status symtd_server_submit(symtd_server* srv, const symtd_problem* pb, const symtd_solve_opts* opts,
                                 uint64_t* id);
/* Move up to `max` finished results into `out` (in completion order); waits up
 * to timeout_ms (0 = do not wait, < 0 = wait until at least one is ready or
 * nothing is pending). */
symtd_status symtd_server_poll(symtd_server* srv, symtd_server_result* out, int32_t max, int32_t* n_out,
                               int32_t timeout_ms);
/* Cancel a request that is still queued (SYMTD_EINVAL if it is not). */
symtd_status symtd_server_cancel(symtd_server* srv, uint64_t id);
symtd_status symtd_server_stats_get(symtd_server* srv, symtd_server_stats* out);
const char* symtd_server_last_error(const symtd_server* srv);
/* Free the host arrays of a result. */
void symtd_server_result_release(symtd_server_result* res);
/* Stop the thread (running requests are abandoned) and free everything. */
void symtd_server_destroy(symtd_server* srv);

/*
 * The tuning table and the autotuners.  The table is process-wide and holds,
 * per (kind, precision, ceil(log2 n), ceil(log2 p), ceil(log2 r)) bucket, the
 * launch shape an autotuner measured fastest:
 *   SYMTD_TUNE_KIND_FG       v0 = blocks sharing the first product, v1 =
 *                            splits of the observations in the second
 *                            product, for symtd_fg and everything built on
 *                            it (r = all evaluated columns, restarts
 *                            included); SYMTD_TUNE_G1_BLOCKS / G2_SPLITS set
 *                            on a context take precedence
 *   SYMTD_TUNE_KIND_GROUPED  v0 = 16-observation blocks per split of the
 *                            grouped second product (batched solve, server),
 *                            r = an instance's columns (restarts included)
 * Evaluations read the table when they are planned: with a fixed table, an
 * instance's launch shape, summation order and result bits depend only on
 * its own sizes.  Changing the table while other threads evaluate is
 * allowed, but their shapes may then change between calls.
 */
typedef enum symtd_tune_kind { SYMTD_TUNE_KIND_FG = 0, SYMTD_TUNE_KIND_GROUPED = 1 } symtd_tune_kind;
typedef struct symtd_tune_entry {
  int kind;                 /* symtd_tune_kind */
  int prec;                 /* symtd_prec: SYMTD_PREC_FP64 or SYMTD_PREC_FP32 */
  int n_bucket, p_bucket, r_bucket;   /* ceil(log2 x) of n, p, r */
  int64_t v0, v1;           /* the launch shape (see above), >= 0 */
  double us;                /* measured time of one evaluation (informational) */
} symtd_tune_entry;
/* Insert an entry, replacing one with the same key. */
symtd_status symtd_tune_put(const symtd_tune_entry* e);
int64_t symtd_tune_count(void);
symtd_status symtd_tune_get(int64_t index, symtd_tune_entry* e);
void symtd_tune_clear(void);

/* Time symtd_fg on the given data for first-product blocks in {1/4, 1/2,
 * 3/4, 1} x compute units and second-product splits in {1/2, 1, 2, 4} x the
 * automatic count (median of three rounds of `reps` calls, after two
 * warm-up calls), put the fastest into the table and return it in *out (may
 * be NULL).  Arguments as in symtd_fg; allocates its own output buffers and
 * restores the context's split settings (symtd_set_tuning) afterwards. */
symtd_status symtd_autotune_fg(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                               const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                               const double* lambda, int64_t r, int d, symtd_prec prec, int reps,
                               symtd_tune_entry* out);

/* Time the grouped evaluation (symtd_fg_batched) of `copies` instances of
 * shape (n, p, d) with `cols` columns each (factors taken from V's first
 * columns) for second-product splits of 4, 8, 16, 32 and 64 blocks of 16
 * observations, put the fastest into the table and return it.  Allocates
 * its own buffers.  While it runs, every grouped evaluation in the process
 * (other threads and servers included) takes the candidate split being
 * timed: tune before serving, not beside it. */
symtd_status symtd_autotune_grouped(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                                    const double* nu, int64_t n, int64_t p, int d, int64_t cols, int copies,
                                    int reps, symtd_tune_entry* out);

/*
 * Work-split tuning of the evaluation kernels (tests force particular splits
 * with it; the autotuners use it). Keys:
 *   SYMTD_TUNE_G1_BLOCKS  blocks sharing the first product V'A (0 = automatic:
 *                         one per compute unit, never more than the number of
 *                         observation slabs; larger requests are clamped)
 *   SYMTD_TUNE_G2_SPLITS  splits of the observations in the second product V W
 *                         (0 = automatic: about one block per compute unit)
 *   SYMTD_TUNE_GRAPH      grouped engine (batched solve, server): 1 (default)
 *                         = capture one evaluation step as a hipGraph and
 *                         replay it; 0 = launch the step's kernels eagerly
 *   SYMTD_TUNE_SPIN_LIMIT polls after which the first product's wait for a
 *                         neighbouring block's partial gives up (0 =
 *                         automatic, 2^24); a give-up is reported as above
 *   SYMTD_TUNE_FAULT_HANDOFF  testing: 1 = the first product's waits watch
 *                         for a flag value that no block writes, so each
 *                         runs out its spin limit and gives up (every kernel
 *                         still exits); 0 (default) = off
 * Values must be >= 0; results do not depend on the split keys beyond
 * rounding order.
 */
typedef enum symtd_tune_key {
  SYMTD_TUNE_G1_BLOCKS = 0, SYMTD_TUNE_G2_SPLITS = 1, SYMTD_TUNE_GRAPH = 3,   /* 2: unused */
  SYMTD_TUNE_SPIN_LIMIT = 4, SYMTD_TUNE_FAULT_HANDOFF = 5
} symtd_tune_key;
symtd_status symtd_set_tuning(symtd_ctx* ctx, symtd_tune_key key, int64_t value);

/*
 * Per-kernel timing. Every launch of a kernel id whose bit is set in `mask`
 * (bit k = id k; 0 = off, 0xffffffff = all) is bracketed by HIP events on
 * its launch stream; symtd_profile_read synchronises those events and
 * returns, for kernel `which`, the summed duration in milliseconds and the
 * number of launches since the last reset. symtd_profile_reset returns the
 * events to a pool that later launches reuse, so that timing a warmed-up
 * loop creates no events. Kernel ids are listed by symtd_profile_name (NULL
 * past the end): gemm1, gemm2, prep (factor copy and A'A), final (G_A and the
 * scalars), normx, reduce.
 */
symtd_status symtd_profile_enable(symtd_ctx* ctx, uint32_t mask);
symtd_status symtd_profile_reset(symtd_ctx* ctx);
symtd_status symtd_profile_read(symtd_ctx* ctx, int which, double* total_ms, int64_t* launches);
const char* symtd_profile_name(int which);

#ifdef __cplusplus
}
#endif

#endif /* SYMTD_H */

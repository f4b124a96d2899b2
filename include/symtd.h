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
 *   - A context is not thread-safe: use one per host thread.
 */
#ifndef SYMTD_H
#define SYMTD_H

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
 * In every precision the column sums w_j, the split reductions, B = A'A,
 * u, f and g_lambda are accumulated in fp64. */
typedef enum symtd_prec { SYMTD_PREC_FP64 = 0, SYMTD_PREC_FP32 = 1 } symtd_prec;

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
 * The constant term alpha = ||X||^2 = nu' [V'V]^d nu (elementwise power),
 * which is Lemma 3.4 applied to X (Section 3.3). O(n p^2) work: the p x p
 * Gram matrix is formed tile by tile on fp64 matrix cores from the values of
 * V exactly as stored (fp32 storage is widened exactly) and never stored.
 * alpha: 1 fp64 value (device). Other arguments as in symtd_fg.
 */
symtd_status symtd_normX(symtd_ctx* ctx, void* stream, symtd_dtype dt,
                         const void* V, int64_t ldv, const double* nu, int64_t n, int64_t p,
                         int d, double* alpha);

/*
 * Work-split tuning of the evaluation kernels (used by the autotuner and by
 * tests that force particular splits). Keys:
 *   SYMTD_TUNE_G1_BLOCKS  blocks sharing the first product V'A (0 = automatic:
 *                         one per compute unit, never more than the number of
 *                         observation slabs; larger requests are clamped)
 *   SYMTD_TUNE_G2_SPLITS  splits of the observations in the second product V W
 *                         (0 = automatic: about one block per compute unit)
 *   SYMTD_TUNE_SERIAL     1 = run the small model-term kernels (A'A, A D C) on
 *                         the caller's stream before the products; 0 (default)
 *                         = on the context's side stream, overlapped with them
 * Values must be >= 0; results do not depend on them beyond rounding order.
 */
typedef enum symtd_tune_key {
  SYMTD_TUNE_G1_BLOCKS = 0, SYMTD_TUNE_G2_SPLITS = 1, SYMTD_TUNE_SERIAL = 2
} symtd_tune_key;
symtd_status symtd_set_tuning(symtd_ctx* ctx, symtd_tune_key key, int64_t value);

/*
 * Per-kernel timing. While enabled, every kernel the context launches is
 * bracketed by HIP events on the launch stream; symtd_profile_read
 * synchronises those events and returns, for kernel `which`, the summed
 * duration in milliseconds and the number of launches since the last
 * reset. Kernel ids are listed by symtd_profile_name (NULL past the end).
 */
symtd_status symtd_profile_enable(symtd_ctx* ctx, int enable);
symtd_status symtd_profile_reset(symtd_ctx* ctx);
symtd_status symtd_profile_read(symtd_ctx* ctx, int which, double* total_ms, int64_t* launches);
const char* symtd_profile_name(int which);

#ifdef __cplusplus
}
#endif

#endif /* SYMTD_H */

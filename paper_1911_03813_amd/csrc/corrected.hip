// Host side of the noise correction: symtd_moment_stats, symtd_fg_corrected
// and symtd_alpha_corrected (corrected.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "corrected.hpp"
#include "explicit.hpp"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace symtd;

namespace symtd {

template <typename T>
void launch_stats(hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n, int64_t p, double* m,
                  double* M2) {
  launch_moment<T>(st, MomentArgs<T>{V, ldv, nu, (int)n, p, 1, 1, nullptr, m});
  if (M2) launch_moment<T>(st, MomentArgs<T>{V, ldv, nu, (int)n, p, 2, n, nullptr, M2});
}
template void launch_stats<float>(hipStream_t, const float*, int64_t, const double*, int64_t, int64_t, double*, double*);
template void launch_stats<double>(hipStream_t, const double*, int64_t, const double*, int64_t, int64_t, double*,
                                   double*);

template <typename T>
symtd_status corrected_alpha(symtd_ctx* ctx, hipStream_t st, const Correction& c, const T* V, int64_t ldv,
                             const double* nu, int64_t n, int64_t p, double alpha, double* out, double* scratch) {
  // scratch: ceil(p / 256) block partials, then one value
  const int64_t blocks = (p + 255) / 256;
  launch_corr_xdot<T>(st, c, V, ldv, nu, (int)n, p, scratch);
  launch_reduce(st, ReduceArgs{scratch, blocks, scratch + blocks});
  std::vector<double> hm((size_t)n), hM2(c.d == 4 ? (size_t)n * n : 0);
  double xdot = 0.0;
  hipError_t e;
  if ((e = hipMemcpyAsync(&xdot, scratch + blocks, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(hm.data(), c.m, sizeof(double) * n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (c.d == 4 && (e = hipMemcpyAsync(hM2.data(), c.M2, sizeof(double) * n * n, hipMemcpyDeviceToHost, st)) !=
                       hipSuccess) ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return ctx->hip_fail(e, "corrected alpha");
  *out = alpha - 2.0 * xdot + corr_delta_norm2(hm.data(), c.d == 4 ? hM2.data() : nullptr, n, c.sigma, c.d);
  return SYMTD_OK;
}
template symtd_status corrected_alpha<float>(symtd_ctx*, hipStream_t, const Correction&, const float*, int64_t,
                                             const double*, int64_t, int64_t, double, double*, double*);
template symtd_status corrected_alpha<double>(symtd_ctx*, hipStream_t, const Correction&, const double*, int64_t,
                                              const double*, int64_t, int64_t, double, double*, double*);

}  // namespace symtd

namespace {

symtd_status check_corr(symtd_ctx* ctx, int64_t n, int d, double sigma, const double* m, const double* M2) {
  if (d != 3 && d != 4) return ctx->fail(SYMTD_EINVAL, "the noise correction is derived for d = 3 and d = 4");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return ctx->fail(SYMTD_EINVAL, "sigma must be finite and >= 0");
  if (n > CORR_NMAX) return ctx->fail(SYMTD_EINVAL, "the noise correction supports n <= %d", CORR_NMAX);
  if (!m || (d == 4 && !M2)) return ctx->fail(SYMTD_EINVAL, "null m (or M2 for d = 4)");
  if (((uintptr_t)m % 8) || ((uintptr_t)M2 % 8)) return ctx->fail(SYMTD_EALIGN, "m or M2 misaligned");
  return SYMTD_OK;
}

}  // namespace

extern "C" {

symtd_status symtd_moment_stats(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                                const double* nu, int64_t n, int64_t p, double* m, double* M2) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if ((s = ctx->check_common(dt, V, ldv, nu, n, p, 2)) != SYMTD_OK) return s;
  if (!m) return ctx->fail(SYMTD_EINVAL, "null m");
  if (((uintptr_t)m % 8) || ((uintptr_t)M2 % 8)) return ctx->fail(SYMTD_EALIGN, "m or M2 misaligned");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64) launch_stats<double>(st, (const double*)V, ldv, nu, n, p, m, M2);
  else launch_stats<float>(st, (const float*)V, ldv, nu, n, p, m, M2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SYMTD_OK : ctx->hip_fail(e, "kernel launch (statistics)");
}

symtd_status symtd_fg_corrected(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                                const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                                const double* lambda, int64_t r, int d, double alpha, symtd_prec prec, double sigma,
                                const double* m, const double* M2, double* f, double* g_lambda, void* G_A,
                                int64_t ldg) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = check_corr(ctx, n, d, sigma, m, M2);
  if (s != SYMTD_OK) return s;
  if ((s = symtd_fg(ctx, stream, dt, V, ldv, nu, n, p, A, lda, lambda, r, d, alpha, prec, f, g_lambda, G_A, ldg)) !=
      SYMTD_OK)
    return s;
  if ((s = ctx->reserve_solver(sizeof(double) * (size_t)r + 256)) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const Correction c{m, M2, sigma, d};
  if (dt == SYMTD_F64)
    launch_correction<double>(st, c, (const double*)A, lda, (int)n, (int)r, 1, lambda, f, g_lambda, (double*)G_A,
                              ldg, (double*)ctx->sws);
  else
    launch_correction<float>(st, c, (const float*)A, lda, (int)n, (int)r, 1, lambda, f, g_lambda, (float*)G_A, ldg,
                             (double*)ctx->sws);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SYMTD_OK : ctx->hip_fail(e, "kernel launch (correction)");
}

symtd_status symtd_alpha_corrected(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                                   const double* nu, int64_t n, int64_t p, int d, double sigma, const double* m,
                                   const double* M2, double alpha, double* alpha_c) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if ((s = ctx->check_common(dt, V, ldv, nu, n, p, d)) != SYMTD_OK) return s;
  if ((s = check_corr(ctx, n, d, sigma, m, M2)) != SYMTD_OK) return s;
  if (!alpha_c) return ctx->fail(SYMTD_EINVAL, "null alpha_c");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  if ((s = ctx->reserve_solver(sizeof(double) * (size_t)((p + 255) / 256 + 1) + 256)) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const Correction c{m, M2, sigma, d};
  if (dt == SYMTD_F64)
    return corrected_alpha<double>(ctx, st, c, (const double*)V, ldv, nu, n, p, alpha, alpha_c, (double*)ctx->sws);
  return corrected_alpha<float>(ctx, st, c, (const float*)V, ldv, nu, n, p, alpha, alpha_c, (double*)ctx->sws);
}

}  // extern "C"

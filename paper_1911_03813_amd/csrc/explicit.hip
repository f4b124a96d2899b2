// Host side of the explicit route: symtd_form_moment and symtd_fg_explicit
// (Algorithm 1, fg_explicit), composed from the kernels of the implicit
// evaluation (explicit.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "explicit.hpp"
#include "kernels.hpp"
#include "runtime.hpp"

using namespace symtd;

namespace {

struct Cut {
  char* base;
  size_t off = 0;
  explicit Cut(void* b) : base((char*)b) {}
  template <typename X>
  X* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X* q = base ? (X*)(base + off) : nullptr;
    off += count * sizeof(X);
    return q;
  }
};

// n^k, or -1 past 2^31
int64_t ipow_checked(int64_t n, int k) {
  int64_t v = 1;
  for (int t = 0; t < k; ++t) {
    v *= n;
    if (v > 0x7fffffffLL) return -1;
  }
  return v;
}

template <typename T>
symtd_status run_fg_explicit(symtd_ctx* ctx, hipStream_t st, const T* X, int64_t n, int d, const T* A, int64_t lda,
                             const double* lambda, int64_t r, double alpha, double* f, double* g, T* G, int64_t ldg) {
  const bool f64 = sizeof(T) == 8;
  const int64_t P = ipow_checked(n, d - 1), m2 = ipow_checked(n, d - 2);
  if (P < 0) return ctx->fail(SYMTD_EINVAL, "n^(d-1) = %lld^%d exceeds 2^31", (long long)n, d - 1);
  const FgPlan Pl = plan_fg(n, P, r, f64, ctx->cu_count, ctx->tune_g1_blocks, 0);
  if (Pl.nblocks > ctx->nflags) return ctx->fail(SYMTD_EINVAL, "internal: %d blocks exceed the flag array", Pl.nblocks);
  auto plan = [&](Cut& c, T** Apad, T** Wp, double** wpart, T** part, T** Y, double** wterm, double** B, double** C,
                  double** fpart, double** ones) {
    *Apad = c.take<T>(Pl.apad);
    *Wp = c.take<T>(Pl.wp);
    *wpart = c.take<double>(Pl.wpart);
    *part = c.take<T>(Pl.part);
    *Y = c.take<T>((size_t)Pl.rp * Pl.npad);
    *wterm = c.take<double>((size_t)n * Pl.rp);
    *B = c.take<double>((size_t)r * r);
    *C = c.take<double>((size_t)r * r);
    *fpart = c.take<double>((size_t)r);
    *ones = c.take<double>((size_t)P);
  };
  T *Apad, *Wp, *part, *Y;
  double *wpart, *wterm, *B, *C, *fpart, *ones;
  Cut probe(nullptr);
  plan(probe, &Apad, &Wp, &wpart, &part, &Y, &wterm, &B, &C, &fpart, &ones);
  symtd_status s = ctx->reserve(probe.off + 256);
  if (s != SYMTD_OK) return s;
  Cut cv(ctx->ws);
  plan(cv, &Apad, &Wp, &wpart, &part, &Y, &wterm, &B, &C, &fpart, &ones);
  const int rt = (int)((r + 15) / 16);

  // the factor copy for the first product, B = A'A and C = B^{d-1}
  {
    PackAArgs<T> pa{A, lda, (int)n, (int)r, Apad, Pl.ldap};
    GramArgs<T> ga{A, lda, (int)n, (int)r, 1, rt, d, B, C};
    const int npack_x = (int)((Pl.ldap + GRAM_THREADS - 1) / GRAM_THREADS);
    const int64_t npack = (int64_t)npack_x * Pl.rp;
    ctx->prof_begin(2, st);
    launch_prep(npack + (int64_t)rt * rt, st, PrepArgs<T>{pa, npack_x, npack, ga});
    ctx->prof_end(2, st);
  }
  launch_fill(st, ones, P, 1.0);
  // Z = X_(1)' A: the first product with unit weights and order 2 stores z itself
  const bool vec = ((uintptr_t)X % 16) == 0 && (n % (int64_t)(16 / sizeof(T))) == 0;
  const bool dma = vec && (n % 4) == 0;
  for (int t0 = 0; t0 < Pl.nt_tot; t0 += Pl.nt1) {
    const int nt = std::min(Pl.nt1, Pl.nt_tot - t0);
    G1Args<T> a1{X, n, ones, (int)n, (int)P, A, lda, (int)r, 16 * t0, Pl.nt_tot, Pl.rp, Pl.nblk,
                 Pl.nslab, Pl.nblocks, 2, Apad, Pl.ldap, Wp, wpart, part, ctx->handoff()};
    ctx->prof_begin(0, st);
    launch_gemm1(nt, dma, dim3(Pl.nblocks), st, a1);
    ctx->prof_end(0, st);
  }
  // the remaining d - 2 modes, and the terms of w
  ctx->prof_begin(1, st);
  launch_ttsv_tail<T>(st, TtsvTailArgs<T>{Wp, Pl.nt_tot, A, lda, (int)n, (int)r, d, m2, Y, Pl.npad, wterm, Pl.rp});
  ctx->prof_end(1, st);
  // G_A, w, u, g_lambda, f
  ctx->prof_begin(3, st);
  {
    const int ct = (int)((r + FINAL_COLS - 1) / FINAL_COLS);
    const int64_t ntile = ((n + 63) / 64) * ct;
    FinalArgs<T> fa{Y, Pl.npad, Pl.rp, 1, 1.0, A, lda, (int)n, (int)r, 1, ct, lambda, B, C, d,
                    wterm, n, alpha, G, ldg, fpart, f, g, ctx->final_count, ntile};
    launch_final(st, fa);
  }
  ctx->prof_end(3, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (explicit)");
  return SYMTD_OK;
}

}  // namespace

extern "C" {

symtd_status symtd_form_moment(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                               const double* nu, int64_t n, int64_t p, int d, void* X) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if ((s = ctx->check_common(dt, V, ldv, nu, n, p, d)) != SYMTD_OK) return s;
  if (!X) return ctx->fail(SYMTD_EINVAL, "null X");
  const size_t esz = dt == SYMTD_F64 ? 8 : 4;
  if ((uintptr_t)X % esz) return ctx->fail(SYMTD_EALIGN, "X misaligned");
  const int64_t cols = ipow_checked(n, d - 1);
  if (cols < 0 || (double)n * (double)cols > 9.0e15)
    return ctx->fail(SYMTD_EINVAL, "n^d = %lld^%d is too large for a dense tensor", (long long)n, d);
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64)
    launch_moment<double>(st, MomentArgs<double>{(const double*)V, ldv, nu, (int)n, p, d, cols, (double*)X, nullptr});
  else
    launch_moment<float>(st, MomentArgs<float>{(const float*)V, ldv, nu, (int)n, p, d, cols, (float*)X, nullptr});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (moment)");
  return SYMTD_OK;
}

symtd_status symtd_fg_explicit(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* X, int64_t n, int d,
                               const void* A, int64_t lda, const double* lambda, int64_t r, double alpha,
                               symtd_prec prec, double* f, double* g_lambda, void* G_A, int64_t ldg) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if (dt != SYMTD_F64 && dt != SYMTD_F32) return ctx->fail(SYMTD_EINVAL, "unknown dtype %d", (int)dt);
  if (n < 1 || n > 0x7fffffffLL || r < 1 || r > 0x7fffffffLL)
    return ctx->fail(SYMTD_EINVAL, "sizes must be >= 1 (n=%lld, r=%lld)", (long long)n, (long long)r);
  if (d < 2 || d > 16) return ctx->fail(SYMTD_EINVAL, "order d=%d outside [2, 16]", d);
  if (lda < n || ldg < n) return ctx->fail(SYMTD_EINVAL, "lda and ldg must be >= n");
  if (!X || !A || !lambda || !f || !g_lambda || !G_A) return ctx->fail(SYMTD_EINVAL, "null pointer argument");
  if (!((dt == SYMTD_F64 && prec == SYMTD_PREC_FP64) || (dt == SYMTD_F32 && prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)dt, (int)prec);
  const size_t esz = dt == SYMTD_F64 ? 8 : 4;
  if (((uintptr_t)X % esz) || ((uintptr_t)A % esz) || ((uintptr_t)G_A % esz) || ((uintptr_t)lambda % 8) ||
      ((uintptr_t)f % 8) || ((uintptr_t)g_lambda % 8))
    return ctx->fail(SYMTD_EALIGN, "misaligned pointer");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64)
    return run_fg_explicit<double>(ctx, st, (const double*)X, n, d, (const double*)A, lda, lambda, r, alpha, f,
                                   g_lambda, (double*)G_A, ldg);
  return run_fg_explicit<float>(ctx, st, (const float*)X, n, d, (const float*)A, lda, lambda, r, alpha, f, g_lambda,
                                (float*)G_A, ldg);
}

}  // extern "C"

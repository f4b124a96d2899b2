// Data handles (prepared copies of V) and the evaluation on them, including
// the fp16 and bf16x3 product paths (lp.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.hpp"
#include "kernels.hpp"
#include "lp.hpp"
#include "runtime.hpp"

using namespace symtd;

struct symtd_data {
  int device = 0;
  symtd_dtype dt = SYMTD_F32;
  symtd_prec prec = SYMTD_PREC_FP32;
  int kind = -1;                 // LP_F16 / LP_BF16X3, or -1 for the fp32 / fp64 products
  const void* V = nullptr;       // the caller's V (fp32 / fp64 products read it directly)
  int64_t ldv = 0;
  const double* nu = nullptr;
  int64_t n = 0, p = 0;
  void* Vc = nullptr;            // 16-bit copy (see lp.hpp)
  int64_t ldc = 0, kc_len = 0, kr_len = 0, plane_c = 0;
  double wscale = 1.0;
};

namespace {

symtd_status run_fg_lp(symtd_ctx* ctx, hipStream_t st, const symtd_data* D, const float* A, int64_t lda,
                       const double* lambda, int64_t r, int d, double alpha, double* f, double* g_lambda, float* G,
                       int64_t ldg) {
  const int kind = D->kind;
  const int PL = kind == LP_F16 ? 1 : 2;
  const int64_t n = D->n, p = D->p;
  const int nt_tot = (int)((r + 15) / 16);
  const int rp = 16 * nt_tot;
  const int nslab1 = (int)(D->kr_len / LP_SLAB);
  const int nblocks1 = std::min(ctx->cu_count, nslab1);
  const int nslab2 = (int)((n + LP_SLAB - 1) / LP_SLAB);
  const int64_t npad = (int64_t)nslab2 * LP_SLAB;
  const int64_t KC2 = D->kr_len / lp_chunk(kind);
  int nsplit = std::max(1, (ctx->cu_count + nslab2 - 1) / nslab2);
  const int cps = (int)((KC2 + nsplit - 1) / nsplit);
  nsplit = (int)((KC2 + cps - 1) / cps);
  if (nblocks1 > ctx->nflags) return ctx->fail(SYMTD_EINVAL, "internal: %d blocks exceed the flag array", nblocks1);

  auto plan = [&](Carver& c, void** Ac, void** W, double** wpart, float** part, float** Ypart, double** B,
                  double** C, double** fpart) {
    *Ac = c.take<uint16_t>((size_t)PL * D->ldc * rp);
    *W = c.take<uint16_t>((size_t)PL * D->kr_len * rp);
    *wpart = c.take<double>((size_t)LP_WAVES * nblocks1 * rp);
    *part = c.take<float>((size_t)nblocks1 * LP_WAVES * LP_MT * LP_NT_MAX * 256);
    *Ypart = c.take<float>((size_t)nsplit * rp * npad);
    *B = c.take<double>((size_t)r * r);
    *C = c.take<double>((size_t)r * r);
    *fpart = c.take<double>((size_t)r);
  };
  void *Ac, *W;
  double *wpart, *B, *C, *fpart;
  float *part, *Ypart;
  Carver sz(nullptr);
  plan(sz, &Ac, &W, &wpart, &part, &Ypart, &B, &C, &fpart);
  symtd_status s = ctx->reserve(sz.off + 256);
  if (s != SYMTD_OK) return s;
  Carver cv(ctx->ws);
  plan(cv, &Ac, &W, &wpart, &part, &Ypart, &B, &C, &fpart);
  const int64_t aplane = D->ldc * rp, wplane = D->kr_len * rp;
  const int rt = (int)((r + 15) / 16);
  // four launches on the caller's stream: prep, gemm1, gemm2, final

  // prep: the 16-bit copy of A, and B = A'A, C = B^{d-1} from the fp32 A
  {
    LpPackArgs pa{A, lda, (int)n, (int)r, Ac, D->ldc, D->kc_len, rp, aplane};
    GramArgs<float> ga{A, lda, (int)n, (int)r, 1, rt, d, B, C};
    ctx->prof_begin(2, st);
    launch_lp_prep(kind, (int64_t)rt * rt, st, pa, ga);
    ctx->prof_end(2, st);
  }
  for (int t0 = 0; t0 < nt_tot; t0 += LP_NT_MAX) {
    const int nt = std::min(LP_NT_MAX, nt_tot - t0);
    LpG1Args a1{D->Vc, D->ldc, D->kc_len, D->plane_c, D->nu, (int)n, (int)p, Ac, aplane, 16 * t0, rp, nslab1,
                nblocks1, d, D->wscale, W, D->kr_len, wplane, wpart, part, ctx->handoff()};
    ctx->prof_begin(0, st);
    launch_lp_gemm1(kind, nt, dim3(nblocks1), st, a1);
    ctx->prof_end(0, st);
  }
  for (int t0 = 0; t0 < nt_tot; t0 += LP_NT_MAX) {
    const int nt = std::min(LP_NT_MAX, nt_tot - t0);
    LpG2Args a2{D->Vc, D->ldc, D->kr_len, D->plane_c, W, wplane, (int)n, 16 * t0, rp, nslab2, nsplit, cps, Ypart, npad};
    ctx->prof_begin(1, st);
    launch_lp_gemm2(kind, nt, dim3((unsigned)(nslab2 * 8 * ((nsplit + 7) / 8))), st, a2);
    ctx->prof_end(1, st);
  }
  // G_A (Y unscaled by 1 / wscale), w, u, g_lambda, f
  ctx->prof_begin(3, st);
  {
    const int ct = (int)((r + FINAL_COLS - 1) / FINAL_COLS);
    const int64_t ntile = ((n + 63) / 64) * ct;
    FinalArgs<float> fa{Ypart, npad, rp, nsplit, 1.0 / D->wscale, A, lda, (int)n, (int)r, 1, ct, lambda, B, C, d,
                        wpart, (int64_t)LP_WAVES * nblocks1, alpha, G, ldg, fpart, f, g_lambda, ctx->final_count,
                        ntile};
    launch_final(st, fa);
  }
  ctx->prof_end(3, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (16-bit products)");
  return SYMTD_OK;
}

}  // namespace

extern "C" {

symtd_status symtd_data_create(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                               const double* nu, int64_t n, int64_t p, symtd_prec prec, symtd_data** out) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  if (!out) return ctx->fail(SYMTD_EINVAL, "null output handle");
  *out = nullptr;
  symtd_status s = ctx->check_common(dt, V, ldv, nu, n, p, 3);
  if (s != SYMTD_OK) return s;
  const bool lp = prec == SYMTD_PREC_FP16 || prec == SYMTD_PREC_BF16X3;
  if (!((dt == SYMTD_F64 && prec == SYMTD_PREC_FP64) || (dt == SYMTD_F32 && (prec == SYMTD_PREC_FP32 || lp))))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)dt, (int)prec);
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  symtd_data* D = new (std::nothrow) symtd_data();
  if (!D) return ctx->fail(SYMTD_ENOMEM, "host allocation");
  D->device = ctx->device;
  D->dt = dt; D->prec = prec; D->V = V; D->ldv = ldv; D->nu = nu; D->n = n; D->p = p;
  if (lp) {
    hipStream_t st = (hipStream_t)stream;
    D->kind = prec == SYMTD_PREC_FP16 ? LP_F16 : LP_BF16X3;
    const int PL = D->kind == LP_F16 ? 1 : 2;
    D->kc_len = LP_PAD * ((n + LP_PAD - 1) / LP_PAD);
    D->kr_len = LP_PAD * ((p + LP_PAD - 1) / LP_PAD);
    D->ldc = D->kc_len + LP_SKEW;
    D->plane_c = D->ldc * D->kr_len;
    hipError_t e;
    if ((e = hipMalloc(&D->Vc, sizeof(uint16_t) * PL * D->plane_c)) != hipSuccess) {
      (void)hipGetLastError();
      symtd_data_destroy(D);
      return ctx->fail(SYMTD_ENOMEM, "device copy of V (%lld x %lld, 16-bit)", (long long)n, (long long)p);
    }
    LpConvArgs ca{(const float*)V, ldv, (int)n, (int)p, D->Vc, D->ldc, D->kc_len, D->kr_len, D->plane_c};
    launch_lp_convert(D->kind, st, ca);
    // W is stored times 2^s with 2^s max(nu) in [1, 2) so that fp16 keeps it normal
    double* dmax = nullptr;
    double hmax = 0.0;
    if ((e = hipMalloc(&dmax, sizeof(double))) != hipSuccess) {
      symtd_data_destroy(D);
      return ctx->hip_fail(e, "hipMalloc");
    }
    launch_max_abs(st, nu, p, dmax);
    e = hipMemcpyAsync(&hmax, dmax, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dmax);
    if (e != hipSuccess) {
      symtd_data_destroy(D);
      return ctx->hip_fail(e, "preparing the 16-bit copies");
    }
    if (!(hmax > 0.0 && std::isfinite(hmax))) {
      symtd_data_destroy(D);
      return ctx->fail(SYMTD_ENONFINITE, "max |nu| = %g", hmax);
    }
    D->wscale = D->kind == LP_F16 ? std::ldexp(1.0, -(int)std::floor(std::log2(hmax))) : 1.0;
  }
  *out = D;
  return SYMTD_OK;
}

void symtd_data_destroy(symtd_data* D) {
  if (!D) return;
  (void)hipSetDevice(D->device);
  if (D->Vc) (void)hipFree(D->Vc);
  delete D;
}

symtd_status symtd_fg_data(symtd_ctx* ctx, void* stream, const symtd_data* D, const void* A, int64_t lda,
                           const double* lambda, int64_t r, int d, double alpha, double* f, double* g_lambda,
                           void* G_A, int64_t ldg) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  if (!D) return ctx->fail(SYMTD_EINVAL, "null data handle");
  if (symtd_status s0 = ctx->take_device_error(); s0 != SYMTD_OK) return s0;
  if (D->kind < 0) {
    return symtd_fg(ctx, stream, D->dt, D->V, D->ldv, D->nu, D->n, D->p, A, lda, lambda, r, d, alpha, D->prec, f,
                    g_lambda, G_A, ldg);
  }
  if (d < 2 || d > 16) return ctx->fail(SYMTD_EINVAL, "order d=%d outside [2, 16]", d);
  if (r < 1 || r > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "rank r=%lld must be >= 1", (long long)r);
  if (lda < D->n || ldg < D->n) return ctx->fail(SYMTD_EINVAL, "lda and ldg must be >= n");
  if (!A || !lambda || !f || !g_lambda || !G_A) return ctx->fail(SYMTD_EINVAL, "null A, lambda, f, g_lambda or G_A");
  if (((uintptr_t)A % 4) || ((uintptr_t)G_A % 4) || ((uintptr_t)lambda % 8) || ((uintptr_t)f % 8) ||
      ((uintptr_t)g_lambda % 8))
    return ctx->fail(SYMTD_EALIGN, "misaligned pointer");
  symtd_status s = ctx->set_device();
  if (s != SYMTD_OK) return s;
  return run_fg_lp(ctx, (hipStream_t)stream, D, (const float*)A, lda, lambda, r, d, alpha, f, g_lambda, (float*)G_A,
                   ldg);
}

}  // extern "C"

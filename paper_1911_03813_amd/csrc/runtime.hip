// Host runtime behind the C ABI of include/symtd.h: the context, its device
// workspace, argument checks, launch planning and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

using namespace symtd;

static const char* kProfileNames[] = {"gemm1", "gemm2", "gram", "final_G", "final_s", "normx", "reduce"};
static constexpr int kNumProfile = sizeof(kProfileNames) / sizeof(kProfileNames[0]);

symtd_status symtd_ctx::fail(symtd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  err = buf;
  return s;
}

symtd_status symtd_ctx::hip_fail(hipError_t e, const char* what) {
  return fail(SYMTD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

symtd_status symtd_ctx::reserve(size_t bytes) {
  if (bytes <= ws_bytes) return SYMTD_OK;
  // Growing replaces the buffer; wait for work that may still use it.
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  if (ws) hipFree(ws);
  ws = nullptr;
  ws_bytes = 0;
  const size_t want = std::max(bytes, (size_t)1 << 20);
  e = hipMalloc(&ws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SYMTD_ENOMEM, "hipMalloc(%zu bytes) for the workspace failed: %s", want, hipGetErrorString(e));
  }
  ws_bytes = want;
  return SYMTD_OK;
}

void symtd_ctx::prof_begin(int which, hipStream_t st) {
  if (!prof) return;
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  hipEventRecord(a, st);
  pending.push_back({which, a, b, st});
}

void symtd_ctx::prof_end(hipStream_t st) {
  if (!prof || pending.empty()) return;
  hipEventRecord(pending.back().stop, st);
  (void)st;
}

symtd_status symtd_ctx::set_device() {
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return SYMTD_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
namespace {

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename X>
  X* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X* p = (X*)(base + off);
    off += count * sizeof(X);
    return p;
  }
};

template <typename X>
bool aligned_to(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

struct FgPlan {
  int nt_tot, rp, nblk, mt, grid1, nsplit, blk_per_split;
  int64_t npad;
  size_t bytes(size_t esz, int r) const {
    // Carve order: Wp, wpart, Ypart, B, C (each 256-byte aligned)
    size_t s = 0;
    auto add = [&](size_t b) { s = ((s + 255) & ~(size_t)255) + b; };
    add((size_t)nblk * 16 * rp * esz);
    add((size_t)grid1 * rp * sizeof(double));
    add((size_t)nsplit * rp * npad * esz);
    add((size_t)r * r * sizeof(double));
    add((size_t)r * r * sizeof(double));
    return s + 256;
  }
};

FgPlan plan_fg(int64_t n, int64_t p, int64_t r, bool f64, int cus) {
  FgPlan P;
  P.nt_tot = (int)((r + 15) / 16);
  P.rp = 16 * P.nt_tot;
  P.nblk = (int)((p + 15) / 16);
  P.mt = f64 ? G1_MT_F64 : G1_MT_F32;
  P.grid1 = (int)((p + 64 * P.mt - 1) / (64 * P.mt));
  P.npad = ((n + 255) / 256) * 256;
  const int rowblocks = (int)(P.npad / 256);
  const int target = 2 * cus;
  int nsplit = std::max(1, (target + rowblocks - 1) / rowblocks);
  nsplit = std::min(nsplit, P.nblk);
  P.blk_per_split = (P.nblk + nsplit - 1) / nsplit;
  P.nsplit = (P.nblk + P.blk_per_split - 1) / P.blk_per_split;
  return P;
}

template <typename T>
symtd_status run_fg(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu,
                    int64_t n, int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r,
                    int d, double alpha, double* f, double* g_lambda, T* G, int64_t ldg) {
  const bool f64 = sizeof(T) == 8;
  const FgPlan P = plan_fg(n, p, r, f64, ctx->cu_count);
  symtd_status s = ctx->reserve(P.bytes(sizeof(T), (int)r));
  if (s != SYMTD_OK) return s;
  Carve cv(ctx->ws);
  T* Wp = cv.take<T>((size_t)P.nblk * 16 * P.rp);
  double* wpart = cv.take<double>((size_t)P.grid1 * P.rp);
  T* Ypart = cv.take<T>((size_t)P.nsplit * P.rp * P.npad);
  double* B = cv.take<double>((size_t)r * r);
  double* C = cv.take<double>((size_t)r * r);

  const int ntmax = f64 ? NT_MAX_F64 : NT_MAX_F32;
  const size_t vq = 16 / sizeof(T);
  const bool vecV = aligned_to<T>(V, 16) && (ldv % vq) == 0;
  const bool vecA = aligned_to<T>(A, 16) && (lda % vq) == 0;

  // B = A'A, C = B^{d-1}
  {
    GramArgs<T> ga{A, lda, (int)n, (int)r, d, B, C};
    const dim3 grid((unsigned)((r + 15) / 16), (unsigned)((r + 15) / 16));
    ctx->prof_begin(2, st);
    launch_gram(grid, st, ga);
    ctx->prof_end(st);
  }
  // Z = V'A and its epilogue, one launch per group of up to NT_MAX column subtiles
  for (int t0 = 0; t0 < P.nt_tot; t0 += ntmax) {
    const int nt = std::min(ntmax, P.nt_tot - t0);
    G1Args<T> a1{V, ldv, nu, (int)n, (int)p, A, lda, (int)r, 16 * t0, P.nt_tot, d, Wp, wpart};
    ctx->prof_begin(0, st);
    launch_gemm1(nt, vecV && vecA, dim3(P.grid1), st, a1);
    ctx->prof_end(st);
  }
  // Y = V W, split over the observations
  for (int t0 = 0; t0 < P.nt_tot; t0 += ntmax) {
    const int nt = std::min(ntmax, P.nt_tot - t0);
    G2Args<T> a2{V, ldv, (int)n, (int)p, Wp, P.nt_tot, 16 * t0, P.nblk, P.blk_per_split, Ypart, P.npad};
    const dim3 grid((unsigned)(P.npad / 256), (unsigned)P.nsplit);
    ctx->prof_begin(1, st);
    launch_gemm2(nt, vecV, grid, st, a2);
    ctx->prof_end(st);
  }
  {
    FinalGArgs<T> ag{Ypart, P.npad, P.rp, P.nsplit, A, lda, (int)n, (int)r, d, lambda, C, G, ldg};
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)r);
    ctx->prof_begin(3, st);
    launch_final_G(grid, st, ag);
    ctx->prof_end(st);
  }
  {
    FinalSArgs as{wpart, P.grid1, P.rp, B, C, lambda, (int)r, alpha, f, g_lambda};
    ctx->prof_begin(4, st);
    launch_final_s(st, as);
    ctx->prof_end(st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (fg)");
  return SYMTD_OK;
}

template <typename S>
symtd_status run_normx(symtd_ctx* ctx, hipStream_t st, const S* V, int64_t ldv, const double* nu,
                       int64_t n, int64_t p, int d, double* alpha) {
  const int64_t T = (p + 127) / 128;
  const int64_t pairs = T * (T + 1) / 2;
  if (pairs > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "normX: p = %lld gives too many tile pairs", (long long)p);
  symtd_status s = ctx->reserve((size_t)pairs * sizeof(double) + 256);
  if (s != SYMTD_OK) return s;
  double* part = (double*)ctx->ws;
  const size_t vq = 16 / sizeof(S);
  const bool vec = aligned_to<S>(V, 16) && (ldv % vq) == 0;
  NormXArgs<S> a{V, ldv, nu, (int)n, (int)p, d, T, part};
  ctx->prof_begin(5, st);
  launch_normx(vec, dim3((unsigned)pairs), st, a);
  ctx->prof_end(st);
  ReduceArgs ra{part, pairs, alpha};
  ctx->prof_begin(6, st);
  launch_reduce(st, ra);
  ctx->prof_end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (normX)");
  return SYMTD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// argument checks shared by the entry points
// ---------------------------------------------------------------------------
symtd_status symtd_ctx::check_common(symtd_dtype dt, const void* V, int64_t ldv, const double* nu,
                                     int64_t n, int64_t p, int d) {
  if (dt != SYMTD_F64 && dt != SYMTD_F32) return fail(SYMTD_EINVAL, "unknown dtype %d", (int)dt);
  if (n < 1 || p < 1) return fail(SYMTD_EINVAL, "sizes must be >= 1 (n=%lld, p=%lld)", (long long)n, (long long)p);
  if (n > 0x7fffffffLL || p > 0x7fffffffLL) return fail(SYMTD_EINVAL, "n and p must be < 2^31");
  if (d < 2 || d > 16) return fail(SYMTD_EINVAL, "order d=%d outside [2, 16]", d);
  if (ldv < n) return fail(SYMTD_EINVAL, "ldv=%lld < n=%lld", (long long)ldv, (long long)n);
  if (!V || !nu) return fail(SYMTD_EINVAL, "null V or nu");
  const size_t esz = dt == SYMTD_F64 ? 8 : 4;
  if (!aligned_to<char>(V, esz)) return fail(SYMTD_EALIGN, "V is not aligned to %zu bytes", esz);
  if (!aligned_to<char>(nu, 8)) return fail(SYMTD_EALIGN, "nu is not aligned to 8 bytes");
  return SYMTD_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* symtd_status_string(symtd_status s) {
  switch (s) {
    case SYMTD_OK: return "SYMTD_OK";
    case SYMTD_EINVAL: return "SYMTD_EINVAL";
    case SYMTD_EALIGN: return "SYMTD_EALIGN";
    case SYMTD_ENOMEM: return "SYMTD_ENOMEM";
    case SYMTD_EDEVICE: return "SYMTD_EDEVICE";
    case SYMTD_EUNSUPPORTED: return "SYMTD_EUNSUPPORTED";
    case SYMTD_ENONFINITE: return "SYMTD_ENONFINITE";
    case SYMTD_EREJECTED: return "SYMTD_EREJECTED";
  }
  return "unknown status";
}

symtd_status symtd_create(int device, symtd_ctx** out) {
  if (!out) return SYMTD_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return SYMTD_EDEVICE;
  }
  if (device < 0 || device >= count) return SYMTD_EINVAL;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return SYMTD_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SYMTD_EUNSUPPORTED;
  symtd_ctx* c = new (std::nothrow) symtd_ctx();
  if (!c) return SYMTD_ENOMEM;
  c->device = device;
  c->cu_count = prop.multiProcessorCount;
  *out = c;
  return SYMTD_OK;
}

void symtd_destroy(symtd_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto& pe : ctx->pending) { hipEventDestroy(pe.start); hipEventDestroy(pe.stop); }
  if (ctx->ws) hipFree(ctx->ws);
  delete ctx;
}

const char* symtd_last_error(const symtd_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

symtd_status symtd_fg(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                      const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                      const double* lambda, int64_t r, int d, double alpha, symtd_prec prec,
                      double* f, double* g_lambda, void* G_A, int64_t ldg) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->check_common(dt, V, ldv, nu, n, p, d);
  if (s != SYMTD_OK) return s;
  if (r < 1 || r > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "rank r=%lld must be >= 1", (long long)r);
  if (lda < n || ldg < n) return ctx->fail(SYMTD_EINVAL, "lda=%lld and ldg=%lld must be >= n=%lld",
                                           (long long)lda, (long long)ldg, (long long)n);
  if (!A || !lambda || !f || !g_lambda || !G_A) return ctx->fail(SYMTD_EINVAL, "null A, lambda, f, g_lambda or G_A");
  if (!((dt == SYMTD_F64 && prec == SYMTD_PREC_FP64) || (dt == SYMTD_F32 && prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)dt, (int)prec);
  const size_t esz = dt == SYMTD_F64 ? 8 : 4;
  if (!aligned_to<char>(A, esz) || !aligned_to<char>(G_A, esz)) return ctx->fail(SYMTD_EALIGN, "A or G_A misaligned");
  if (!aligned_to<char>(lambda, 8) || !aligned_to<char>(f, 8) || !aligned_to<char>(g_lambda, 8))
    return ctx->fail(SYMTD_EALIGN, "lambda, f or g_lambda misaligned");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64)
    return run_fg<double>(ctx, st, (const double*)V, ldv, nu, n, p, (const double*)A, lda, lambda, r, d, alpha, f,
                          g_lambda, (double*)G_A, ldg);
  return run_fg<float>(ctx, st, (const float*)V, ldv, nu, n, p, (const float*)A, lda, lambda, r, d, alpha, f,
                       g_lambda, (float*)G_A, ldg);
}

symtd_status symtd_normX(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                         const double* nu, int64_t n, int64_t p, int d, double* alpha) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->check_common(dt, V, ldv, nu, n, p, d);
  if (s != SYMTD_OK) return s;
  if (!alpha) return ctx->fail(SYMTD_EINVAL, "null alpha");
  if (!aligned_to<char>(alpha, 8)) return ctx->fail(SYMTD_EALIGN, "alpha misaligned");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64) return run_normx<double>(ctx, st, (const double*)V, ldv, nu, n, p, d, alpha);
  return run_normx<float>(ctx, st, (const float*)V, ldv, nu, n, p, d, alpha);
}

symtd_status symtd_profile_enable(symtd_ctx* ctx, int enable) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->prof = enable != 0;
  return SYMTD_OK;
}

symtd_status symtd_profile_reset(symtd_ctx* ctx) {
  if (!ctx) return SYMTD_EINVAL;
  for (auto& pe : ctx->pending) {
    hipEventSynchronize(pe.stop);
    hipEventDestroy(pe.start);
    hipEventDestroy(pe.stop);
  }
  ctx->pending.clear();
  return SYMTD_OK;
}

symtd_status symtd_profile_read(symtd_ctx* ctx, int which, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return SYMTD_EINVAL;
  if (which < 0 || which >= kNumProfile) return ctx->fail(SYMTD_EINVAL, "no kernel id %d", which);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& pe : ctx->pending) {
    if (pe.which != which) continue;
    hipError_t e = hipEventSynchronize(pe.stop);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pe.start, pe.stop);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipEventElapsedTime");
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return SYMTD_OK;
}

const char* symtd_profile_name(int which) {
  if (which < 0 || which >= kNumProfile) return nullptr;
  return kProfileNames[which];
}

}  // extern "C"

// Host runtime behind the C ABI of include/symtd.h: the context, its device
// workspace, argument checks, launch planning and per-kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "corrected.hpp"
#include "kernels.hpp"
#include "model_dev.hpp"
#include "lbfgs.hpp"
#include "runtime.hpp"

using namespace symtd;

static const char* kProfileNames[] = {"gemm1", "gemm2", "prep", "final", "normx", "reduce"};
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
  if (ws) (void)hipFree(ws);
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

symtd_status symtd_ctx::reserve_solver(size_t bytes) {
  if (bytes <= sws_bytes) return SYMTD_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  if (sws) (void)hipFree(sws);
  sws = nullptr;
  sws_bytes = 0;
  const size_t want = std::max(bytes, (size_t)1 << 20);
  e = hipMalloc(&sws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SYMTD_ENOMEM, "hipMalloc(%zu bytes) for the solver state failed: %s", want, hipGetErrorString(e));
  }
  sws_bytes = want;
  return SYMTD_OK;
}

hipEvent_t symtd_ctx::pool_event() {
  if (!ev_pool.empty()) {
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void symtd_ctx::prof_begin(int which, hipStream_t st) {
  if (!((prof_mask >> which) & 1u)) return;
  hipEvent_t a = pool_event(), b = pool_event();
  if (!a || !b) {
    if (a) ev_pool.push_back(a);
    if (b) ev_pool.push_back(b);
    return;
  }
  (void)hipEventRecord(a, st);
  pending.push_back({which, a, b});
}

void symtd_ctx::prof_end(int which, hipStream_t st) {
  if (!((prof_mask >> which) & 1u) || pending.empty() || pending.back().which != which) return;
  (void)hipEventRecord(pending.back().stop, st);
}

symtd::Handoff symtd_ctx::handoff() {
  symtd::Handoff h;
  h.flag = flags;
  h.err = err_dev;
  h.epoch = epoch_word;
  h.spin = (unsigned)(tune_spin > 0 ? std::min<int64_t>(tune_spin, 0x7fffffff) : (1 << 24)) |
           (tune_fault ? 0x80000000u : 0u);
  return h;
}

symtd_status symtd_ctx::take_device_error() {
  if (!err_host || __atomic_load_n(err_host, __ATOMIC_ACQUIRE) == 0) return SYMTD_OK;
  __atomic_store_n(err_host, 0, __ATOMIC_RELEASE);
  return fail(SYMTD_EDEVICE,
              "a split product's hand-off wait gave up in an earlier call on this context; the results of that "
              "call are invalid");
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

}  // namespace

namespace symtd {

FgPlan plan_fg(int64_t n, int64_t p, int64_t r, bool f64, int cus, int64_t g1_blocks, int64_t g2_splits) {
  FgPlan P;
  P.nt_tot = (int)((r + 15) / 16);
  P.rp = 16 * P.nt_tot;
  P.nblk = (int)((p + 15) / 16);
  P.nt1 = f64 ? NT_MAX_G1_F64 : NT_MAX_G1_F32;
  P.nt2 = f64 ? NT_MAX_G2_F64 : NT_MAX_G2_F32;
  // gemm1: one block per CU, never more blocks than slabs
  const int mt = f64 ? g1_mt<double>() : g1_mt<float>();
  P.g1w = f64 ? g1_waves<double>() : g1_waves<float>();
  P.nslab = (int)((p + 16 * mt * P.g1w - 1) / (16 * mt * P.g1w));
  P.nblocks = (int)std::min<int64_t>(g1_blocks > 0 ? std::min<int64_t>(g1_blocks, cus) : cus, P.nslab);
  // gemm2: row blocks of 256 x splits of the observations, one block per CU
  P.npad = ((n + 255) / 256) * 256;
  P.rowblocks = (int)(P.npad / 256);
  int nsplit = g2_splits > 0 ? (int)std::min<int64_t>(g2_splits, 1 << 20)
                             : std::max(1, (cus + P.rowblocks - 1) / P.rowblocks);
  nsplit = std::min(nsplit, P.nblk);
  P.blk_per_split = (P.nblk + nsplit - 1) / nsplit;
  P.nsplit = (P.nblk + P.blk_per_split - 1) / P.blk_per_split;
  const int kch = f64 ? g1_chunk<double>() : g1_chunk<float>();
  P.ldap = ((n + kch - 1) / kch) * kch;
  P.apad = (size_t)P.rp * P.ldap;
  P.wp = (size_t)P.nblk * 16 * P.rp;
  P.wpart = (size_t)P.g1w * P.nblocks * P.rp;
  P.part = (size_t)P.nblocks * P.g1w * mt * P.nt1 * 256;
  P.ypart = (size_t)P.nsplit * P.rp * P.npad;
  P.rr = (size_t)r * r;
  P.fp = (size_t)r;
  return P;
}


template <typename T>
symtd_status run_fg(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu,
                    int64_t n, int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r, int ng,
                    int d, double alpha, double* f, double* g_lambda, T* G, int64_t ldg,
                    void* fixed_ws, size_t fixed_bytes) {
  const bool f64 = sizeof(T) == 8;
  const int64_t r1 = r;            // columns of one model
  r = r1 * ng;                     // columns of all models (the products see them all)
  int64_t g1 = ctx->tune_g1_blocks, g2 = ctx->tune_g2_splits;
  if (g1 == 0 || g2 == 0) {
    int64_t t1 = 0, t2 = 0;
    if (tuned_fg(f64, n, p, r, &t1, &t2)) {
      if (g1 == 0) g1 = t1;
      if (g2 == 0) g2 = t2;
    }
  }
  FgPlan P = plan_fg(n, p, r, f64, ctx->cu_count, g1, g2);
  P.rr = (size_t)ng * r1 * r1;      // B and C: one r1 x r1 block per model
  if (P.nblocks > ctx->nflags) return ctx->fail(SYMTD_EINVAL, "internal: %d blocks exceed the flag array", P.nblocks);
  const size_t need = P.bytes(sizeof(T));
  void* base = fixed_ws;
  const uint32_t prof_mask = ctx->prof_mask;
  if (fixed_ws) {
    if (need > fixed_bytes)
      return ctx->fail(SYMTD_EINVAL, "the evaluation needs %zu bytes of workspace, more than the %zu of the fixed "
                       "scratch array", need, fixed_bytes);
    ctx->prof_mask = 0;
  } else {
    symtd_status s = ctx->reserve(need);
    if (s != SYMTD_OK) return s;
    base = ctx->ws;
  }
  Carve cv(base);
  T* Apad = cv.take<T>(P.apad);
  T* Wp = cv.take<T>(P.wp);
  double* wpart = cv.take<double>(P.wpart);
  T* part = cv.take<T>(P.part);
  T* Ypart = cv.take<T>(P.ypart);
  double* B = cv.take<double>(P.rr);
  double* C = cv.take<double>(P.rr);
  double* fpart = cv.take<double>(P.fp);

  const size_t vq = 16 / sizeof(T);
  const bool vecV = aligned_to<T>(V, 16) && (ldv % vq) == 0;
  const int rt = (int)((r1 + 15) / 16);
  if (ng > symtd_ctx::kFinalCounters)
    return ctx->fail(SYMTD_EINVAL, "%d models side by side exceed the %d supported", ng, symtd_ctx::kFinalCounters);
  // four launches on the caller's stream: prep, gemm1, gemm2, final

  // prep: zero-padded factor copy for gemm1, and B = A'A, C = B^{d-1}
  {
    PackAArgs<T> pa{A, lda, (int)n, (int)r, Apad, P.ldap};
    GramArgs<T> ga{A, lda, (int)n, (int)r1, ng, rt, d, B, C};
    const int npack_x = (int)((P.ldap + GRAM_THREADS - 1) / GRAM_THREADS);
    const int64_t npack = (int64_t)npack_x * P.rp;
    ctx->prof_begin(2, st);
    launch_prep(npack + (int64_t)rt * rt * ng, st, PrepArgs<T>{pa, npack_x, npack, ga});
    ctx->prof_end(2, st);
  }
  // Z = V'A and its epilogue, one launch per column group; the direct
  // global-to-LDS path needs 16-byte aligned columns holding whole quads
  const bool dma = vecV && (n % 4) == 0;
  for (int t0 = 0; t0 < P.nt_tot; t0 += P.nt1) {
    const int nt = std::min(P.nt1, P.nt_tot - t0);
    G1Args<T> a1{V, ldv, nu, (int)n, (int)p, A, lda, (int)r, 16 * t0, P.nt_tot, P.rp, P.nblk,
                 P.nslab, P.nblocks, d, Apad, P.ldap, Wp, wpart, part, ctx->handoff()};
    // the launch's last column subtile: at most 4 factor columns go on the narrow form
    const bool narrow = r - (16 * (int64_t)t0 + 16 * (nt - 1)) <= 4;
    ctx->prof_begin(0, st);
    launch_gemm1(nt, dma, dim3(P.nblocks), st, a1, narrow);
    ctx->prof_end(0, st);
  }
  // Y = V W, split over the observations
  for (int t0 = 0; t0 < P.nt_tot; t0 += P.nt2) {
    const int nt = std::min(P.nt2, P.nt_tot - t0);
    G2Args<T> a2{V, ldv, (int)n, (int)p, Wp, P.nt_tot, P.rp, 16 * t0, P.nblk, P.blk_per_split,
                 P.nsplit, P.rowblocks, Ypart, P.npad};
    const unsigned blocks = (unsigned)(P.rowblocks * 8 * ((P.nsplit + 7) / 8));
    const bool narrow = r - (16 * (int64_t)t0 + 16 * (nt - 1)) <= 4;
    ctx->prof_begin(1, st);
    launch_gemm2(nt, vecV && (n % 4) == 0, dim3(blocks), st, a2, narrow);
    ctx->prof_end(1, st);
  }
  // G_A, w, u, g_lambda, f
  ctx->prof_begin(3, st);
  {
    const int ct = (int)((r1 + FINAL_COLS - 1) / FINAL_COLS);
    const int64_t ntile = ((n + 63) / 64) * ct * ng;
    FinalArgs<T> fa{Ypart, P.npad, P.rp, P.nsplit, 1.0, A, lda, (int)n, (int)r1, ng, ct, lambda, B, C, d,
                    wpart, (int64_t)P.g1w * P.nblocks, alpha, G, ldg, fpart, f, g_lambda, ctx->final_count,
                    ntile};
    launch_final(st, fa);
  }
  ctx->prof_end(3, st);
  ctx->prof_mask = prof_mask;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (fg)");
  return SYMTD_OK;
}

template symtd_status run_fg<float>(symtd_ctx*, hipStream_t, const float*, int64_t, const double*, int64_t,
                                    int64_t, const float*, int64_t, const double*, int64_t, int, int, double,
                                    double*, double*, float*, int64_t, void*, size_t);
template symtd_status run_fg<double>(symtd_ctx*, hipStream_t, const double*, int64_t, const double*, int64_t,
                                     int64_t, const double*, int64_t, const double*, int64_t, int, int, double,
                                     double*, double*, double*, int64_t, void*, size_t);

template <typename T>
symtd_status run_rrf(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, int64_t n, int64_t p, int64_t r,
                     int restarts, uint64_t seed, const LbLane<T>* lanes_dev) {
  const bool f64 = sizeof(T) == 8;
  const FgPlan P = plan_fg(n, p, r * restarts, f64, ctx->cu_count, 0, ctx->tune_g2_splits);
  symtd_status s = ctx->reserve(P.bytes(sizeof(T)));
  if (s != SYMTD_OK) return s;
  Carve cv(ctx->ws);
  T* Wp = cv.take<T>(P.wp);
  T* Ypart = cv.take<T>(P.ypart);
  launch_omega_packed<T>(dim3((unsigned)((P.wp + 255) / 256)), st, Wp, p, (int)r, restarts, P.nt_tot, P.nblk, seed);
  const size_t vq = 16 / sizeof(T);
  const bool vecV = aligned_to<T>(V, 16) && (ldv % vq) == 0;
  for (int t0 = 0; t0 < P.nt_tot; t0 += P.nt2) {
    const int nt = std::min(P.nt2, P.nt_tot - t0);
    G2Args<T> a2{V, ldv, (int)n, (int)p, Wp, P.nt_tot, P.rp, 16 * t0, P.nblk, P.blk_per_split,
                 P.nsplit, P.rowblocks, Ypart, P.npad};
    const unsigned blocks = (unsigned)(P.rowblocks * 8 * ((P.nsplit + 7) / 8));
    launch_gemm2(nt, vecV && (n % 4) == 0, dim3(blocks), st, a2);
  }
  launch_rrf_finish<T>(restarts, (int)r, st, lanes_dev, Ypart, P.npad, P.rp, P.nsplit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (rrf)");
  return SYMTD_OK;
}

template symtd_status run_rrf<float>(symtd_ctx*, hipStream_t, const float*, int64_t, int64_t, int64_t, int64_t, int,
                                     uint64_t, const LbLane<float>*);
template symtd_status run_rrf<double>(symtd_ctx*, hipStream_t, const double*, int64_t, int64_t, int64_t, int64_t,
                                      int, uint64_t, const LbLane<double>*);

template <typename T>
symtd_status final_fp64_enqueue(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n,
                                int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r, int d,
                                double alpha, double* f_dev, const Correction* corr) {
  // scratch: [V64 n x p][A64 n x r][G64 n x r][g r][f 1][correction terms r]
  auto plan = [&](Carve& c, double** V64, double** A64, double** G64, double** g, double** f, double** lc) {
    *V64 = std::is_same<T, float>::value ? c.take<double>((size_t)n * p) : nullptr;
    *A64 = std::is_same<T, float>::value ? c.take<double>((size_t)n * r) : nullptr;
    *G64 = c.take<double>((size_t)n * r);
    *g = c.take<double>((size_t)r);
    *f = c.take<double>(1);
    *lc = c.take<double>((size_t)r);
  };
  double *V64, *A64, *G64, *g, *fd, *lc;
  Carve probe((void*)256);
  plan(probe, &V64, &A64, &G64, &g, &fd, &lc);
  const size_t need = probe.off + 512;
  hipError_t e;
  if (need > ctx->wide_bytes) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return ctx->hip_fail(e, "hipDeviceSynchronize");
    if (ctx->wide) (void)hipFree(ctx->wide);
    ctx->wide = nullptr;
    ctx->wide_bytes = 0;
    if ((e = hipMalloc(&ctx->wide, need)) != hipSuccess) {
      (void)hipGetLastError();
      return ctx->fail(SYMTD_ENOMEM, "hipMalloc(%zu) for the fp64 evaluation failed", need);
    }
    ctx->wide_bytes = need;
  }
  Carve c(ctx->wide);
  plan(c, &V64, &A64, &G64, &g, &fd, &lc);
  if (f_dev) fd = f_dev;
  symtd_status s;
  if constexpr (std::is_same<T, float>::value) {
    launch_widen(st, V, ldv, V64, n, n, p);
    launch_widen(st, A, lda, A64, n, n, r);
    s = run_fg<double>(ctx, st, V64, n, nu, n, p, A64, n, lambda, r, 1, d, alpha, fd, g, G64, n);
    if (s == SYMTD_OK && corr) launch_correction<double>(st, *corr, A64, n, (int)n, (int)r, 1, lambda, fd, g, G64, n, lc);
  } else {
    s = run_fg<double>(ctx, st, V, ldv, nu, n, p, A, lda, lambda, r, 1, d, alpha, fd, g, G64, n);
    if (s == SYMTD_OK && corr) launch_correction<double>(st, *corr, A, lda, (int)n, (int)r, 1, lambda, fd, g, G64, n, lc);
  }
  if (s != SYMTD_OK) return s;
  if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "final fp64 evaluation");
  if (!f_dev) ctx->wide_f = fd;
  return SYMTD_OK;
}

template <typename T>
symtd_status final_fp64(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n,
                        int64_t p, const T* A, int64_t lda, const double* lambda, int64_t r, int d, double alpha,
                        double* f_out, const Correction* corr) {
  symtd_status s = final_fp64_enqueue<T>(ctx, st, V, ldv, nu, n, p, A, lda, lambda, r, d, alpha, nullptr, corr);
  if (s != SYMTD_OK) return s;
  hipError_t e;
  if ((e = hipMemcpyAsync(&ctx->fwide_host, ctx->wide_f, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return ctx->hip_fail(e, "final fp64 evaluation");
  *f_out = ctx->fwide_host;
  return SYMTD_OK;
}

template symtd_status final_fp64_enqueue<float>(symtd_ctx*, hipStream_t, const float*, int64_t, const double*, int64_t,
                                                int64_t, const float*, int64_t, const double*, int64_t, int, double,
                                                double*, const Correction*);
template symtd_status final_fp64_enqueue<double>(symtd_ctx*, hipStream_t, const double*, int64_t, const double*,
                                                 int64_t, int64_t, const double*, int64_t, const double*, int64_t, int,
                                                 double, double*, const Correction*);

template symtd_status final_fp64<float>(symtd_ctx*, hipStream_t, const float*, int64_t, const double*, int64_t, int64_t,
                                        const float*, int64_t, const double*, int64_t, int, double, double*,
                                        const Correction*);
template symtd_status final_fp64<double>(symtd_ctx*, hipStream_t, const double*, int64_t, const double*, int64_t,
                                         int64_t, const double*, int64_t, const double*, int64_t, int, double, double*,
                                         const Correction*);

template <typename S>
symtd_status run_normx(symtd_ctx* ctx, hipStream_t st, const S* V, int64_t ldv, const double* nu,
                       int64_t n, int64_t p, int d, double* alpha) {
  const int64_t T = (p + 127) / 128;
  const int64_t pairs = T * (T + 1) / 2;
  if (pairs > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "normX: p = %lld gives too many tile pairs", (long long)p);
  symtd_status s = ctx->reserve((size_t)pairs * sizeof(double) + 256);
  if (s != SYMTD_OK) return s;
  double* part = (double*)ctx->ws;
  // vector loads of clamped quads need whole quads in every column
  const bool vec = aligned_to<S>(V, 16) && (ldv % 4) == 0;
  NormXArgs<S> a{V, ldv, nu, (int)n, (int)p, d, T, part};
  ctx->prof_begin(4, st);
  launch_normx(vec, dim3((unsigned)pairs), st, a);
  ctx->prof_end(4, st);
  ReduceArgs ra{part, pairs, alpha};
  ctx->prof_begin(5, st);
  launch_reduce(st, ra);
  ctx->prof_end(5, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->hip_fail(e, "kernel launch (normX)");
  return SYMTD_OK;
}

template <typename S>
symtd_status run_normx_grouped(symtd_ctx* ctx, hipStream_t st, const std::vector<NormXJob<S>>& jobs) {
  if (jobs.empty()) return SYMTD_OK;
  bool vec = true;
  int64_t total = 0;
  std::vector<int64_t> npairs(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    const NormXJob<S>& J = jobs[j];
    vec = vec && aligned_to<S>(J.V, 16) && (J.ldv % 4) == 0;
    const int64_t T = (J.p + 127) / 128;
    npairs[j] = T * (T + 1) / 2;
    total += npairs[j];
  }
  if (!vec || total > 0x7fffffffLL || jobs.size() > 0x7fffffffULL) {
    // one launch pair per set
    for (const NormXJob<S>& J : jobs) {
      symtd_status s = run_normx<S>(ctx, st, J.V, J.ldv, J.nu, J.n, J.p, J.d, J.alpha);
      if (s != SYMTD_OK) return s;
    }
    hipError_t e = hipStreamSynchronize(st);
    return e == hipSuccess ? SYMTD_OK : ctx->hip_fail(e, "normX sync");
  }
  // workspace: [partials][set descriptors][items]
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_part = up((size_t)total * sizeof(double));
  const size_t b_sets = up(jobs.size() * sizeof(GNormX<S>));
  const size_t b_items = up((size_t)total * sizeof(NormXItem));
  symtd_status s = ctx->reserve(b_part + b_sets + b_items);
  if (s != SYMTD_OK) return s;
  char* base = (char*)ctx->ws;
  double* part = (double*)base;
  GNormX<S>* d_sets = (GNormX<S>*)(base + b_part);
  NormXItem* d_items = (NormXItem*)(base + b_part + b_sets);
  std::vector<GNormX<S>> sets(jobs.size());
  std::vector<NormXItem> items((size_t)total);
  int64_t off = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    const NormXJob<S>& J = jobs[j];
    sets[j].a = NormXArgs<S>{J.V, J.ldv, J.nu, (int)J.n, (int)J.p, J.d, (J.p + 127) / 128, part + off};
    sets[j].pairs = npairs[j];
    sets[j].alpha = J.alpha;
    for (int64_t b = 0; b < npairs[j]; ++b) items[(size_t)(off + b)] = NormXItem{(int)j, (int)b};
    off += npairs[j];
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(d_sets, sets.data(), sets.size() * sizeof(GNormX<S>), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(NormXItem), hipMemcpyHostToDevice, st)) !=
          hipSuccess)
    return ctx->hip_fail(e, "normX tables");
  launch_normx_grouped((int)total, (int)jobs.size(), st, d_sets, d_items);
  if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "kernel launch (grouped normX)");
  // the host tables above must outlive their copies
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return ctx->hip_fail(e, "normX sync");
  return SYMTD_OK;
}

template symtd_status run_normx_grouped<float>(symtd_ctx*, hipStream_t, const std::vector<NormXJob<float>>&);
template symtd_status run_normx_grouped<double>(symtd_ctx*, hipStream_t, const std::vector<NormXJob<double>>&);

template symtd_status run_normx<float>(symtd_ctx*, hipStream_t, const float*, int64_t, const double*, int64_t,
                                       int64_t, int, double*);
template symtd_status run_normx<double>(symtd_ctx*, hipStream_t, const double*, int64_t, const double*, int64_t,
                                        int64_t, int, double*);

}  // namespace symtd

// ---------------------------------------------------------------------------
// the fixed scratch array of symtd_fg_noalloc: one copy per device, alive
// until the process ends.  In host code `scratch` only stands in for the
// symbol; its device address (per device) comes from hipGetSymbolAddress.
// ---------------------------------------------------------------------------
static constexpr size_t kNoallocBytes = SYMTD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // device address of `scratch`, per device id

// with `device` current: its address of the scratch array (looked up once)
symtd_status scratch_address(symtd_ctx* c, int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize((size_t)device + 1, nullptr);
  if (!g_scratch_addr[(size_t)device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return SYMTD_EDEVICE;
    }
    g_scratch_addr[(size_t)device] = ptr;
  }
  c->noalloc_ws = g_scratch_addr[(size_t)device];
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
  // flags and the arrival counters in one zeroed allocation; the error word
  // in pinned, device-mapped host memory
  const size_t words = 4 * (size_t)c->cu_count + symtd_ctx::kFinalCounters + 2;
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->flags, sizeof(int) * words) != hipSuccess ||
      hipMemset(c->flags, 0, sizeof(int) * words) != hipSuccess ||
      hipHostMalloc((void**)&c->err_host, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->err_dev, c->err_host, 0) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    symtd_destroy(c);
    return SYMTD_EDEVICE;
  }
  *c->err_host = 0;
  c->nflags = 4 * c->cu_count;  // >= the blocks of any split product
  c->final_count = c->flags + c->nflags;
  c->epoch_word = c->final_count + symtd_ctx::kFinalCounters;
  if (scratch_address(c, device) != SYMTD_OK) {
    symtd_destroy(c);
    return SYMTD_EDEVICE;
  }
  *out = c;
  return SYMTD_OK;
}

void symtd_destroy(symtd_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& pe : ctx->pending) { (void)hipEventDestroy(pe.start); (void)hipEventDestroy(pe.stop); }
  for (hipEvent_t ev : ctx->ev_pool) (void)hipEventDestroy(ev);
  if (ctx->flags) (void)hipFree(ctx->flags);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->sws) (void)hipFree(ctx->sws);
  if (ctx->wide) (void)hipFree(ctx->wide);
  if (ctx->host_flag) (void)hipHostFree(ctx->host_flag);
  if (ctx->err_host) (void)hipHostFree(ctx->err_host);
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
  return symtd_fg_multi(ctx, stream, dt, V, ldv, nu, n, p, A, lda, lambda, r, 1, d, alpha, prec, f, g_lambda,
                        G_A, ldg);
}

static symtd_status fg_multi_impl(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                                  const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                                  const double* lambda, int64_t r, int64_t models, int d, double alpha,
                                  symtd_prec prec, double* f, double* g_lambda, void* G_A, int64_t ldg,
                                  void* fixed_ws, size_t fixed_bytes) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if ((s = ctx->check_common(dt, V, ldv, nu, n, p, d)) != SYMTD_OK) return s;
  if (r < 1 || models < 1 || r * models > 0x7fffffffLL)
    return ctx->fail(SYMTD_EINVAL, "rank r=%lld and models=%lld must be >= 1", (long long)r, (long long)models);
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
    return run_fg<double>(ctx, st, (const double*)V, ldv, nu, n, p, (const double*)A, lda, lambda, r, (int)models, d,
                          alpha, f, g_lambda, (double*)G_A, ldg, fixed_ws, fixed_bytes);
  return run_fg<float>(ctx, st, (const float*)V, ldv, nu, n, p, (const float*)A, lda, lambda, r, (int)models, d,
                       alpha, f, g_lambda, (float*)G_A, ldg, fixed_ws, fixed_bytes);
}

symtd_status symtd_fg_multi(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                            const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                            const double* lambda, int64_t r, int64_t models, int d, double alpha, symtd_prec prec,
                            double* f, double* g_lambda, void* G_A, int64_t ldg) {
  Marker mk("symtd_fg");
  return fg_multi_impl(ctx, stream, dt, V, ldv, nu, n, p, A, lda, lambda, r, models, d, alpha, prec, f, g_lambda,
                       G_A, ldg, nullptr, 0);
}

symtd_status symtd_fg_noalloc(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                              const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                              const double* lambda, int64_t r, int d, double alpha, symtd_prec prec,
                              double* f, double* g_lambda, void* G_A, int64_t ldg) {
  if (!ctx) return SYMTD_EINVAL;
  if (!ctx->noalloc_ws) return ctx->fail(SYMTD_EDEVICE, "the fixed scratch array has no device address");
  return fg_multi_impl(ctx, stream, dt, V, ldv, nu, n, p, A, lda, lambda, r, 1, d, alpha, prec, f, g_lambda, G_A,
                       ldg, ctx->noalloc_ws, kNoallocBytes);
}

symtd_status symtd_normX(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                         const double* nu, int64_t n, int64_t p, int d, double* alpha) {
  if (!ctx) return SYMTD_EINVAL;
  Marker mk("symtd_normX");
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if ((s = ctx->check_common(dt, V, ldv, nu, n, p, d)) != SYMTD_OK) return s;
  if (!alpha) return ctx->fail(SYMTD_EINVAL, "null alpha");
  if (!aligned_to<char>(alpha, 8)) return ctx->fail(SYMTD_EALIGN, "alpha misaligned");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64) return run_normx<double>(ctx, st, (const double*)V, ldv, nu, n, p, d, alpha);
  return run_normx<float>(ctx, st, (const float*)V, ldv, nu, n, p, d, alpha);
}

symtd_status symtd_set_tuning(symtd_ctx* ctx, symtd_tune_key key, int64_t value) {
  if (!ctx) return SYMTD_EINVAL;
  if (value < 0) return ctx->fail(SYMTD_EINVAL, "tuning value %lld < 0", (long long)value);
  switch (key) {
    case SYMTD_TUNE_G1_BLOCKS: ctx->tune_g1_blocks = value; return SYMTD_OK;
    case SYMTD_TUNE_G2_SPLITS: ctx->tune_g2_splits = value; return SYMTD_OK;
    case SYMTD_TUNE_GRAPH: ctx->tune_graph = value; return SYMTD_OK;
    case SYMTD_TUNE_SPIN_LIMIT: ctx->tune_spin = value; return SYMTD_OK;
    case SYMTD_TUNE_FAULT_HANDOFF: ctx->tune_fault = value; return SYMTD_OK;
  }
  return ctx->fail(SYMTD_EINVAL, "unknown tuning key %d", (int)key);
}

symtd_status symtd_check(symtd_ctx* ctx, void* stream) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->set_device();
  if (s != SYMTD_OK) return s;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
  return ctx->take_device_error();
}

symtd_status symtd_profile_enable(symtd_ctx* ctx, uint32_t mask) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->prof_mask = mask;
  return SYMTD_OK;
}

symtd_status symtd_profile_reset(symtd_ctx* ctx) {
  if (!ctx) return SYMTD_EINVAL;
  for (auto& pe : ctx->pending) {
    (void)hipEventSynchronize(pe.stop);
    ctx->ev_pool.push_back(pe.start);
    ctx->ev_pool.push_back(pe.stop);
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

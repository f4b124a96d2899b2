// The tuning table and the autotuners (symtd_tune_*, symtd_autotune_*).
//
// The table is process-wide: every context, the grouped engine and the
// server consult it when they plan an evaluation.  An entry is keyed by
// (kind, precision, ceil(log2 n), ceil(log2 p), ceil(log2 columns)) and holds
// the launch shape measured fastest for that bucket:
//   SYMTD_TUNE_KIND_FG       v0 = blocks of the first product, v1 = splits
//                            of the observations in the second product
//   SYMTD_TUNE_KIND_GROUPED  v0 = 16-observation blocks per split of the
//                            grouped second product
// The shape is read from the table when an evaluation (or a grouped
// instance) is planned, so with a fixed table an instance's launch shape,
// and hence its summation order and its bits, depend only on its own sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <vector>

#include "grouped.hpp"
#include "runtime.hpp"

using namespace symtd;

namespace {

std::mutex g_mu;
std::vector<symtd_tune_entry> g_table;
std::atomic<int> g_force_split{0};   // set while the grouped tuner times a candidate

int bucket(int64_t x) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) ++b;
  return b;
}

bool same_key(const symtd_tune_entry& a, const symtd_tune_entry& b) {
  return a.kind == b.kind && a.prec == b.prec && a.n_bucket == b.n_bucket && a.p_bucket == b.p_bucket &&
         a.r_bucket == b.r_bucket;
}

bool lookup(int kind, int prec, int64_t n, int64_t p, int64_t cols, symtd_tune_entry* out) {
  symtd_tune_entry key{};
  key.kind = kind; key.prec = prec;
  key.n_bucket = bucket(n); key.p_bucket = bucket(p); key.r_bucket = bucket(cols);
  std::lock_guard<std::mutex> lk(g_mu);
  for (const symtd_tune_entry& e : g_table)
    if (same_key(e, key)) {
      *out = e;
      return true;
    }
  return false;
}

void put(const symtd_tune_entry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (symtd_tune_entry& x : g_table)
    if (same_key(x, e)) {
      x = e;
      return;
    }
  g_table.push_back(e);
}

symtd_tune_entry key_of(int kind, int prec, int64_t n, int64_t p, int64_t cols) {
  symtd_tune_entry e{};
  e.kind = kind; e.prec = prec;
  e.n_bucket = bucket(n); e.p_bucket = bucket(p); e.r_bucket = bucket(cols);
  return e;
}

}  // namespace

namespace symtd {

bool tuned_fg(bool f64, int64_t n, int64_t p, int64_t cols, int64_t* g1_blocks, int64_t* g2_splits) {
  symtd_tune_entry e;
  if (!lookup(SYMTD_TUNE_KIND_FG, f64 ? SYMTD_PREC_FP64 : SYMTD_PREC_FP32, n, p, cols, &e)) return false;
  *g1_blocks = e.v0;
  *g2_splits = e.v1;
  return true;
}

int grouped_split_blocks(bool f64, int64_t n, int64_t p, int64_t cols) {
  const int forced = g_force_split.load();
  if (forced > 0) return forced;
  symtd_tune_entry e;
  if (lookup(SYMTD_TUNE_KIND_GROUPED, f64 ? SYMTD_PREC_FP64 : SYMTD_PREC_FP32, n, p, cols, &e) && e.v0 > 0)
    return (int)std::min<int64_t>(e.v0, 1 << 20);
  return GG2_SPLIT_BLK;
}

}  // namespace symtd

namespace {

// seconds per call of fn (median of `rounds` timings of `reps` calls each)
template <typename F>
symtd_status time_calls(symtd_ctx* ctx, hipStream_t st, int reps, F fn, double* sec) {
  hipEvent_t a, b;
  hipError_t e;
  if ((e = hipEventCreate(&a)) != hipSuccess) return ctx->hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return ctx->hip_fail(e, "hipEventCreate");
  }
  symtd_status s = SYMTD_OK;
  std::vector<double> t;
  for (int w = 0; w < 2 && s == SYMTD_OK; ++w) s = fn();
  for (int round = 0; round < 3 && s == SYMTD_OK; ++round) {
    (void)hipEventRecord(a, st);
    for (int k = 0; k < reps && s == SYMTD_OK; ++k) s = fn();
    (void)hipEventRecord(b, st);
    if ((e = hipEventSynchronize(b)) != hipSuccess) {
      s = ctx->hip_fail(e, "hipEventSynchronize");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    t.push_back(1e-3 * ms / reps);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s != SYMTD_OK) return s;
  std::sort(t.begin(), t.end());
  *sec = t[t.size() / 2];
  return SYMTD_OK;
}

}  // namespace

extern "C" {

symtd_status symtd_tune_put(const symtd_tune_entry* e) {
  if (!e || (e->kind != SYMTD_TUNE_KIND_FG && e->kind != SYMTD_TUNE_KIND_GROUPED) || e->v0 < 0 || e->v1 < 0)
    return SYMTD_EINVAL;
  put(*e);
  return SYMTD_OK;
}

int64_t symtd_tune_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int64_t)g_table.size();
}

symtd_status symtd_tune_get(int64_t i, symtd_tune_entry* e) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!e || i < 0 || i >= (int64_t)g_table.size()) return SYMTD_EINVAL;
  *e = g_table[(size_t)i];
  return SYMTD_OK;
}

void symtd_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

symtd_status symtd_autotune_fg(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                               const double* nu, int64_t n, int64_t p, const void* A, int64_t lda,
                               const double* lambda, int64_t r, int d, symtd_prec prec, int reps,
                               symtd_tune_entry* out) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->check_common(dt, V, ldv, nu, n, p, d);
  if (s != SYMTD_OK) return s;
  if (!A || !lambda || r < 1 || lda < n || reps < 1) return ctx->fail(SYMTD_EINVAL, "bad A, lambda, r, lda or reps");
  if (!((dt == SYMTD_F64 && prec == SYMTD_PREC_FP64) || (dt == SYMTD_F32 && prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "the tuner covers the fp64 and fp32 products");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const bool f64 = dt == SYMTD_F64;
  const size_t esz = f64 ? 8 : 4;
  void* outs = nullptr;
  hipError_t e = hipMalloc(&outs, 2048 + 8 * (size_t)r + esz * (size_t)n * r);
  if (e != hipSuccess) return ctx->fail(SYMTD_ENOMEM, "tuner outputs");
  double* f = (double*)outs;
  double* g = f + 32;
  void* G = (char*)(g + r) + 256;
  G = (void*)(((uintptr_t)G + 255) & ~(uintptr_t)255);
  const FgPlan P = plan_fg(n, p, r, f64, ctx->cu_count, 0, 0);
  std::vector<int64_t> c1, c2;
  for (int q = 1; q <= 4; ++q) c1.push_back(std::max<int64_t>(1, std::min<int64_t>(P.nslab, ctx->cu_count * q / 4)));
  const int64_t base = std::max<int64_t>(1, (ctx->cu_count + P.rowblocks - 1) / P.rowblocks);
  for (int64_t m : {base / 2, base, 2 * base, 4 * base}) c2.push_back(std::max<int64_t>(1, std::min<int64_t>(P.nblk, m)));
  std::sort(c1.begin(), c1.end());
  c1.erase(std::unique(c1.begin(), c1.end()), c1.end());
  std::sort(c2.begin(), c2.end());
  c2.erase(std::unique(c2.begin(), c2.end()), c2.end());
  const int64_t keep1 = ctx->tune_g1_blocks, keep2 = ctx->tune_g2_splits;
  // every candidate is timed once in each of kRounds rounds, the candidates
  // in turn, so that a drift of clocks or caches over the sweep reaches them
  // all alike; a candidate's time is its median over the rounds
  struct Cand {
    int64_t x1, x2;
    std::vector<double> t;
  };
  std::vector<Cand> cs;
  for (int64_t x1 : c1)
    for (int64_t x2 : c2) cs.push_back(Cand{x1, x2, {}});
  constexpr int kRounds = 5;
  for (int round = 0; round < kRounds && s == SYMTD_OK; ++round)
    for (Cand& cd : cs) {
      ctx->tune_g1_blocks = cd.x1;
      ctx->tune_g2_splits = cd.x2;
      double sec = 0.0;
      s = time_calls(ctx, st, reps, [&]() {
        return symtd_fg(ctx, stream, dt, V, ldv, nu, n, p, A, lda, lambda, r, d, 0.0, prec, f, g, G, n);
      }, &sec);
      if (s != SYMTD_OK) break;
      cd.t.push_back(sec);
    }
  double best = INFINITY;
  int64_t b1 = c1.back(), b2 = base;
  for (Cand& cd : cs) {
    if (cd.t.empty()) continue;
    std::sort(cd.t.begin(), cd.t.end());
    const double med = cd.t[cd.t.size() / 2];
    if (med < best) { best = med; b1 = cd.x1; b2 = cd.x2; }
  }
  ctx->tune_g1_blocks = keep1;
  ctx->tune_g2_splits = keep2;
  (void)hipStreamSynchronize(st);
  (void)hipFree(outs);
  if (s != SYMTD_OK) return s;
  symtd_tune_entry en = key_of(SYMTD_TUNE_KIND_FG, prec, n, p, r);
  en.v0 = b1; en.v1 = b2; en.us = 1e6 * best;
  put(en);
  if (out) *out = en;
  return SYMTD_OK;
}

symtd_status symtd_autotune_grouped(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                                    const double* nu, int64_t n, int64_t p, int d, int64_t cols, int copies,
                                    int reps, symtd_tune_entry* out) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status s = ctx->check_common(dt, V, ldv, nu, n, p, d);
  if (s != SYMTD_OK) return s;
  if (cols < 1 || cols > 4096 || copies < 1 || copies > 4096 || reps < 1)
    return ctx->fail(SYMTD_EINVAL, "cols in [1, 4096], copies in [1, 4096], reps >= 1");
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const bool f64 = dt == SYMTD_F64;
  const size_t esz = f64 ? 8 : 4;
  const int64_t ld = (n + 3) / 4 * 4;
  // every copy evaluates the same factors (a scaled copy of V's first
  // columns, so that the products are not all zero) into its own outputs
  const size_t per = ((esz * (size_t)ld * cols + 255) / 256 + (8 * (size_t)cols + 255) / 256 + 2) * 256;
  const size_t shared = ((esz * (size_t)ld * cols + 255) / 256 + (8 * (size_t)cols + 255) / 256) * 256;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, shared + per * (size_t)copies);
  if (e != hipSuccess) return ctx->fail(SYMTD_ENOMEM, "tuner buffers");
  char* A = (char*)mem;
  double* lam = (double*)(A + (esz * (size_t)ld * cols + 255) / 256 * 256);
  std::vector<double> ones((size_t)cols, 1.0);
  e = hipMemsetAsync(A, 0, esz * (size_t)ld * cols, st);
  for (int64_t j = 0; j < cols && e == hipSuccess; ++j)
    e = hipMemcpyAsync(A + esz * (size_t)ld * j, (const char*)V + esz * (size_t)ldv * (j % p), esz * (size_t)n,
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(lam, ones.data(), 8 * (size_t)cols, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return ctx->hip_fail(e, "tuner set-up");
  }
  std::vector<symtd_fg_item> items((size_t)copies);
  char* q = (char*)mem + shared;
  for (int c = 0; c < copies; ++c, q += per) {
    symtd_fg_item& it = items[(size_t)c];
    it.V = V; it.ldv = ldv; it.nu = nu; it.n = n; it.p = p; it.d = d;
    it.A = A; it.lda = ld; it.lambda = lam; it.r = cols; it.models = 1; it.alpha = 0.0;
    it.G_A = q; it.ldg = ld;
    it.g_lambda = (double*)(q + (esz * (size_t)ld * cols + 255) / 256 * 256);
    it.f = (double*)(q + per - 256);
  }
  const symtd_prec prec = f64 ? SYMTD_PREC_FP64 : SYMTD_PREC_FP32;
  double best = INFINITY;
  int bsplit = GG2_SPLIT_BLK;
  const int64_t nblk = (p + 15) / 16;
  for (int sb : {4, 8, 16, 32, 64}) {
    if (sb > 4 && (int64_t)sb / 2 >= nblk) break;     // one split already covers every block
    g_force_split.store(sb);
    double sec = 0.0;
    s = time_calls(ctx, st, reps, [&]() {
      return symtd_fg_batched(ctx, stream, dt, prec, copies, items.data());
    }, &sec);
    g_force_split.store(0);
    if (s != SYMTD_OK) break;
    if (sec < best) { best = sec; bsplit = sb; }
  }
  (void)hipFree(mem);
  if (s != SYMTD_OK) return s;
  symtd_tune_entry en = key_of(SYMTD_TUNE_KIND_GROUPED, prec, n, p, cols);
  en.v0 = bsplit; en.v1 = 0; en.us = 1e6 * best;
  put(en);
  if (out) *out = en;
  return SYMTD_OK;
}

}  // extern "C"

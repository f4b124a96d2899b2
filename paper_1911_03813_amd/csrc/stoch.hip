// Host side of the stochastic objective (symtd_fg_sampled) and of the
// device Adam solver (symtd_solve_adam), Section 5 of the paper.
//
// An Adam step is: gather the draw's columns (k_gather), the four launches
// of Algorithm 2 on them for every lane side by side (run_fg), the Adam
// update of every running lane, and a tick of the step and draw counters.
// After every epoch the objective is estimated on the fixed set (run_fg
// again), and the decide / apply kernels keep or restore each lane's
// snapshot.  The host only reads the number of stopped lanes, once per
// epoch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lbfgs.hpp"
#include "runtime.hpp"
#include "stoch.hpp"

using namespace symtd;

namespace {

struct Slab {
  char* base;
  size_t off = 0;
  explicit Slab(void* b) : base((char*)b) {}
  template <typename X>
  X* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X* q = base ? (X*)(base + off) : nullptr;
    off += count * sizeof(X);
    return q;
  }
};

inline int64_t round4(int64_t n) { return (n + 3) / 4 * 4; }

template <typename T>
symtd_status run_fg_sampled(symtd_ctx* ctx, hipStream_t st, const T* V, int64_t ldv, const double* nu, int64_t n,
                            int64_t p, int64_t s, uint64_t seed, int64_t draw, const T* A, int64_t lda,
                            const double* lambda, int64_t r, int d, double* f, double* g, T* G, int64_t ldg,
                            int64_t* idx) {
  const int64_t lds = round4(n);
  Slab probe(nullptr);
  probe.take<T>((size_t)lds * s);
  probe.take<double>((size_t)s);
  symtd_status rc = ctx->reserve_solver(probe.off + 256);
  if (rc != SYMTD_OK) return rc;
  Slab cv(ctx->sws);
  T* Vs = cv.take<T>((size_t)lds * s);
  double* nus = cv.take<double>((size_t)s);
  GatherArgs<T> ga{V, ldv, nu, n, p, s, seed, STREAM_SAMPLE, nullptr, draw, Vs, lds, nus, idx};
  launch_gather<T>(st, ga);
  return run_fg<T>(ctx, st, Vs, lds, nus, n, s, A, lda, lambda, r, 1, d, 0.0, f, g, G, ldg);
}

template <typename T>
struct AdamLayout {
  double *x, *m, *v, *xs, *ms, *vs, *lam_t, *f_t, *glam_t, *f_est, *trace;
  T *A_t, *G_t, *Vs, *Ve;
  double *nus, *nue;
  LbLane<T>* starts;
  AdamLane<T>* lanes;
  AdamState* states;
  int64_t* draw;
  int* done;
  void carve(void* base, int64_t N, int64_t n, int64_t r, int R, int64_t lds, int64_t s, int64_t se, int64_t tl,
             size_t* bytes) {
    Slab t(base);
    x = t.take<double>((size_t)R * N);
    m = t.take<double>((size_t)R * N);
    v = t.take<double>((size_t)R * N);
    xs = t.take<double>((size_t)R * N);
    ms = t.take<double>((size_t)R * N);
    vs = t.take<double>((size_t)R * N);
    lam_t = t.take<double>((size_t)R * r);
    f_t = t.take<double>((size_t)R);
    glam_t = t.take<double>((size_t)R * r);
    f_est = t.take<double>((size_t)R);
    trace = t.take<double>((size_t)R * std::max<int64_t>(tl, 1));
    A_t = t.take<T>((size_t)R * n * r);
    G_t = t.take<T>((size_t)R * n * r);
    Vs = t.take<T>((size_t)lds * s);
    Ve = t.take<T>((size_t)lds * se);
    nus = t.take<double>((size_t)s);
    nue = t.take<double>((size_t)se);
    starts = t.take<LbLane<T>>((size_t)R);
    lanes = t.take<AdamLane<T>>((size_t)R);
    states = t.take<AdamState>((size_t)R);
    draw = t.take<int64_t>(1);
    done = t.take<int>(1);
    *bytes = t.off + 256;
  }
};

symtd_status check_adam(symtd_ctx* ctx, const symtd_problem* pb, const symtd_adam_opts* o,
                        const symtd_solve_result* out) {
  if (!pb || !o || !out) return ctx->fail(SYMTD_EINVAL, "null problem, options or result");
  symtd_status s = ctx->check_common(pb->dt, pb->V, pb->ldv, pb->nu, pb->n, pb->p, pb->d);
  if (s != SYMTD_OK) return s;
  if (pb->r < 1 || pb->r > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "rank r=%lld must be >= 1", (long long)pb->r);
  if (!((pb->dt == SYMTD_F64 && o->prec == SYMTD_PREC_FP64) || (pb->dt == SYMTD_F32 && o->prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)pb->dt, (int)o->prec);
  if (o->samples < 1 || o->samples > 0x7fffffffLL || o->est_samples < 1 || o->est_samples > 0x7fffffffLL)
    return ctx->fail(SYMTD_EINVAL, "samples and est_samples must be in [1, 2^31)");
  if (o->epoch_len < 1 || o->max_epochs < 1) return ctx->fail(SYMTD_EINVAL, "epoch_len and max_epochs must be >= 1");
  if (o->restarts < 1 || o->restarts > symtd_ctx::kFinalCounters)
    return ctx->fail(SYMTD_EINVAL, "restarts=%d outside [1, %d]", o->restarts, symtd_ctx::kFinalCounters);
  if (!(o->lr0 > 0.0) || !(o->lr1 > 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) ||
      !(o->beta2 >= 0.0 && o->beta2 < 1.0) || !(o->eps > 0.0))
    return ctx->fail(SYMTD_EINVAL, "Adam parameters out of range (lr > 0, 0 <= beta < 1, eps > 0)");
  if (o->init != SYMTD_INIT_GAUSS && o->init != SYMTD_INIT_RRF) return ctx->fail(SYMTD_EINVAL, "unknown init %d", (int)o->init);
  if (!out->A || !out->lambda || out->lda < pb->n) return ctx->fail(SYMTD_EINVAL, "bad result A, lambda or lda");
  if (out->trace_len < 0) return ctx->fail(SYMTD_EINVAL, "trace_len < 0");
  const size_t esz = pb->dt == SYMTD_F64 ? 8 : 4;
  if (((uintptr_t)out->A % esz) || ((uintptr_t)out->lambda % 8)) return ctx->fail(SYMTD_EALIGN, "result A or lambda misaligned");
  if (o->A0 && ((uintptr_t)o->A0 % esz)) return ctx->fail(SYMTD_EALIGN, "A0 misaligned");
  if (pb->r * o->restarts > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "r * restarts too large");
  return SYMTD_OK;
}

template <typename T>
symtd_status run_adam(symtd_ctx* ctx, hipStream_t st, const symtd_problem& pb, const symtd_adam_opts& o,
                      symtd_solve_result* out) {
  const T* V = (const T*)pb.V;
  const int64_t n = pb.n, p = pb.p, r = pb.r;
  const int R = o.restarts, d = pb.d;
  const int64_t N = r + n * r;
  const int64_t lds = round4(n), s = o.samples, se = o.est_samples;
  const int nb = (int)((N + AD_CHUNK - 1) / AD_CHUNK);
  const int lbnb = (int)((N + LB_CHUNK - 1) / LB_CHUNK);
  const int64_t tl = out->f_trace ? out->trace_len : 0;
  hipError_t e;

  AdamLayout<T> Lay;
  size_t bytes = 0;
  Lay.carve(nullptr, N, n, r, R, lds, s, se, tl, &bytes);
  symtd_status rc = ctx->reserve_solver(bytes);
  if (rc != SYMTD_OK) return rc;
  Lay.carve(ctx->sws, N, n, r, R, lds, s, se, tl, &bytes);
  if (!ctx->host_flag) {
    if ((e = hipHostMalloc((void**)&ctx->host_flag, sizeof(int) * 16, hipHostMallocDefault)) != hipSuccess)
      return ctx->hip_fail(e, "hipHostMalloc");
  }

  // start lanes (the solver's start kernels write x and the trial point)
  std::vector<LbLane<T>> sl(R);
  std::vector<AdamLane<T>> al(R);
  for (int k = 0; k < R; ++k) {
    LbLane<T>& L = sl[k];
    std::memset(&L, 0, sizeof(L));
    L.N = N; L.n = (int)n; L.r = (int)r; L.ld = (int)n; L.nb = lbnb; L.inst = 0;
    L.seed = o.seed; L.restart = k;
    L.A0 = o.A0 ? (const T*)o.A0 + (size_t)k * r * n : nullptr;
    L.x = Lay.x + (size_t)k * N;
    L.lam_t = Lay.lam_t + (size_t)k * r;
    L.A_t = Lay.A_t + (size_t)k * r * n;
    L.scale = 1.0;
    AdamLane<T>& A = al[k];
    A.N = N; A.r = (int)r; A.n = (int)n;
    A.x = Lay.x + (size_t)k * N; A.m = Lay.m + (size_t)k * N; A.v = Lay.v + (size_t)k * N;
    A.xs = Lay.xs + (size_t)k * N; A.ms = Lay.ms + (size_t)k * N; A.vs = Lay.vs + (size_t)k * N;
    A.lam_t = L.lam_t; A.A_t = L.A_t;
    A.glam = Lay.glam_t + (size_t)k * r; A.G = Lay.G_t + (size_t)k * r * n;
    A.f_est = Lay.f_est + k;
    A.state = Lay.states + k;
    A.trace = tl > 0 ? Lay.trace + (size_t)k * tl : nullptr;
    A.trace_len = tl;
  }
  const size_t vb = (size_t)R * N * sizeof(double);
  if ((e = hipMemcpyAsync(Lay.starts, sl.data(), sizeof(LbLane<T>) * R, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(Lay.lanes, al.data(), sizeof(AdamLane<T>) * R, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.m, 0, vb, st)) != hipSuccess || (e = hipMemsetAsync(Lay.v, 0, vb, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.states, 0, sizeof(AdamState) * R, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.draw, 0, sizeof(int64_t), st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.done, 0, sizeof(int), st)) != hipSuccess ||
      (tl > 0 && (e = hipMemsetAsync(Lay.trace, 0xFF, sizeof(double) * R * tl, st)) != hipSuccess))
    return ctx->hip_fail(e, "Adam set-up");
  if (o.A0) {
    launch_init_given<T>(lbnb, R, st, Lay.starts);
  } else if (o.init == SYMTD_INIT_GAUSS) {
    launch_init_gauss<T>(lbnb, R, st, Lay.starts);
    launch_norm_cols<T>(R, (int)r, st, Lay.starts);
  } else {
    if ((rc = run_rrf<T>(ctx, st, V, pb.ldv, n, p, r, R, o.seed, Lay.starts)) != SYMTD_OK) return rc;
  }

  AdamParams prm{o.lr0, o.lr1, o.beta1, o.beta2, o.eps, o.max_epochs, Lay.draw, Lay.done};
  // the fixed estimation set, the first estimate and the first snapshot
  GatherArgs<T> ge{V, pb.ldv, pb.nu, n, p, se, o.seed, STREAM_ESTIMATE, nullptr, 0, Lay.Ve, lds, Lay.nue, nullptr};
  launch_gather<T>(st, ge);
  auto estimate = [&]() {
    return run_fg<T>(ctx, st, Lay.Ve, lds, Lay.nue, n, se, Lay.A_t, n, Lay.lam_t, r, R, d, 0.0, Lay.f_est,
                     Lay.glam_t, Lay.G_t, n);
  };
  if ((rc = estimate()) != SYMTD_OK) return rc;
  launch_adam_init<T>(R, st, Lay.lanes, prm);
  launch_adam_apply<T>(nb, R, st, Lay.lanes);
  GatherArgs<T> gs{V, pb.ldv, pb.nu, n, p, s, o.seed, STREAM_SAMPLE, Lay.draw, 0, Lay.Vs, lds, Lay.nus, nullptr};
  for (int64_t ep = 0; ep < o.max_epochs; ++ep) {
    for (int k = 0; k < o.epoch_len; ++k) {
      launch_gather<T>(st, gs);
      if ((rc = run_fg<T>(ctx, st, Lay.Vs, lds, Lay.nus, n, s, Lay.A_t, n, Lay.lam_t, r, R, d, 0.0, Lay.f_t,
                          Lay.glam_t, Lay.G_t, n)) != SYMTD_OK)
        return rc;
      launch_adam_step<T>(nb, R, st, Lay.lanes, prm);
      launch_adam_tick<T>(R, st, Lay.lanes, prm);
    }
    if ((rc = estimate()) != SYMTD_OK) return rc;
    launch_adam_decide<T>(R, st, Lay.lanes, prm);
    launch_adam_apply<T>(nb, R, st, Lay.lanes);
    if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "Adam kernels");
    if ((e = hipMemcpyAsync(ctx->host_flag, Lay.done, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return ctx->hip_fail(e, "polling the Adam lanes");
    if ((rc = ctx->take_device_error()) != SYMTD_OK) return rc;
    if (ctx->host_flag[0] >= R) break;
  }

  // every lane's shifted objective on the whole data set, at its final point
  if ((rc = run_fg<T>(ctx, st, V, pb.ldv, pb.nu, n, p, Lay.A_t, n, Lay.lam_t, r, R, d, 0.0, Lay.f_t, Lay.glam_t,
                      Lay.G_t, n)) != SYMTD_OK)
    return rc;
  std::vector<double> fl(R);
  std::vector<AdamState> hs(R);
  if ((e = hipMemcpyAsync(fl.data(), Lay.f_t, sizeof(double) * R, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(hs.data(), Lay.states, sizeof(AdamState) * R, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return ctx->hip_fail(e, "reading the Adam lanes");
  if ((rc = ctx->take_device_error()) != SYMTD_OK) return rc;
  int best = 0;
  for (int k = 1; k < R; ++k)
    if (fl[k] < fl[best] || (std::isnan(fl[best]) && !std::isnan(fl[k]))) best = k;
  const T* Ab = Lay.A_t + (size_t)best * r * n;
  const double* lb = Lay.lam_t + (size_t)best * r;
  if ((e = hipMemcpy2DAsync(out->A, (size_t)out->lda * sizeof(T), Ab, (size_t)n * sizeof(T), (size_t)n * sizeof(T),
                            (size_t)r, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(out->lambda, lb, sizeof(double) * r, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return ctx->hip_fail(e, "copying the result");
  auto exit_of = [](const AdamState& a) {
    return a.reason == AD_CONVERGED ? SYMTD_EXIT_FTOL : SYMTD_EXIT_MAX_ITERS;
  };
  for (int k = 0; k < R; ++k) {
    if (out->f_restarts) out->f_restarts[k] = fl[k];
    if (out->iters_restarts) out->iters_restarts[k] = hs[k].steps;
    if (out->evals_restarts) out->evals_restarts[k] = hs[k].epochs;
    if (out->exit_restarts) out->exit_restarts[k] = exit_of(hs[k]);
  }
  if (tl > 0) {
    std::vector<double> tr((size_t)R * tl);
    if ((e = hipMemcpy(tr.data(), Lay.trace, sizeof(double) * tr.size(), hipMemcpyDeviceToHost)) != hipSuccess)
      return ctx->hip_fail(e, "reading the estimate trace");
    std::memcpy(out->f_trace, tr.data(), sizeof(double) * tr.size());
  }
  // the reported f: the shifted objective at the best lane, fp64 products
  double fb = 0.0;
  if ((rc = final_fp64<T>(ctx, st, V, pb.ldv, pb.nu, n, p, Ab, n, lb, r, d, 0.0, &fb)) != SYMTD_OK) return rc;
  out->f = fb;
  out->alpha = 0.0;
  out->rel_err = NAN;
  out->iters = hs[best].steps;
  out->evals = hs[best].epochs;
  out->exit_reason = exit_of(hs[best]);
  out->best_restart = best;
  out->steps = 0;
  for (int k = 0; k < R; ++k) out->steps = std::max<int64_t>(out->steps, hs[k].steps);
  return SYMTD_OK;
}

}  // namespace

extern "C" {

symtd_status symtd_fg_sampled(symtd_ctx* ctx, void* stream, symtd_dtype dt, const void* V, int64_t ldv,
                              const double* nu, int64_t n, int64_t p, int64_t s, uint64_t seed, int64_t draw,
                              const void* A, int64_t lda, const double* lambda, int64_t r, int d, symtd_prec prec,
                              double* f, double* g_lambda, void* G_A, int64_t ldg, int64_t* idx) {
  if (!ctx) return SYMTD_EINVAL;
  ctx->err.clear();
  symtd_status rc = ctx->take_device_error();
  if (rc != SYMTD_OK) return rc;
  if ((rc = ctx->check_common(dt, V, ldv, nu, n, p, d)) != SYMTD_OK) return rc;
  if (s < 1 || s > 0x7fffffffLL || draw < 0) return ctx->fail(SYMTD_EINVAL, "samples must be in [1, 2^31), draw >= 0");
  if (r < 1 || r > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "rank r=%lld must be >= 1", (long long)r);
  if (lda < n || ldg < n) return ctx->fail(SYMTD_EINVAL, "lda and ldg must be >= n");
  if (!A || !lambda || !f || !g_lambda || !G_A) return ctx->fail(SYMTD_EINVAL, "null A, lambda, f, g_lambda or G_A");
  if (!((dt == SYMTD_F64 && prec == SYMTD_PREC_FP64) || (dt == SYMTD_F32 && prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)dt, (int)prec);
  const size_t esz = dt == SYMTD_F64 ? 8 : 4;
  if (((uintptr_t)A % esz) || ((uintptr_t)G_A % esz) || ((uintptr_t)lambda % 8) || ((uintptr_t)f % 8) ||
      ((uintptr_t)g_lambda % 8) || ((uintptr_t)idx % 8))
    return ctx->fail(SYMTD_EALIGN, "misaligned pointer");
  if ((rc = ctx->set_device()) != SYMTD_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (dt == SYMTD_F64)
    return run_fg_sampled<double>(ctx, st, (const double*)V, ldv, nu, n, p, s, seed, draw, (const double*)A, lda,
                                  lambda, r, d, f, g_lambda, (double*)G_A, ldg, idx);
  return run_fg_sampled<float>(ctx, st, (const float*)V, ldv, nu, n, p, s, seed, draw, (const float*)A, lda, lambda,
                               r, d, f, g_lambda, (float*)G_A, ldg, idx);
}

symtd_status symtd_adam_opts_default(symtd_adam_opts* o) {
  if (!o) return SYMTD_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->prec = SYMTD_PREC_FP32;
  o->samples = 100;
  o->est_samples = 1000;
  o->epoch_len = 100;
  o->max_epochs = 1000;
  o->lr0 = 0.01;
  o->lr1 = 0.001;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
  o->restarts = 1;
  o->seed = 0;
  o->init = SYMTD_INIT_RRF;
  o->A0 = nullptr;
  return SYMTD_OK;
}

symtd_status symtd_solve_adam(symtd_ctx* ctx, void* stream, const symtd_problem* pb, const symtd_adam_opts* o,
                              symtd_solve_result* out) {
  if (!ctx) return SYMTD_EINVAL;
  Marker mk("symtd_solve_adam");
  ctx->err.clear();
  symtd_status rc = ctx->take_device_error();
  if (rc != SYMTD_OK) return rc;
  if ((rc = check_adam(ctx, pb, o, out)) != SYMTD_OK) return rc;
  if ((rc = ctx->set_device()) != SYMTD_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (pb->dt == SYMTD_F64) return run_adam<double>(ctx, st, *pb, *o, out);
  return run_adam<float>(ctx, st, *pb, *o, out);
}

}  // extern "C"

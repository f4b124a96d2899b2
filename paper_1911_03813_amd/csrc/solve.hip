// Host driver of symtd_solve: restarted L-BFGS with the state on the device.
//
// All restarts of a problem are evaluated together as side-by-side models
// (one pass over V per evaluation step), and each restart is one lane of the
// device L-BFGS (lbfgs.hpp).  The host enqueues evaluation steps in batches
// and only reads back one counter of finished lanes between batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.hpp"
#include "lbfgs.hpp"
#include "corrected.hpp"
#include "runtime.hpp"

using namespace symtd;

namespace {

struct Take {
  char* base;
  size_t off = 0;
  explicit Take(void* b) : base((char*)b) {}
  template <typename X>
  X* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X* p = base ? (X*)(base + off) : nullptr;
    off += count * sizeof(X);
    return p;
  }
};

template <typename T>
struct SolveLayout {
  double *x, *g, *dd, *S, *Y, *part, *lam_t, *f_t, *glam_t, *trace, *alpha;
  double *cm, *cM2, *clc, *cxd;   // noise correction: m, M2, terms per column, <X, Delta> partials
  bool corr = false, d4 = false;
  int64_t p = 0;
  T *A_t, *G_t;
  LbLane<T>* lanes;
  LbState* states;
  int* done;
  // zero-initialised region [x, S/Y end) and states
  size_t bytes;
  void carve(void* base, int64_t N, int64_t n, int64_t r, int R, int m, int nb, int64_t trace_len) {
    Take t(base);
    x = t.take<double>((size_t)R * N);
    g = t.take<double>((size_t)R * N);
    dd = t.take<double>((size_t)R * N);
    S = t.take<double>((size_t)R * m * N);
    Y = t.take<double>((size_t)R * m * N);
    part = t.take<double>((size_t)R * nb * LB_ND);
    lam_t = t.take<double>((size_t)R * r);
    f_t = t.take<double>((size_t)R);
    glam_t = t.take<double>((size_t)R * r);
    trace = t.take<double>((size_t)R * std::max<int64_t>(trace_len, 1));
    alpha = t.take<double>(1);
    A_t = t.take<T>((size_t)n * r * R);
    G_t = t.take<T>((size_t)n * r * R);
    lanes = t.take<LbLane<T>>((size_t)R);
    states = t.take<LbState>((size_t)R);
    done = t.take<int>(1);
    cm = t.take<double>((size_t)(corr ? n : 0));
    cM2 = t.take<double>((size_t)(corr && d4 ? n * n : 0));
    clc = t.take<double>((size_t)(corr ? R * r : 0));
    cxd = t.take<double>((size_t)(corr ? (p + 255) / 256 + 1 : 0));
    bytes = t.off + 256;
  }
};

// The saved state of a paused solve: a header, then the persistent device
// arrays in a fixed order, each at an 8-byte aligned offset.  Everything
// else on the device (the evaluation outputs, the dot partials, the
// correction's per-column terms) is rewritten by every step before it is
// read, and the lane descriptors follow from the problem and the options.
struct StateHeader {
  char magic[8];
  int32_t version, dt, prec, d, R, m, nb, init, alpha_mode, pad;
  int64_t n, p, r, N, trace_len, max_iters, max_evals, steps;
  uint64_t seed;
  double pgtol, ftol, sigma, alpha_given, alpha, scale;
  uint64_t bytes;
};
constexpr char kStateMagic[8] = {'S', 'Y', 'M', 'T', 'D', 'S', 'T', '1'};

struct StateLayout {
  size_t x, g, dd, S, Y, lam, A, states, done, trace, bytes;
  StateLayout(size_t esz, int64_t N, int64_t n, int64_t r, int R, int m, int64_t trace_len) {
    size_t off = sizeof(StateHeader);
    auto put = [&](size_t len) { off = (off + 7) & ~(size_t)7; const size_t at = off; off += len; return at; };
    x = put(sizeof(double) * R * N);
    g = put(sizeof(double) * R * N);
    dd = put(sizeof(double) * R * N);
    S = put(sizeof(double) * R * m * N);
    Y = put(sizeof(double) * R * m * N);
    lam = put(sizeof(double) * R * r);
    A = put(esz * n * r * R);
    states = put(sizeof(LbState) * R);
    done = put(sizeof(int));
    trace = put(sizeof(double) * R * trace_len);
    bytes = (off + 7) & ~(size_t)7;
  }
};

}  // namespace

namespace symtd {

symtd_status check_solve(symtd_ctx* ctx, const symtd_problem* pb, const symtd_solve_opts* o,
                         const symtd_solve_result* out) {
  if (!pb || !o || !out) return ctx->fail(SYMTD_EINVAL, "null problem, options or result");
  if (pb->r < 1 || pb->r > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "rank r=%lld must be >= 1", (long long)pb->r);
  if (o->m < 1 || o->m > LB_MMAX) return ctx->fail(SYMTD_EINVAL, "memory m=%d outside [1, %d]", o->m, LB_MMAX);
  if (!(o->pgtol >= 0.0) || !(o->ftol >= 0.0)) return ctx->fail(SYMTD_EINVAL, "pgtol and ftol must be >= 0");
  if (o->max_iters < 1 || o->max_evals < 1) return ctx->fail(SYMTD_EINVAL, "max_iters and max_evals must be >= 1");
  if (o->restarts < 1 || o->restarts > 4096) return ctx->fail(SYMTD_EINVAL, "restarts=%d outside [1, 4096]", o->restarts);
  if (o->init != SYMTD_INIT_GAUSS && o->init != SYMTD_INIT_RRF) return ctx->fail(SYMTD_EINVAL, "unknown init %d", (int)o->init);
  if (o->alpha_mode != SYMTD_ALPHA_COMPUTE && o->alpha_mode != SYMTD_ALPHA_GIVEN && o->alpha_mode != SYMTD_ALPHA_NONE)
    return ctx->fail(SYMTD_EINVAL, "unknown alpha mode %d", (int)o->alpha_mode);
  if (o->alpha_mode == SYMTD_ALPHA_GIVEN && !(o->alpha > 0.0 && std::isfinite(o->alpha)))
    return ctx->fail(SYMTD_EINVAL, "a given alpha must be positive and finite");
  if (!((pb->dt == SYMTD_F64 && o->prec == SYMTD_PREC_FP64) || (pb->dt == SYMTD_F32 && o->prec == SYMTD_PREC_FP32)))
    return ctx->fail(SYMTD_EINVAL, "unsupported storage/precision pair (dt=%d, prec=%d)", (int)pb->dt, (int)o->prec);
  if (!out->A || !out->lambda) return ctx->fail(SYMTD_EINVAL, "null result A or lambda");
  if (out->lda < pb->n) return ctx->fail(SYMTD_EINVAL, "result lda=%lld < n", (long long)out->lda);
  if (out->trace_len < 0) return ctx->fail(SYMTD_EINVAL, "trace_len < 0");
  if (o->check_every < 0) return ctx->fail(SYMTD_EINVAL, "check_every < 0");
  const size_t esz = pb->dt == SYMTD_F64 ? 8 : 4;
  if (((uintptr_t)out->A % esz) || ((uintptr_t)out->lambda % 8)) return ctx->fail(SYMTD_EALIGN, "result A or lambda misaligned");
  if (o->A0 && ((uintptr_t)o->A0 % esz)) return ctx->fail(SYMTD_EALIGN, "A0 misaligned");
  symtd_status s = ctx->check_common(pb->dt, pb->V, pb->ldv, pb->nu, pb->n, pb->p, pb->d);
  if (s != SYMTD_OK) return s;
  if ((int64_t)pb->r * o->restarts > 0x7fffffffLL) return ctx->fail(SYMTD_EINVAL, "r * restarts too large");
  if (!(o->sigma >= 0.0) || !std::isfinite(o->sigma)) return ctx->fail(SYMTD_EINVAL, "sigma must be finite and >= 0");
  if (o->sigma > 0.0 && ((pb->d != 3 && pb->d != 4) || pb->n > CORR_NMAX))
    return ctx->fail(SYMTD_EINVAL, "the noise correction is derived for d = 3 and d = 4 (n <= %d)", CORR_NMAX);
  if (o->pause_after < 0) return ctx->fail(SYMTD_EINVAL, "pause_after < 0");
  return SYMTD_OK;
}

}  // namespace symtd

namespace {

template <typename T>
symtd_status run_solve(symtd_ctx* ctx, hipStream_t st, const symtd_problem& pb, const symtd_solve_opts& o,
                       symtd_solve_result* out) {
  const T* V = (const T*)pb.V;
  const int64_t n = pb.n, p = pb.p, r = pb.r;
  const int R = o.restarts, m = o.m, d = pb.d;
  const int64_t N = r + n * r;
  const int nb = (int)((N + LB_CHUNK - 1) / LB_CHUNK);
  const int64_t trace_len = out->f_trace ? out->trace_len : 0;
  hipError_t e;

  SolveLayout<T> Lay;
  Lay.corr = o.sigma > 0.0;
  Lay.d4 = d == 4;
  Lay.p = p;
  Lay.carve(nullptr, N, n, r, R, m, nb, trace_len);
  symtd_status s = ctx->reserve_solver(Lay.bytes);
  if (s != SYMTD_OK) return s;
  Lay.carve(ctx->sws, N, n, r, R, m, nb, trace_len);
  if (!ctx->host_flag) {
    e = hipHostMalloc((void**)&ctx->host_flag, sizeof(int) * 16, hipHostMallocDefault);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipHostMalloc");
  }

  // a saved state to continue from: it must come from this problem and these options
  const StateLayout SL(sizeof(T), N, n, r, R, m, trace_len);
  StateHeader H{};
  if (o.state_in) {
    std::memcpy(&H, o.state_in, sizeof(H));
    const bool same = std::memcmp(H.magic, kStateMagic, 8) == 0 && H.version == 1 && H.dt == (int)pb.dt &&
                      H.prec == (int)o.prec && H.d == d && H.R == R && H.m == m && H.nb == nb &&
                      H.init == (int)o.init && H.alpha_mode == (int)o.alpha_mode && H.n == n && H.p == p &&
                      H.r == r && H.N == N && H.trace_len == trace_len && H.max_iters == o.max_iters &&
                      H.max_evals == o.max_evals && H.seed == o.seed && H.pgtol == o.pgtol && H.ftol == o.ftol &&
                      H.sigma == o.sigma && H.alpha_given == (o.alpha_mode == SYMTD_ALPHA_GIVEN ? o.alpha : 0.0) &&
                      H.bytes == SL.bytes;
    if (!same) return ctx->fail(SYMTD_EINVAL, "the saved state belongs to another problem or other options");
    if (o.pause_after > 0 && o.pause_after <= H.steps)
      return ctx->fail(SYMTD_EINVAL, "pause_after=%lld is not past the %lld steps of the saved state",
                       (long long)o.pause_after, (long long)H.steps);
  }

  // alpha and the scale of the objective
  double alpha = 0.0;
  if (o.state_in) {
    alpha = H.alpha;
  } else if (o.alpha_mode == SYMTD_ALPHA_COMPUTE) {
    if ((s = run_normx<T>(ctx, st, V, pb.ldv, pb.nu, n, p, d, Lay.alpha)) != SYMTD_OK) return s;
    if ((e = hipMemcpyAsync(&ctx->host_flag[2], Lay.alpha, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return ctx->hip_fail(e, "reading alpha");
    std::memcpy(&alpha, &ctx->host_flag[2], sizeof(double));
    if (!(alpha > 0.0 && std::isfinite(alpha))) return ctx->fail(SYMTD_ENONFINITE, "||X||^2 = %g is not positive", alpha);
  } else if (o.alpha_mode == SYMTD_ALPHA_GIVEN) {
    alpha = o.alpha;
  }
  // noise correction: the data's statistics, and alpha_c from alpha
  const Correction corr{Lay.cm, Lay.cM2, o.sigma, d};
  if (Lay.corr) {
    launch_stats<T>(st, V, pb.ldv, pb.nu, n, p, Lay.cm, d == 4 ? Lay.cM2 : nullptr);
    if (o.alpha_mode == SYMTD_ALPHA_COMPUTE && !o.state_in) {
      if ((s = corrected_alpha<T>(ctx, st, corr, V, pb.ldv, pb.nu, n, p, alpha, &alpha, Lay.cxd)) != SYMTD_OK) return s;
      if (!(alpha > 0.0 && std::isfinite(alpha)))
        return ctx->fail(SYMTD_ENONFINITE, "||X - Delta||^2 = %g is not positive", alpha);
    }
  }
  const double scale = o.state_in ? H.scale : (alpha > 0.0 ? alpha : 1.0);

  // lane descriptors and zeroed state
  std::vector<LbLane<T>> lanes(R);
  for (int k = 0; k < R; ++k) {
    LbLane<T>& L = lanes[k];
    L.N = N; L.n = (int)n; L.r = (int)r; L.ld = (int)n; L.nb = nb; L.inst = 0;
    L.seed = o.seed; L.restart = k;
    L.A0 = o.A0 ? (const T*)o.A0 + (size_t)k * r * n : nullptr;
    L.x = Lay.x + (size_t)k * N; L.g = Lay.g + (size_t)k * N; L.d = Lay.dd + (size_t)k * N;
    L.S = Lay.S + (size_t)k * m * N; L.Y = Lay.Y + (size_t)k * m * N;
    L.lam_t = Lay.lam_t + (size_t)k * r; L.A_t = Lay.A_t + (size_t)k * r * n;
    L.f_t = Lay.f_t + k; L.glam_t = Lay.glam_t + (size_t)k * r; L.G_t = Lay.G_t + (size_t)k * r * n;
    L.scale = scale;
    L.part = Lay.part + (size_t)k * nb * LB_ND;
    L.trace = trace_len > 0 ? Lay.trace + (size_t)k * trace_len : nullptr;
    L.trace_len = trace_len;
    L.state = Lay.states + k;
    L.done_flag = nullptr;
    L.m = m; L.pgtol = o.pgtol; L.ftol = o.ftol; L.max_iters = o.max_iters; L.max_evals = o.max_evals;
  }
  const size_t vec_bytes = (size_t)R * N * sizeof(double);
  // the persistent arrays and where the saved state keeps them
  struct Part { void* dev; size_t off, len; };
  const Part parts[] = {
      {Lay.x, SL.x, vec_bytes}, {Lay.g, SL.g, vec_bytes}, {Lay.dd, SL.dd, vec_bytes},
      {Lay.S, SL.S, vec_bytes * m}, {Lay.Y, SL.Y, vec_bytes * m}, {Lay.lam_t, SL.lam, sizeof(double) * R * r},
      {Lay.A_t, SL.A, sizeof(T) * n * r * R}, {Lay.states, SL.states, sizeof(LbState) * R},
      {Lay.done, SL.done, sizeof(int)}, {Lay.trace, SL.trace, sizeof(double) * R * trace_len}};
  int64_t steps = 0;
  if (o.state_in) {
    if ((e = hipMemcpyAsync(Lay.lanes, lanes.data(), sizeof(LbLane<T>) * R, hipMemcpyHostToDevice, st)) != hipSuccess)
      return ctx->hip_fail(e, "solver set-up");
    for (const Part& q : parts)
      if (q.len > 0 && (e = hipMemcpyAsync(q.dev, (const char*)o.state_in + q.off, q.len, hipMemcpyHostToDevice,
                                           st)) != hipSuccess)
        return ctx->hip_fail(e, "restoring the saved state");
    steps = H.steps;
  } else if ((e = hipMemcpyAsync(Lay.lanes, lanes.data(), sizeof(LbLane<T>) * R, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.g, 0, vec_bytes, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.dd, 0, vec_bytes, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.S, 0, vec_bytes * m, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.Y, 0, vec_bytes * m, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.states, 0, sizeof(LbState) * R, st)) != hipSuccess ||
      (e = hipMemsetAsync(Lay.done, 0, sizeof(int), st)) != hipSuccess ||
      (trace_len > 0 && (e = hipMemsetAsync(Lay.trace, 0xFF, sizeof(double) * R * trace_len, st)) != hipSuccess))
    return ctx->hip_fail(e, "solver set-up");

  // starts (a resumed solve has its points already)
  if (o.state_in) {
  } else if (o.A0) {
    launch_init_given<T>(nb, R, st, Lay.lanes);
  } else if (o.init == SYMTD_INIT_GAUSS) {
    launch_init_gauss<T>(nb, R, st, Lay.lanes);
    launch_norm_cols<T>(R, (int)r, st, Lay.lanes);
  } else {
    if ((s = run_rrf<T>(ctx, st, V, pb.ldv, n, p, r, R, o.seed, Lay.lanes)) != SYMTD_OK) return s;
  }
  if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "start kernels");

  LbParams prm{Lay.done};
  // steps between polls: enough to keep the queue ahead of the device, few
  // enough that little work is done after the last lane has stopped
  const double work = 4.0 * (double)n * (double)p * (double)r * R;
  const int K = o.check_every > 0 ? o.check_every : (work > 1e9 ? 4 : work > 1e7 ? 16 : 64);
  const int64_t step_cap = o.max_evals + 2;   // every running lane spends one evaluation per step
  while (true) {
    // a pause falls on a poll
    const int64_t Kr = o.pause_after > 0 ? std::min<int64_t>(K, o.pause_after - steps) : K;
    Marker mk("solve steps");
    for (int64_t k = 0; k < Kr; ++k) {
      if ((s = run_fg<T>(ctx, st, V, pb.ldv, pb.nu, n, p, Lay.A_t, n, Lay.lam_t, r, R, d, alpha, Lay.f_t, Lay.glam_t,
                         Lay.G_t, n)) != SYMTD_OK)
        return s;
      if (Lay.corr)
        launch_correction<T>(st, corr, Lay.A_t, n, (int)n, (int)r, R, Lay.lam_t, Lay.f_t, Lay.glam_t, Lay.G_t, n,
                             Lay.clc);
      launch_lb_dots<T>(nb, R, st, Lay.lanes);
      launch_lb_step<T>(R, st, Lay.lanes, prm);
      launch_lb_apply<T>(nb, R, st, Lay.lanes);
      ++steps;
    }
    if ((e = hipGetLastError()) != hipSuccess) return ctx->hip_fail(e, "solver kernels");
    if ((e = hipMemcpyAsync(ctx->host_flag, Lay.done, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return ctx->hip_fail(e, "polling the solver");
    if ((s = ctx->take_device_error()) != SYMTD_OK) return s;
    if (ctx->host_flag[0] >= R) break;
    if (o.pause_after > 0 && steps >= o.pause_after) {
      // pause: save the state between two steps
      if (o.state_out) {
        StateHeader W{};
        std::memcpy(W.magic, kStateMagic, 8);
        W.version = 1; W.dt = (int)pb.dt; W.prec = (int)o.prec; W.d = d; W.R = R; W.m = m; W.nb = nb;
        W.init = (int)o.init; W.alpha_mode = (int)o.alpha_mode;
        W.n = n; W.p = p; W.r = r; W.N = N; W.trace_len = trace_len; W.max_iters = o.max_iters;
        W.max_evals = o.max_evals; W.steps = steps; W.seed = o.seed; W.pgtol = o.pgtol; W.ftol = o.ftol;
        W.sigma = o.sigma; W.alpha_given = o.alpha_mode == SYMTD_ALPHA_GIVEN ? o.alpha : 0.0;
        W.alpha = alpha; W.scale = scale; W.bytes = SL.bytes;
        for (const Part& q : parts)
          if (q.len > 0 && (e = hipMemcpyAsync((char*)o.state_out + q.off, q.dev, q.len, hipMemcpyDeviceToHost,
                                               st)) != hipSuccess)
            return ctx->hip_fail(e, "saving the state");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return ctx->hip_fail(e, "saving the state");
        std::memcpy(o.state_out, &W, sizeof(W));
      }
      out->exit_reason = SYMTD_EXIT_RUNNING;
      out->steps = steps;
      return SYMTD_OK;
    }
    if (steps > step_cap) return ctx->fail(SYMTD_EDEVICE, "solver did not stop within %lld steps", (long long)steps);
  }

  // results
  std::vector<LbState> hs(R);
  if ((e = hipMemcpy(hs.data(), Lay.states, sizeof(LbState) * R, hipMemcpyDeviceToHost)) != hipSuccess)
    return ctx->hip_fail(e, "reading the solver state");
  int best = 0;
  for (int k = 1; k < R; ++k)
    if (hs[k].f < hs[best].f || (std::isnan(hs[best].f) && !std::isnan(hs[k].f))) best = k;
  const LbLane<T>& B = lanes[best];
  if ((e = hipMemcpy2DAsync(out->A, (size_t)out->lda * sizeof(T), B.A_t, (size_t)n * sizeof(T), (size_t)n * sizeof(T),
                            (size_t)r, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(out->lambda, B.lam_t, sizeof(double) * r, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return ctx->hip_fail(e, "copying the result");
  if (out->f_trace && trace_len > 0 &&
      (e = hipMemcpyAsync(out->f_trace, Lay.trace, sizeof(double) * R * trace_len, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return ctx->hip_fail(e, "copying the trace");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return ctx->hip_fail(e, "finishing the solve");
  for (int k = 0; k < R; ++k) {
    if (out->f_restarts) out->f_restarts[k] = hs[k].f * scale;
    if (out->iters_restarts) out->iters_restarts[k] = hs[k].iters;
    if (out->evals_restarts) out->evals_restarts[k] = hs[k].evals;
    if (out->exit_restarts) out->exit_restarts[k] = hs[k].reason;
  }
  // the reported f and relative error come from an fp64 evaluation at the
  // best restart's final point (the working precision may be fp32)
  double f64 = 0.0;
  if ((s = final_fp64<T>(ctx, st, V, pb.ldv, pb.nu, n, p, B.A_t, n, B.lam_t, r, d, alpha, &f64,
                         Lay.corr ? &corr : nullptr)) != SYMTD_OK)
    return s;
  out->f = f64;
  out->alpha = alpha;
  out->rel_err = alpha > 0.0 ? std::sqrt(std::max(out->f, 0.0) / alpha) : NAN;
  out->iters = hs[best].iters;
  out->evals = hs[best].evals;
  out->exit_reason = hs[best].reason;
  out->best_restart = best;
  out->steps = steps;
  return SYMTD_OK;
}

}  // namespace

extern "C" {

symtd_status symtd_solve_opts_default(symtd_solve_opts* o) {
  if (!o) return SYMTD_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->prec = SYMTD_PREC_FP32;
  o->m = 5;
  o->pgtol = 1e-4;
  o->ftol = 2.220446049250313e-09;
  o->max_iters = 10000;
  o->max_evals = 50000;
  o->restarts = 1;
  o->seed = 0;
  o->init = SYMTD_INIT_RRF;
  o->alpha_mode = SYMTD_ALPHA_COMPUTE;
  o->alpha = 0.0;
  o->A0 = nullptr;
  o->check_every = 0;
  o->sigma = 0.0;
  o->pause_after = 0;
  o->state_out = nullptr;
  o->state_in = nullptr;
  return SYMTD_OK;
}

symtd_status symtd_solve_state_bytes(const symtd_problem* pb, const symtd_solve_opts* o, int64_t trace_len,
                                     size_t* bytes) {
  if (!pb || !o || !bytes || pb->r < 1 || pb->n < 1 || o->restarts < 1 || o->restarts > 4096 || o->m < 1 ||
      o->m > LB_MMAX || trace_len < 0 || (pb->dt != SYMTD_F64 && pb->dt != SYMTD_F32))
    return SYMTD_EINVAL;
  const int64_t N = pb->r + pb->n * pb->r;
  *bytes = StateLayout(pb->dt == SYMTD_F64 ? 8 : 4, N, pb->n, pb->r, o->restarts, o->m, trace_len).bytes;
  return SYMTD_OK;
}

symtd_status symtd_solve(symtd_ctx* ctx, void* stream, const symtd_problem* pb, const symtd_solve_opts* o,
                         symtd_solve_result* out) {
  if (!ctx) return SYMTD_EINVAL;
  Marker mk("symtd_solve");
  ctx->err.clear();
  symtd_status s = ctx->take_device_error();
  if (s != SYMTD_OK) return s;
  if ((s = check_solve(ctx, pb, o, out)) != SYMTD_OK) return s;
  if ((s = ctx->set_device()) != SYMTD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (pb->dt == SYMTD_F64) return run_solve<double>(ctx, st, *pb, *o, out);
  return run_solve<float>(ctx, st, *pb, *o, out);
}

}  // extern "C"

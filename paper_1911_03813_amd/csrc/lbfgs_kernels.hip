// Kernels of the device-resident L-BFGS solve and of its starting points.
//
// Readings of the paper's optimiser (Section 4: L-BFGS, memory m, limits on
// iterations and evaluations, gradient tolerance) that these kernels follow:
//   * direction: the L-BFGS inverse Hessian of the last m pairs with
//     H0 = gamma I, gamma = s'y / y'y of the newest pair; a pair is kept only
//     if s'y > 1e-10 y'y; a direction that is not a descent direction clears
//     the memory and uses -g;
//   * line search: strong Wolfe (c1 = 1e-3, c2 = 0.9); first trial
//     min(1, 1/||g||_2) along -g, else 1; bracketing doubles the trial (up to
//     1e10); zoom takes the minimiser of the cubic through both ends' values
//     and slopes, or the midpoint if that is not finite or falls outside the
//     middle 80% of the interval (or the upper end's values are not finite);
//     at most 20 evaluations, and an interval shorter than 1e-14 of its ends
//     fails the search;
//   * stopping after each accepted step: ||g||_inf <= pgtol, then
//     phi_k - phi_{k+1} <= ftol max(|phi_k|, |phi_{k+1}|, 1), then the
//     iteration limit, then the evaluation limit.
#include <math.h>

#include "grouped.hpp"
#include "kcommon.hpp"
#include "lbfgs.hpp"
#include "philox.hpp"

namespace symtd {

namespace {

constexpr double LB_C1 = 1e-3;
constexpr double LB_C2 = 0.9;
constexpr int LB_MAXLS = 20;
constexpr double LB_STEP_MAX = 1e10;
constexpr double LB_SKIP = 1e-10;
constexpr double LB_COLLAPSE = 1e-14;

enum { EX_PGTOL = 1, EX_FTOL = 2, EX_MAX_ITERS = 3, EX_MAX_EVALS = 4, EX_LINESEARCH = 5, EX_NONFINITE = 6 };

// trial gradient element e of a lane (divided by the scale)
// (both sources are read from valid elements and the value selected after:
// a conditional load would be a branch that waits for its value)
template <typename T>
__device__ __forceinline__ double trial_grad(const LbLane<T>& ln, int64_t e) {
  const bool lam = e < ln.r;
  const double a = gload(ln.glam_t + (lam ? e : ln.r - 1));
  const double b = (double)gload(ln.G_t + (lam ? 0 : e - ln.r));
  return (lam ? a : b) / ln.scale;
}

template <typename T>
__device__ __forceinline__ void write_trial(const LbLane<T>& ln, int64_t e, double xt) {
  if (e < ln.r) gstore(ln.lam_t + e, xt);
  else gstore(ln.A_t + (e - ln.r), (T)xt);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

}  // namespace

// ---------------------------------------------------------------------------
// k_lb_dots: one pass over a lane's vectors computing, for the trial gradient
// gt, y_t = gt - g and the stored pairs (slots s < count):
//   gt'gt, gt'd, y_t'y_t, y_t'd, y_t'gt, max|gt|, gt'S_s, gt'Y_s, S_s'y_t, Y_s'y_t
// as per-block partials (fixed order: thread-strided, then a fixed tree).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_lb_dots(const LbLane<T>* lanes, const LbItem* items) {
  int L = blockIdx.y, b = blockIdx.x;
  if (items) {
    const LbItem it = items[blockIdx.x];
    L = it.lane;
    b = it.blk;
  }
  const LbLane<T> ln = lanes[L];
  if (b >= ln.nb) return;
  const int phase = ln.state->phase;
  if (phase == LB_DONE) return;
  const int cnt = ln.state->count;
  double acc[LB_ND];
#pragma unroll
  for (int i = 0; i < LB_ND; ++i) acc[i] = 0.0;
  double mx = 0.0;
  for (int k = 0; k < LB_CHUNK / 256; ++k) {
    const int64_t e = (int64_t)b * LB_CHUNK + k * 256 + threadIdx.x;
    if (e >= ln.N) break;
    const double gt = trial_grad(ln, e);
    const double ge = gload(ln.g + e), de = gload(ln.d + e);
    const double yt = gt - ge;
    acc[LB_GTGT] = fma(gt, gt, acc[LB_GTGT]);
    acc[LB_GTD] = fma(gt, de, acc[LB_GTD]);
    acc[LB_YTYT] = fma(yt, yt, acc[LB_YTYT]);
    acc[LB_YTD] = fma(yt, de, acc[LB_YTD]);
    acc[LB_YTGT] = fma(yt, gt, acc[LB_YTGT]);
    mx = fmax(mx, fabs(gt));
    // the stored pairs: every slot read (unused ones from slot 0, a valid
    // one), so that all loads are in flight together; only s < cnt count
    double Sv[LB_MMAX], Yv[LB_MMAX];
#pragma unroll
    for (int s = 0; s < LB_MMAX; ++s) {
      const int64_t sq = s < cnt ? s : 0;
      Sv[s] = gload(ln.S + sq * ln.N + e);
      Yv[s] = gload(ln.Y + sq * ln.N + e);
    }
#pragma unroll
    for (int s = 0; s < LB_MMAX; ++s) {
      if (s < cnt) {
        acc[LB_GTS + s] = fma(gt, Sv[s], acc[LB_GTS + s]);
        acc[LB_GTY + s] = fma(gt, Yv[s], acc[LB_GTY + s]);
        acc[LB_SYT + s] = fma(Sv[s], yt, acc[LB_SYT + s]);
        acc[LB_YYT + s] = fma(Yv[s], yt, acc[LB_YYT + s]);
      }
    }
  }
  acc[LB_MAXG] = mx;
  __shared__ double red[4][LB_ND];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < LB_ND; ++i) {
    const double v = i == LB_MAXG ? wave_max(acc[i]) : wave_sum(acc[i]);
    if (lane == 0) red[wave][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < LB_ND) {
    const int i = threadIdx.x;
    double v;
    if (i == LB_MAXG) v = fmax(fmax(red[0][i], red[1][i]), fmax(red[2][i], red[3][i]));
    else v = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
    ln.part[(int64_t)b * LB_ND + i] = v;
  }
}

// ---------------------------------------------------------------------------
// k_lb_step: the decisions of one lane (one block of 64 threads; the sums of
// the partials in fixed order by 38 threads, the logic on thread 0).
// ---------------------------------------------------------------------------
namespace {

__device__ double cubic_min(double a, double fa, double da, double b, double fb, double db, bool& ok) {
  ok = false;
  const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - da * db;
  if (!isfinite(disc) || disc < 0.0) return 0.0;
  const double d2 = copysign(sqrt(disc), b - a);
  const double den = db - da + 2.0 * d2;
  if (den == 0.0 || !isfinite(den)) return 0.0;
  const double t = b - (b - a) * (db + d2 - d1) / den;
  ok = isfinite(t);
  return t;
}

__device__ double zoom_trial(const LbState& s) {
  const double left = fmin(s.lo_a, s.hi_a), right = fmax(s.lo_a, s.hi_a);
  const double width = right - left;
  const double mid = 0.5 * (s.lo_a + s.hi_a);
  if (!s.hi_fin) return mid;
  bool ok;
  const double t = cubic_min(s.lo_a, s.lo_f, s.lo_d, s.hi_a, s.hi_f, s.hi_d, ok);
  if (!ok || t < left + 0.1 * width || t > right - 0.1 * width) return mid;
  return t;
}

template <typename T>
__device__ void begin_search(LbState& s, const LbLane<T>& ln, double a1) {
  s.phase = LB_BRACKET;
  s.a = a1;
  s.ls_i = 1;
  s.ls_evals = 0;
  s.ls_limit = min((int64_t)LB_MAXLS, ln.max_evals - s.evals);
  s.a_prev = 0.0;
  s.f_prev = s.f;
  s.d_prev = s.dphi0;
}

template <typename T>
__device__ void finish(LbState& s, const LbLane<T>& ln, const LbParams& prm, int reason, int action) {
  s.phase = LB_DONE;
  s.reason = reason;
  s.action = action;
  if (prm.done_count) atomicAdd(prm.done_count, 1);
  if (ln.done_flag) *ln.done_flag = 1;
}

// a new direction at the accepted point (g = gt), using the pairs in the ring
template <typename T>
__device__ void new_direction(LbState& s, const LbLane<T>& ln, const double* D) {
  const int m = ln.m;
  const double gtgt = D[LB_GTGT];
  for (int i = 0; i < LB_MMAX; ++i) { s.cs[i] = 0.0; s.cy[i] = 0.0; }
  bool reset = s.count == 0;
  if (!reset) {
    const int c = s.count;
    int o[LB_MMAX];
    double u[LB_MMAX], v[LB_MMAX], t[LB_MMAX], w[LB_MMAX], top[LB_MMAX];
    for (int i = 0; i < c; ++i) {
      o[i] = ((s.head - c + i) % m + m) % m;
      const int sl = o[i];
      if (s.store && sl == s.slot) {
        u[i] = s.a_acc * D[LB_GTD];     // s_new' gt = a (d' gt)
        v[i] = D[LB_YTGT];              // y_new' gt
      } else {
        u[i] = D[LB_GTS + sl];
        v[i] = D[LB_GTY + sl];
      }
    }
    // t = R^{-1} u with R[i][j] = s_{o_i}' y_{o_j} (i <= j)
    for (int i = c - 1; i >= 0; --i) {
      double acc = u[i];
      for (int j = i + 1; j < c; ++j) acc -= s.SY[o[i]][o[j]] * t[j];
      t[i] = acc / s.SY[o[i]][o[i]];
    }
    // w = (D + gamma Y'Y) t - gamma v
    for (int i = 0; i < c; ++i) {
      double acc = s.SY[o[i]][o[i]] * t[i];
      double yy = 0.0;
      for (int j = 0; j < c; ++j) yy += s.YY[o[i]][o[j]] * t[j];
      w[i] = acc + s.gamma * yy - s.gamma * v[i];
    }
    // top = R^{-T} w
    for (int i = 0; i < c; ++i) {
      double acc = w[i];
      for (int j = 0; j < i; ++j) acc -= s.SY[o[j]][o[i]] * top[j];
      top[i] = acc / s.SY[o[i]][o[i]];
    }
    // d = -gamma gt - S top + gamma Y t
    double dphi = -s.gamma * gtgt;
    for (int i = 0; i < c; ++i) {
      s.cs[o[i]] = -top[i];
      s.cy[o[i]] = s.gamma * t[i];
      dphi += -top[i] * u[i] + s.gamma * t[i] * v[i];
    }
    s.coef_g = -s.gamma;
    s.dphi0 = dphi;
    if (!(isfinite(dphi) && dphi < 0.0)) reset = true;
  }
  if (reset) {
    s.count = 0;
    s.head = 0;
    s.store = 0;
    for (int i = 0; i < LB_MMAX; ++i) { s.cs[i] = 0.0; s.cy[i] = 0.0; }
    s.coef_g = -1.0;
    s.dphi0 = -gtgt;
    begin_search(s, ln, fmin(1.0, 1.0 / sqrt(gtgt)));
  } else {
    begin_search(s, ln, 1.0);
  }
}

template <typename T>
__device__ void accept(LbState& s, const LbLane<T>& ln, const LbParams& prm, const double* D, double phi) {
  const int m = ln.m;
  s.a_acc = s.a;
  s.iters += 1;
  const double sy = s.a_acc * D[LB_YTD];
  const double yy = D[LB_YTYT];
  const double f_old = s.f;
  s.f = phi;
  if (ln.trace && s.iters < ln.trace_len) ln.trace[s.iters] = phi * ln.scale;
  int reason = 0;
  if (D[LB_MAXG] <= ln.pgtol) reason = EX_PGTOL;
  else if (f_old - phi <= ln.ftol * fmax(fmax(fabs(f_old), fabs(phi)), 1.0)) reason = EX_FTOL;
  else if (s.iters >= ln.max_iters) reason = EX_MAX_ITERS;
  else if (s.evals >= ln.max_evals) reason = EX_MAX_EVALS;
  if (reason) {
    s.store = 0;
    finish(s, ln, prm, reason, LB_ACCEPT_FINAL);
    return;
  }
  s.store = sy > LB_SKIP * yy;
  if (s.store) {
    const int slot = s.head;
    s.slot = slot;
    // entries with the pairs that stay (the slot being replaced is not among them)
    const int c_old = s.count;
    for (int q = 0; q < c_old; ++q) {
      const int sl = ((s.head - c_old + q) % m + m) % m;
      if (sl == slot) continue;
      s.SY[sl][slot] = D[LB_SYT + sl];
      s.YY[sl][slot] = D[LB_YYT + sl];
      s.YY[slot][sl] = D[LB_YYT + sl];
    }
    s.SY[slot][slot] = sy;
    s.YY[slot][slot] = yy;
    s.head = (slot + 1) % m;
    s.count = min(s.count + 1, m);
    s.gamma = sy / yy;
  }
  s.action = LB_ACCEPT_DIR;
  new_direction(s, ln, D);
}

}  // namespace

// the line search and the new direction of one lane on its state s (staged in
// LDS by k_lb_step) and the inner products D of this evaluation
template <typename T>
__device__ void lb_decide(LbState& s, const LbLane<T>& ln, const LbParams& prm, const double* D);

template <typename T>
__global__ __launch_bounds__(64) void k_lb_step(const LbLane<T>* lanes, LbParams prm) {
  const int L = blockIdx.x;
  const LbLane<T> ln = lanes[L];
  if (ln.state->phase == LB_DONE) {
    if (threadIdx.x == 0) {
      ln.state->action = LB_NONE;
      if (ln.done_flag) *ln.done_flag = 1;   // kept raised (tables may have been rebuilt)
    }
    return;
  }
  // the state moves to LDS with one load per word across the block, so that
  // the serial logic below waits on LDS rather than on a chain of global loads
  static_assert(sizeof(LbState) % 8 == 0, "LbState is copied in 8-byte words");
  constexpr int NW = (int)(sizeof(LbState) / 8);
  __shared__ LbState sh;
  for (int i = threadIdx.x; i < NW; i += 64)
    reinterpret_cast<uint64_t*>(&sh)[i] = gload(reinterpret_cast<const uint64_t*>(ln.state) + i);
  __shared__ double D[LB_ND];
  if (threadIdx.x < LB_ND) {
    const int i = threadIdx.x;
    double v = 0.0;
    // the chunk partials in order, eight loads in flight at a time (from
    // valid chunks; those past nb are not used)
    for (int b0 = 0; b0 < ln.nb; b0 += 8) {
      double pv[8];
#pragma unroll
      for (int h = 0; h < 8; ++h) pv[h] = gload(ln.part + (int64_t)min(b0 + h, ln.nb - 1) * LB_ND + i);
#pragma unroll
      for (int h = 0; h < 8; ++h)
        if (b0 + h < ln.nb) v = i == LB_MAXG ? fmax(v, pv[h]) : v + pv[h];
    }
    D[i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) lb_decide<T>(sh, ln, prm, D);
  __syncthreads();
  for (int i = threadIdx.x; i < NW; i += 64)
    gstore(reinterpret_cast<uint64_t*>(ln.state) + i, reinterpret_cast<const uint64_t*>(&sh)[i]);
}

template <typename T>
__device__ void lb_decide(LbState& s, const LbLane<T>& ln, const LbParams& prm, const double* D) {
  const double phi = ln.f_t[0] / ln.scale;
  const double gtd = D[LB_GTD];
  s.evals += 1;
  s.action = LB_NONE;

  if (s.phase == LB_START) {
    s.f = phi;
    if (ln.trace && ln.trace_len > 0) ln.trace[0] = phi * ln.scale;
    if (!(isfinite(phi) && isfinite(D[LB_GTGT]))) { finish(s, ln, prm, EX_NONFINITE, LB_RESTORE); return; }
    if (D[LB_MAXG] <= ln.pgtol) { finish(s, ln, prm, EX_PGTOL, LB_RESTORE); return; }
    if (s.evals >= ln.max_evals) { finish(s, ln, prm, EX_MAX_EVALS, LB_RESTORE); return; }
    s.count = 0;
    s.head = 0;
    s.store = 0;
    s.gamma = 1.0;
    s.coef_g = -1.0;
    s.dphi0 = -D[LB_GTGT];
    s.action = LB_START_DIR;
    begin_search(s, ln, fmin(1.0, 1.0 / sqrt(D[LB_GTGT])));
    return;
  }

  const bool fin = isfinite(phi) && isfinite(gtd);
  const double armijo = s.f + LB_C1 * s.a * s.dphi0;
  s.ls_evals += 1;
  bool to_zoom = false;
  if (s.phase == LB_BRACKET) {
    if (!fin || phi > armijo || (s.ls_i > 1 && phi >= s.f_prev)) {
      s.lo_a = s.a_prev; s.lo_f = s.f_prev; s.lo_d = s.d_prev;
      s.hi_a = s.a; s.hi_f = phi; s.hi_d = gtd; s.hi_fin = fin;
      to_zoom = true;
    } else if (fabs(gtd) <= -LB_C2 * s.dphi0) {
      accept(s, ln, prm, D, phi);
      return;
    } else if (gtd >= 0.0) {
      s.lo_a = s.a; s.lo_f = phi; s.lo_d = gtd;
      s.hi_a = s.a_prev; s.hi_f = s.f_prev; s.hi_d = s.d_prev; s.hi_fin = 1;
      to_zoom = true;
    } else {
      if (s.ls_evals >= s.ls_limit) {
        finish(s, ln, prm, s.evals >= ln.max_evals ? EX_MAX_EVALS : EX_LINESEARCH, LB_RESTORE);
        return;
      }
      s.a_prev = s.a; s.f_prev = phi; s.d_prev = gtd;
      s.a = fmin(2.0 * s.a, LB_STEP_MAX);
      s.ls_i += 1;
      s.action = LB_TRIAL;
      return;
    }
  } else {   // LB_ZOOM
    if (!fin || phi > armijo || phi >= s.lo_f) {
      s.hi_a = s.a; s.hi_f = phi; s.hi_d = gtd; s.hi_fin = fin;
    } else {
      if (fabs(gtd) <= -LB_C2 * s.dphi0) {
        accept(s, ln, prm, D, phi);
        return;
      }
      if (gtd * (s.hi_a - s.lo_a) >= 0.0) {
        s.hi_a = s.lo_a; s.hi_f = s.lo_f; s.hi_d = s.lo_d; s.hi_fin = 1;
      }
      s.lo_a = s.a; s.lo_f = phi; s.lo_d = gtd;
    }
    to_zoom = true;
  }
  if (to_zoom) {
    if (s.ls_evals >= s.ls_limit ||
        fabs(s.hi_a - s.lo_a) <= LB_COLLAPSE * fmax(fabs(s.lo_a), fabs(s.hi_a))) {
      finish(s, ln, prm, s.evals >= ln.max_evals ? EX_MAX_EVALS : EX_LINESEARCH, LB_RESTORE);
      return;
    }
    s.phase = LB_ZOOM;
    s.a = zoom_trial(s);
    s.action = LB_TRIAL;
  }
}

// ---------------------------------------------------------------------------
// k_lb_apply: carry out a lane's action elementwise and write its next trial
// point (or, when it has finished, its final point) into the evaluation inputs
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_lb_apply(const LbLane<T>* lanes, const LbItem* items) {
  int L = blockIdx.y, b = blockIdx.x;
  if (items) {
    const LbItem it = items[blockIdx.x];
    L = it.lane;
    b = it.blk;
  }
  const LbLane<T> ln = lanes[L];
  if (b >= ln.nb) return;
  const LbState& s = *ln.state;
  const int act = s.action;
  if (act == LB_NONE) return;
  const double a = s.a, a_acc = s.a_acc, coef_g = s.coef_g;
  const int cnt = s.count, store = s.store, slot = s.slot;
  double cs[LB_MMAX], cy[LB_MMAX];
#pragma unroll
  for (int i = 0; i < LB_MMAX; ++i) { cs[i] = s.cs[i]; cy[i] = s.cy[i]; }
  for (int k = 0; k < LB_CHUNK / 256; ++k) {
    const int64_t e = (int64_t)b * LB_CHUNK + k * 256 + threadIdx.x;
    if (e >= ln.N) break;
    double xe = gload(ln.x + e);
    double xt;
    if (act == LB_START_DIR) {
      const double gt = trial_grad(ln, e);
      gstore(ln.g + e, gt);
      gstore(ln.d + e, -gt);
      xt = xe + a * (-gt);
    } else if (act == LB_TRIAL) {
      xt = xe + a * gload(ln.d + e);
    } else if (act == LB_ACCEPT_DIR || act == LB_ACCEPT_FINAL) {
      const double de = gload(ln.d + e);
      const double gold = gload(ln.g + e);
      const double gt = trial_grad(ln, e);
      xe = xe + a_acc * de;
      gstore(ln.x + e, xe);
      gstore(ln.g + e, gt);
      if (act == LB_ACCEPT_FINAL) {
        xt = xe;
      } else {
        const double snew = a_acc * de, ynew = gt - gold;
        if (store) {
          gstore(ln.S + (int64_t)slot * ln.N + e, snew);
          gstore(ln.Y + (int64_t)slot * ln.N + e, ynew);
        }
        // every slot read (unused ones from a valid slot) before any is used
        double Sv[LB_MMAX], Yv[LB_MMAX];
#pragma unroll
        for (int q = 0; q < LB_MMAX; ++q) {
          const int64_t sq = q < cnt ? q : 0;
          Sv[q] = gload(ln.S + sq * ln.N + e);
          Yv[q] = gload(ln.Y + sq * ln.N + e);
        }
        double dn = coef_g * gt;
#pragma unroll
        for (int q = 0; q < LB_MMAX; ++q) {
          if (q < cnt) {
            const bool fresh = store && q == slot;
            const double Sq = fresh ? snew : Sv[q];
            const double Yq = fresh ? ynew : Yv[q];
            dn = fma(cs[q], Sq, fma(cy[q], Yq, dn));
          }
        }
        gstore(ln.d + e, dn);
        xt = xe + a * dn;
      }
    } else {   // LB_RESTORE
      xt = xe;
    }
    write_trial(ln, e, xt);
  }
}

// ---------------------------------------------------------------------------
// starts
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_init_gauss(const LbLane<T>* lanes) {
  const int L = blockIdx.y;
  const LbLane<T> ln = lanes[L];
  if ((int)blockIdx.x >= ln.nb) return;
  for (int k = 0; k < LB_CHUNK / 256; ++k) {
    const int64_t e = (int64_t)blockIdx.x * LB_CHUNK + k * 256 + threadIdx.x;
    if (e >= ln.N) break;
    double v = 1.0;
    if (e >= ln.r) {
      const int64_t q = e - ln.r, j = q / ln.ld, i = q - j * ln.ld;
      v = i < ln.n ? normal_at(ln.seed, (uint32_t)ln.restart, STREAM_GAUSS_A0, i + j * ln.n) : 0.0;
    }
    ln.x[e] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_given(const LbLane<T>* lanes) {
  const int L = blockIdx.y;
  const LbLane<T> ln = lanes[L];
  if ((int)blockIdx.x >= ln.nb) return;
  for (int k = 0; k < LB_CHUNK / 256; ++k) {
    const int64_t e = (int64_t)blockIdx.x * LB_CHUNK + k * 256 + threadIdx.x;
    if (e >= ln.N) break;
    double v = 1.0;
    if (e >= ln.r) {
      const int64_t q = e - ln.r, j = q / ln.ld, i = q - j * ln.ld;
      v = i < ln.n ? (double)ln.A0[i + j * ln.n] : 0.0;
    }
    ln.x[e] = v;
    write_trial(ln, e, v);
  }
}

namespace {
__device__ double block_sum(double v, double* sm) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sm[wave] = v;
  __syncthreads();
  const double t = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  __syncthreads();
  return t;
}
}  // namespace

// one block per (column, lane): unit column, lambda_j = 1, trial point = x
template <typename T>
__global__ __launch_bounds__(256) void k_norm_cols(const LbLane<T>* lanes) {
  __shared__ double sm[4];
  const int L = blockIdx.y, j = blockIdx.x;
  const LbLane<T> ln = lanes[L];
  if (j >= ln.r) return;
  double* col = ln.x + ln.r + (int64_t)j * ln.ld;
  double ss = 0.0;
  for (int i = threadIdx.x; i < ln.n; i += 256) ss = fma(col[i], col[i], ss);
  const double nrm = sqrt(block_sum(ss, sm));
  for (int i = threadIdx.x; i < ln.ld; i += 256) {
    const double v = i < ln.n ? col[i] / nrm : 0.0;
    col[i] = v;
    ln.A_t[(int64_t)j * ln.ld + i] = (T)v;
  }
  if (threadIdx.x == 0) {
    ln.x[j] = 1.0;
    ln.lam_t[j] = 1.0;
  }
}

// Omega of every restart in the packed layout of the second product:
// element (l, k r + j) = normal (l + p j) of (seed, k, stream 2)
template <typename T>
__global__ __launch_bounds__(256) void k_omega_packed(T* Wp, int64_t p, int r, int restarts, int nt_tot,
                                                      int64_t total, uint64_t seed) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int s = (int)(idx & 3);
  const int lane = (int)((idx >> 2) & 63);
  const int g = lane >> 4, c = lane & 15;
  const int64_t bt = idx >> 8;
  const int t = (int)(bt % nt_tot);
  const int64_t b = bt / nt_tot;
  const int64_t l = 16 * b + Mfma<T>::row(g, s);
  const int col = 16 * t + c;
  double v = 0.0;
  if (l < p && col < r * restarts) {
    const int k = col / r, j = col - k * r;
    v = normal_at(seed, (uint32_t)k, STREAM_RRF_OMEGA, l + p * (int64_t)j);
  }
  Wp[idx] = (T)v;
}

// one block per (column, lane): column (restart r + j) of V Omega from the
// split partials, normalised
template <typename T>
__global__ __launch_bounds__(256) void k_rrf_finish(const LbLane<T>* lanes, const T* Ypart, int64_t npad,
                                                    int64_t rp, int nsplit) {
  __shared__ double sm[4];
  const int L = blockIdx.y, j = blockIdx.x;
  const LbLane<T> ln = lanes[L];
  if (j >= ln.r) return;
  const int64_t colg = (int64_t)ln.restart * ln.r + j;
  double* col = ln.x + ln.r + (int64_t)j * ln.ld;
  double ss = 0.0;
  for (int i = threadIdx.x; i < ln.n; i += 256) {
    double y = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) y += (double)Ypart[((int64_t)sp * rp + colg) * npad + i];
    col[i] = y;
    ss = fma(y, y, ss);
  }
  const double nrm = sqrt(block_sum(ss, sm));
  for (int i = threadIdx.x; i < ln.ld; i += 256) {
    const double v = i < ln.n ? col[i] / nrm : 0.0;
    col[i] = v;
    ln.A_t[(int64_t)j * ln.ld + i] = (T)v;
  }
  if (threadIdx.x == 0) {
    ln.x[j] = 1.0;
    ln.lam_t[j] = 1.0;
  }
}

// grouped form: the partials of the lane's instance ([split][nt*16][ldy])
template <typename T>
__global__ __launch_bounds__(256) void k_grrf_finish(const LbLane<T>* lanes, const GInst<T>* insts) {
  __shared__ double sm[4];
  const int L = blockIdx.y, j = blockIdx.x;
  const LbLane<T> ln = lanes[L];
  if (j >= ln.r) return;
  const GInst<T>& I = insts[ln.inst];
  const int64_t colg = (int64_t)ln.restart * ln.r + j;
  const int64_t rp = (int64_t)I.nt * 16;
  const int nsplit = I.nsplit;
  const int64_t ldy = I.ldy;
  const T* Yp = I.Ypart;
  double* col = ln.x + ln.r + (int64_t)j * ln.ld;
  double ss = 0.0;
  for (int i = threadIdx.x; i < ln.n; i += 256) {
    double y = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) y += (double)Yp[((int64_t)sp * rp + colg) * ldy + i];
    col[i] = y;
    ss = fma(y, y, ss);
  }
  const double nrm = sqrt(block_sum(ss, sm));
  for (int i = threadIdx.x; i < ln.ld; i += 256) {
    const double v = i < ln.n ? col[i] / nrm : 0.0;
    col[i] = v;
    ln.A_t[(int64_t)j * ln.ld + i] = (T)v;
  }
  if (threadIdx.x == 0) {
    ln.x[j] = 1.0;
    ln.lam_t[j] = 1.0;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_lb_dots(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev, const LbItem* items,
                    int nitems) {
  if (items) {
    if (nitems > 0) hipLaunchKernelGGL(k_lb_dots<T>, dim3(nitems), dim3(256), 0, st, lanes_dev, items);
  } else {
    hipLaunchKernelGGL(k_lb_dots<T>, dim3(nbmax, lanes), dim3(256), 0, st, lanes_dev, items);
  }
}
template <typename T>
void launch_lb_step(int lanes, hipStream_t st, const LbLane<T>* lanes_dev, const LbParams& prm) {
  hipLaunchKernelGGL(k_lb_step<T>, dim3(lanes), dim3(64), 0, st, lanes_dev, prm);
}
template <typename T>
void launch_lb_apply(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev, const LbItem* items,
                     int nitems) {
  if (items) {
    if (nitems > 0) hipLaunchKernelGGL(k_lb_apply<T>, dim3(nitems), dim3(256), 0, st, lanes_dev, items);
  } else {
    hipLaunchKernelGGL(k_lb_apply<T>, dim3(nbmax, lanes), dim3(256), 0, st, lanes_dev, items);
  }
}
template <typename T>
void launch_init_gauss(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev) {
  hipLaunchKernelGGL(k_init_gauss<T>, dim3(nbmax, lanes), dim3(256), 0, st, lanes_dev);
}
template <typename T>
void launch_init_given(int nbmax, int lanes, hipStream_t st, const LbLane<T>* lanes_dev) {
  hipLaunchKernelGGL(k_init_given<T>, dim3(nbmax, lanes), dim3(256), 0, st, lanes_dev);
}
template <typename T>
void launch_norm_cols(int lanes, int r, hipStream_t st, const LbLane<T>* lanes_dev) {
  hipLaunchKernelGGL(k_norm_cols<T>, dim3(r, lanes), dim3(256), 0, st, lanes_dev);
}
template <typename T>
void launch_grrf_finish(int lanes, int rmax, hipStream_t st, const LbLane<T>* lanes_dev, const GInst<T>* insts) {
  hipLaunchKernelGGL(k_grrf_finish<T>, dim3(rmax, lanes), dim3(256), 0, st, lanes_dev, insts);
}
template <typename T>
void launch_omega_packed(dim3 grid, hipStream_t st, T* Wp, int64_t p, int r, int restarts, int nt_tot,
                         int64_t nblk, uint64_t seed) {
  const int64_t total = nblk * nt_tot * 256;
  hipLaunchKernelGGL(k_omega_packed<T>, grid, dim3(256), 0, st, Wp, p, r, restarts, nt_tot, total, seed);
}
template <typename T>
void launch_rrf_finish(int lanes, int r, hipStream_t st, const LbLane<T>* lanes_dev, const T* Ypart, int64_t npad,
                       int64_t rp, int nsplit) {
  hipLaunchKernelGGL(k_rrf_finish<T>, dim3(r, lanes), dim3(256), 0, st, lanes_dev, Ypart, npad, rp, nsplit);
}

#define SYMTD_LB_INST(T)                                                                                       \
  template void launch_lb_dots<T>(int, int, hipStream_t, const LbLane<T>*, const LbItem*, int);                \
  template void launch_lb_step<T>(int, hipStream_t, const LbLane<T>*, const LbParams&);                         \
  template void launch_lb_apply<T>(int, int, hipStream_t, const LbLane<T>*, const LbItem*, int);               \
  template void launch_init_gauss<T>(int, int, hipStream_t, const LbLane<T>*);                                  \
  template void launch_init_given<T>(int, int, hipStream_t, const LbLane<T>*);                                  \
  template void launch_norm_cols<T>(int, int, hipStream_t, const LbLane<T>*);                                   \
  template void launch_grrf_finish<T>(int, int, hipStream_t, const LbLane<T>*, const GInst<T>*);                 \
  template void launch_omega_packed<T>(dim3, hipStream_t, T*, int64_t, int, int, int, int64_t, uint64_t);      \
  template void launch_rrf_finish<T>(int, int, hipStream_t, const LbLane<T>*, const T*, int64_t, int64_t, int);
SYMTD_LB_INST(float)
SYMTD_LB_INST(double)

}  // namespace symtd

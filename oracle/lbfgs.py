"""Reference L-BFGS driver (fp64, host) for the decomposition (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4 of the paper minimises f over (lambda, A) with L-BFGS-B (memory
m = 5, no active bounds, default options, limits on iterations and on
function/gradient evaluations, and a gradient tolerance pgtol).  With no
bounds that is unconstrained L-BFGS; the paper does not state the line
search, so this package takes the following reading, which the device solver
implements as well:

Direction (limited-memory BFGS, Nocedal & Wright, Numerical Optimization,
Alg. 7.4 - the two-loop recursion): d = -H g with H the inverse-Hessian
approximation built from the last m pairs (s_i, y_i) starting from
H0 = gamma I, gamma = s'y / y'y of the newest pair.  A pair is stored only if
s'y > 1e-10 y'y.  The first direction, and any direction that is not a
descent direction, is -g (memory cleared).

Line search (strong Wolfe, Nocedal & Wright Alg. 3.5 with zoom Alg. 3.6),
with c1 = 1e-3, c2 = 0.9, phi(a) = f(x + a d):
  * first trial a = min(1, 1/||g||_2) for a steepest-descent direction,
    a = 1 otherwise;
  * bracketing: a trial fails the sufficient-decrease test (or is not finite,
    or, after the first trial, phi(a) >= phi(previous trial)) -> zoom on
    (previous, a); it satisfies |phi'(a)| <= -c2 phi'(0) -> accept;
    phi'(a) >= 0 -> zoom on (a, previous); otherwise the next trial is
    min(2a, 1e10);
  * zoom keeps (lo, hi) with phi(lo) the lowest sufficient-decrease value seen;
    the trial is the minimiser of the cubic through (lo, phi, phi') and
    (hi, phi, phi') (Nocedal & Wright eq. (3.59)), replaced by the midpoint
    when it is not finite, when hi's values are not finite, or when it lies
    outside the middle 80% of the interval;
  * at most 20 evaluations per line search, and an interval shorter than
    1e-14 max(lo, hi) ends it; either ends the solve (LINESEARCH) at the last
    accepted point.

Stopping, tested after every accepted step (and pgtol at the start):
||g||_inf <= pgtol (PGTOL); f_k - f_{k+1} <= ftol max(|f_k|, |f_{k+1}|, 1)
(FTOL, L-BFGS-B's relative-reduction test); accepted steps >= max_iters
(MAX_ITERS); after any evaluation, evaluations >= max_evals (MAX_EVALS).  A
non-finite value at the starting point ends the solve (NONFINITE).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# exit reasons (same numeric codes as the library's symtd_exit enum)
RUNNING, PGTOL, FTOL, MAX_ITERS, MAX_EVALS, LINESEARCH, NONFINITE = 0, 1, 2, 3, 4, 5, 6
REASONS = {PGTOL: "PGTOL", FTOL: "FTOL", MAX_ITERS: "MAX_ITERS", MAX_EVALS: "MAX_EVALS",
           LINESEARCH: "LINESEARCH", NONFINITE: "NONFINITE"}

C1 = 1e-3
C2 = 0.9
MAXLS = 20
STEP_MAX = 1e10
SKIP_TOL = 1e-10
COLLAPSE = 1e-14


@dataclass
class LbResult:
    x: np.ndarray
    f: float
    g: np.ndarray
    iters: int
    evals: int
    reason: int
    f_hist: list = field(default_factory=list)     # f at the start and after every accepted step
    steps: list = field(default_factory=list)      # accepted step lengths


def two_loop(g, S, Y, gamma):
    """H g for the L-BFGS inverse Hessian of the pairs S[i], Y[i] (oldest first), H0 = gamma I."""
    q = np.array(g, dtype=np.float64, copy=True)
    k = len(S)
    rho = [1.0 / float(Y[i] @ S[i]) for i in range(k)]
    a = [0.0] * k
    for i in range(k - 1, -1, -1):
        a[i] = rho[i] * float(S[i] @ q)
        q -= a[i] * Y[i]
    r = gamma * q
    for i in range(k):
        b = rho[i] * float(Y[i] @ r)
        r += (a[i] - b) * S[i]
    return r


def cubic_min(a, fa, da, b, fb, db):
    """Minimiser of the cubic with values/slopes (fa, da) at a and (fb, db) at b (eq. (3.59)), or None."""
    d1 = da + db - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - da * db
    if not np.isfinite(disc) or disc < 0.0:
        return None
    d2 = np.copysign(np.sqrt(disc), b - a)
    den = db - da + 2.0 * d2
    if den == 0.0 or not np.isfinite(den):
        return None
    t = b - (b - a) * (db + d2 - d1) / den
    return t if np.isfinite(t) else None


def zoom_trial(lo, hi):
    """Next zoom trial from lo = (a, phi, dphi) and hi = (a, phi, dphi, finite)."""
    a_lo, a_hi = lo[0], hi[0]
    left, right = min(a_lo, a_hi), max(a_lo, a_hi)
    width = right - left
    mid = 0.5 * (a_lo + a_hi)
    if not hi[3]:
        return mid
    t = cubic_min(a_lo, lo[1], lo[2], a_hi, hi[1], hi[2])
    if t is None or t < left + 0.1 * width or t > right - 0.1 * width:
        return mid
    return t


def line_search(phi, f0, dphi0, a1, limit=MAXLS):
    """Strong-Wolfe line search of the reading above.

    phi(a) -> (value, slope, payload).  At most `limit` evaluations.  Returns
    (a, value, payload, evals) on success, or (None, None, None, evals) on
    failure.
    """
    evals = 0
    a_prev, f_prev, d_prev = 0.0, f0, dphi0
    a = a1
    i = 1
    # bracketing
    while True:
        fa, da, pay = phi(a)
        evals += 1
        fin = bool(np.isfinite(fa) and np.isfinite(da))
        if (not fin) or fa > f0 + C1 * a * dphi0 or (i > 1 and fa >= f_prev):
            lo, hi = (a_prev, f_prev, d_prev), (a, fa, da, fin)
            break
        if abs(da) <= -C2 * dphi0:
            return a, fa, pay, evals
        if da >= 0.0:
            lo, hi = (a, fa, da), (a_prev, f_prev, d_prev, True)
            break
        if evals >= limit:
            return None, None, None, evals
        a_prev, f_prev, d_prev = a, fa, da
        a = min(2.0 * a, STEP_MAX)
        i += 1
    # zoom
    while True:
        if evals >= limit or abs(hi[0] - lo[0]) <= COLLAPSE * max(abs(lo[0]), abs(hi[0])):
            return None, None, None, evals
        a = zoom_trial(lo, hi)
        fa, da, pay = phi(a)
        evals += 1
        fin = bool(np.isfinite(fa) and np.isfinite(da))
        if (not fin) or fa > f0 + C1 * a * dphi0 or fa >= lo[1]:
            hi = (a, fa, da, fin)
        else:
            if abs(da) <= -C2 * dphi0:
                return a, fa, pay, evals
            if da * (hi[0] - lo[0]) >= 0.0:
                hi = (lo[0], lo[1], lo[2], True)
            lo = (a, fa, da)


def lbfgs(fun, x0, m=5, pgtol=1e-5, ftol=2.220446049250313e-09, max_iters=10000, max_evals=50000):
    """Minimise fun(x) -> (f, g) from x0 with the L-BFGS reading above."""
    x = np.array(x0, dtype=np.float64, copy=True)
    f, g = fun(x)
    evals = 1
    hist = [f]
    steps = []
    if not (np.isfinite(f) and np.all(np.isfinite(g))):
        return LbResult(x, f, g, 0, evals, NONFINITE, hist, steps)
    if np.max(np.abs(g)) <= pgtol:
        return LbResult(x, f, g, 0, evals, PGTOL, hist, steps)
    S, Y = [], []
    gamma = 1.0
    iters = 0
    while True:
        if S:
            d = -two_loop(g, S, Y, gamma)
            dphi0 = float(g @ d)
            first = False
            if not (np.isfinite(dphi0) and dphi0 < 0.0):
                S, Y = [], []
                first = True
        else:
            first = True
        if first:
            d = -g
            dphi0 = -float(g @ g)
        a1 = min(1.0, 1.0 / np.sqrt(-dphi0)) if first else 1.0

        def phi(a):
            xt = x + a * d
            ft, gt = fun(xt)
            return ft, float(gt @ d), gt

        a, ft, gt, used = line_search(phi, f, dphi0, a1, min(MAXLS, max_evals - evals))
        evals += used
        if a is None:
            return LbResult(x, f, g, iters, evals, MAX_EVALS if evals >= max_evals else LINESEARCH, hist, steps)
        xn = x + a * d
        s = a * d
        yv = gt - g
        sy = float(s @ yv)
        yy = float(yv @ yv)
        if sy > SKIP_TOL * yy:
            S.append(s)
            Y.append(yv)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
            gamma = sy / yy
        f_old = f
        x, f, g = xn, ft, gt
        iters += 1
        hist.append(f)
        steps.append(a)
        if np.max(np.abs(g)) <= pgtol:
            return LbResult(x, f, g, iters, evals, PGTOL, hist, steps)
        if f_old - f <= ftol * max(abs(f_old), abs(f), 1.0):
            return LbResult(x, f, g, iters, evals, FTOL, hist, steps)
        if iters >= max_iters:
            return LbResult(x, f, g, iters, evals, MAX_ITERS, hist, steps)
        if evals >= max_evals:
            return LbResult(x, f, g, iters, evals, MAX_EVALS, hist, steps)

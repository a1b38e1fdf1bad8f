"""FP64 oracle of the bounded limited-memory quasi-Newton fit (L-BFGS-B).

TEST INFRASTRUCTURE ONLY (see ``oracle/salt64.py``): imported by ``tests/``
and the ``cpu_baseline`` leg of ``bench.py``, never by the library, and shares
no code with it.

The paper's optimisation example fits the free SALT parameters with a bounded
quasi-Newton method, L-BFGS-B (section "Implementation", the example
scripts).  The algorithm is the one of Byrd, Lu, Nocedal and Zhu, "A limited
memory algorithm for bound constrained optimization", SIAM J. Sci. Comput. 16
(1995) 1190-1208 (BLNZ below), restated here step by step for a problem of n
variables with bounds l <= x <= u:

1. The quasi-Newton matrix (BLNZ section 3): B = theta I updated by the BFGS
   formula with the stored correction pairs (s_i, y_i), oldest first.  BLNZ
   keep B in the compact form theta I - W M W^T (Byrd, Nocedal and Schnabel
   1994), which is the same matrix; with n = 4 the dense form is the plain one.
   theta = y^T y / s^T y of the newest pair (1 with no pair).
2. The generalized Cauchy point (BLNZ section 4): along the projected
   steepest-descent path x(t) = P(x - t g) the quadratic model
   m(x) = f + g^T (x - x_k) + (x - x_k)^T B (x - x_k) / 2 is piecewise
   quadratic between the breakpoints where a variable reaches a bound; the
   segments are examined in order and x^c is the first local minimiser.
3. Subspace minimisation (BLNZ section 5.1, direct primal method): with the
   variables at bounds in x^c held, the model is minimised over the others from
   x^c, and the step is cut back to the largest multiple (at most 1) that stays
   feasible, giving xbar.
4. The line search (BLNZ section 6) along d = xbar - x_k with step at most the
   largest feasible one, first trial step min(1/||d||, max) at the first
   iteration and min(1, max) afterwards, ends at a step satisfying the
   sufficient-decrease and curvature conditions f(x + a d) <= f + ftol a g^T d
   and |g(x + a d)^T d| <= gtol |g^T d|, ftol = 1e-3, gtol = 0.9.
5. The new pair s = x_{k+1} - x_k, y = g_{k+1} - g_k is kept only if
   s^T y > eps y^T y (eps the machine epsilon); at most m pairs are kept.

Readings where BLNZ leave a choice (listed with the design notes):

* The line search is a bracketing search with safeguarded cubic
  interpolation (the strong-Wolfe search of Nocedal and Wright, Numerical
  Optimization, 2006, algorithms 3.5 and 3.6), not the Fortran routine of
  More and Thuente that BLNZ call; it enforces the same two conditions.  A
  step that reaches the largest feasible step with the sufficient decrease
  holding ends the search there.  After MAX_LS trials without an acceptable
  step, or for a direction that is not a descent direction, the pairs are
  dropped and the iteration starts again from steepest descent (BLNZ
  section 6, restart).
* The budget is a number of function-and-gradient evaluations after the one
  at the start (the fit's iteration count), not a convergence test; a zero
  projected gradient (x^c = x and xbar = x) ends the fit early.
"""
from __future__ import annotations

import numpy as np

FTOL = 1e-3
GTOL = 0.9
MAX_LS = 20
EPS64 = np.finfo(np.float64).eps


def bfgs_matrix(pairs, theta, n):
    """B = theta I updated by BFGS with the pairs (s, y), oldest first (BLNZ section 3)."""
    B = theta * np.eye(n)
    for s, y in pairs:
        Bs = B @ s
        B = B - np.outer(Bs, Bs) / (s @ Bs) + np.outer(y, y) / (y @ s)
    return B


def breakpoints(x, g, l, u):
    """t_i at which variable i of the path P(x - t g) reaches its bound (inf if never)."""
    t = np.full(len(x), np.inf)
    neg, pos = g < 0, g > 0
    t[neg] = (x[neg] - u[neg]) / g[neg]
    t[pos] = (x[pos] - l[pos]) / g[pos]
    return t


def cauchy_point(x, g, l, u, B):
    """Generalized Cauchy point x^c of the quadratic model along the projected gradient path,
    examining the segments between breakpoints in increasing order (BLNZ section 4)."""
    n = len(x)
    tb = breakpoints(x, g, l, u)
    d = np.where(tb > 0, -g, 0.0)
    xc = x.copy()
    z = np.zeros(n)                     # x(t_old) - x
    order = [i for i in np.argsort(tb, kind="stable") if tb[i] > 0 and np.isfinite(tb[i])]
    t_old = 0.0
    for b in order:
        fp = g @ d + d @ B @ z          # slope of the model at the segment start
        fpp = d @ B @ d                 # curvature along the segment
        if fp >= 0.0:                   # the model rises from here: x(t_old) is the minimiser
            return x + z
        dt = tb[b] - t_old
        dt_min = -fp / fpp if fpp > 0 else np.inf
        if dt_min < dt:                 # the minimiser lies inside this segment
            return x + z + dt_min * d
        # move to the breakpoint; variable b reaches its bound and is held from here on
        z = z + dt * d
        z[b] = (u[b] if d[b] > 0 else l[b]) - x[b]
        d[b] = 0.0
        t_old = tb[b]
    # past the last finite breakpoint: the free direction continues without bound
    fp = g @ d + d @ B @ z
    fpp = d @ B @ d
    if fp >= 0.0 or not np.any(d != 0.0):
        return x + z
    dt_min = -fp / fpp if fpp > 0 else 0.0
    xc = x + z + dt_min * d
    return xc


def subspace_min(x, g, l, u, B, xc):
    """Direct primal subspace minimisation from x^c over the variables not at a bound, truncated
    to the feasible region (BLNZ section 5.1).  Returns xbar."""
    free = (xc > l) & (xc < u)
    if not np.any(free):
        return xc.copy()
    r = g + B @ (xc - x)                # gradient of the model at x^c
    F = np.flatnonzero(free)
    dF = np.linalg.solve(B[np.ix_(F, F)], -r[F])
    alpha = 1.0
    for k, i in enumerate(F):
        if dF[k] > 0:
            alpha = min(alpha, (u[i] - xc[i]) / dF[k])
        elif dF[k] < 0:
            alpha = min(alpha, (l[i] - xc[i]) / dF[k])
    xbar = xc.copy()
    xbar[F] = xc[F] + alpha * dF
    return xbar


def max_step(x, d, l, u):
    """Largest a with l <= x + a d <= u (inf if d points nowhere bounded)."""
    a = np.inf
    for i in range(len(x)):
        if d[i] > 0:
            a = min(a, (u[i] - x[i]) / d[i])
        elif d[i] < 0:
            a = min(a, (l[i] - x[i]) / d[i])
    return a


def cubic_step(a, fa, ga, b, fb, gb):
    """Minimiser of the cubic through (a, fa, ga) and (b, fb, gb), kept inside the interval
    [lo + 0.1 w, hi - 0.1 w] of width w; the midpoint if the cubic has no minimiser."""
    lo, hi = min(a, b), max(a, b)
    w = hi - lo
    d1 = ga + gb - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - ga * gb
    if disc < 0.0:
        return 0.5 * (a + b)
    d2 = np.copysign(np.sqrt(disc), b - a)
    den = gb - ga + 2.0 * d2
    if den == 0.0:
        return 0.5 * (a + b)
    x = b - (b - a) * (gb + d2 - d1) / den
    return min(max(x, lo + 0.1 * w), hi - 0.1 * w)


def lbfgsb(fun, x0, lower, upper, m=5, max_evals=50, eps=EPS64):
    """Minimise fun (x -> (f, g)) from x0 within [lower, upper] with at most max_evals
    evaluations after the one at x0.  Returns dict(x, f, g, evals, n_iter, history, pairs)."""
    l = np.asarray(lower, np.float64)
    u = np.asarray(upper, np.float64)
    x = np.clip(np.asarray(x0, np.float64), l, u)
    n = len(x)
    f, g = fun(x)
    pairs = []
    evals = 0
    n_iter = 0
    history = [f]
    first = True
    while evals < max_evals:
        theta = 1.0 if not pairs else (pairs[-1][1] @ pairs[-1][1]) / (pairs[-1][0] @ pairs[-1][1])
        B = bfgs_matrix(pairs, theta, n)
        xc = cauchy_point(x, g, l, u, B)
        xbar = subspace_min(x, g, l, u, B, xc)
        d = xbar - x
        gd = g @ d
        if not np.any(d != 0.0):
            break                         # projected gradient zero: x is stationary
        if not gd < 0.0:
            if pairs:
                pairs = []                # not a descent direction: restart from steepest descent
                continue
            break
        amax = max_step(x, d, l, u)
        a = min(1.0 / np.linalg.norm(d), amax) if first else min(1.0, amax)
        # line search: lo holds the best step with sufficient decrease so far
        a_lo, f_lo, g_lo = 0.0, f, gd
        hi = None
        accepted = None
        trials = 0
        while evals < max_evals and trials < MAX_LS:
            ft, gt = fun(np.clip(x + a * d, l, u))
            evals += 1
            trials += 1
            dt = gt @ d
            if not np.isfinite(ft) or ft > f + FTOL * a * gd or ft >= f_lo:
                hi = (a, ft if np.isfinite(ft) else np.inf, dt if np.isfinite(dt) else 0.0)
            elif abs(dt) <= -GTOL * gd:
                accepted = (a, ft, gt)
                break
            else:
                # the new point is the best so far; the minimiser lies on the side its slope
                # points down to: the previous best becomes the other end if it lies there
                if (hi is None and dt >= 0.0) or (hi is not None and dt * (hi[0] - a_lo) >= 0.0):
                    hi = (a_lo, f_lo, g_lo)
                a_lo, f_lo, g_lo = a, ft, dt
                if hi is None and a >= amax:
                    accepted = (a, ft, gt)    # the largest feasible step, with sufficient decrease
                    break
            if hi is None:
                a = min(4.0 * a_lo, amax)
            elif not np.isfinite(hi[1]):
                a = a_lo + 0.5 * (hi[0] - a_lo)
            else:
                a = cubic_step(a_lo, f_lo, g_lo, hi[0], hi[1], hi[2])
        if accepted is None:
            if pairs and evals < max_evals:
                pairs = []                    # line search failed: restart from steepest descent
                first = True
                continue
            break
        a, ft, gt = accepted
        xn = np.clip(x + a * d, l, u)
        s, y = xn - x, gt - g
        if s @ y > eps * (y @ y):
            pairs.append((s, y))
            if len(pairs) > m:
                pairs.pop(0)
        x, f, g = xn, ft, gt
        history.append(f)
        n_iter += 1
        first = False
    return dict(x=x, f=f, g=g, evals=evals, n_iter=n_iter, history=history, pairs=pairs)

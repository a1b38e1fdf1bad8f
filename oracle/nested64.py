"""FP64 oracle of the nested-sampling driver (the paper's nested-sampling example).

TEST INFRASTRUCTURE ONLY (see ``oracle/salt64.py``): imported by ``tests/`` and the
``cpu_baseline`` leg of ``bench.py``, never by the library, and shares no code with it.

The paper's second example script samples the SALT parameters' posterior by nested
sampling (section "Implementation", the example scripts).  The method is Skilling's
(Bayesian Analysis 1, 2006, 833-860), restated here:

* N live points drawn from the prior; each iteration the live point of lowest
  likelihood L* becomes a dead point with prior mass X_i = exp(-i/N) (the expected
  shrinkage), weight w_i = X_{i-1} - X_i, and is replaced by a draw from the prior
  restricted to L > L*;
* Z = sum_i L_i w_i, accumulated in logs, with the information
  H = sum_i (L_i w_i / Z) ln(L_i / Z) and the error estimate sqrt(H / N);
* the run stops after max_iter dead points, or when the live points can add no more
  than a factor exp(dlogz) to Z (ln(Z + L_max X_i) - ln Z < dlogz); the live points
  then join the sum with weights X_final / N each.

Readings (listed with the design notes):

* Priors are independent per parameter (z, t0, x0, x1, c): fixed, uniform on
  [a, b], or log-uniform on [a, b]; the prior transform maps a point u of the unit
  cube to the parameters.
* The constrained draw is rejection sampling from the prior inside an enlarged box
  around the live points in the unit cube: the box spans each coordinate's live
  range, widened about its centre by the factor ``enlarge`` and clipped to [0, 1].
  Candidates are drawn and evaluated in batches; those above the current L* are kept
  in draw order and used, for the following iterations too, while they stay above
  the rising threshold; a batch is drawn only when none is left (a candidate above a
  later L* is a draw from the prior restricted to that higher contour, which the
  earlier box contains).
* The random numbers are Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC11, 2011):
  coordinate d of draw n is output d mod 4 of the block with counter (n, d div 4, 0, 0)
  and key (seed, KEY1), mapped to ((x >> 11) + 1/2) 2^-53 in (0, 1).  Draws 0..N-1
  are the initial live points, from the whole unit cube.
* Ties of L* go to the lowest live index.
"""
from __future__ import annotations

from collections import deque

import numpy as np

KEY1 = 0x5A17BF1A5A17BF1A      # second key word of the draws' generator
_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1

FIXED, UNIFORM, LOG_UNIFORM = 0, 1, 2


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds: counter of four 64-bit words, key of two."""
    x = [int(v) & _MASK for v in ctr]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for _ in range(10):
        p0 = _M0 * x[0]
        p1 = _M1 * x[2]
        x = [(p1 >> 64) ^ x[1] ^ k0, p1 & _MASK, (p0 >> 64) ^ x[3] ^ k1, p0 & _MASK]
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return x


def unit_draws(seed, first, n):
    """Points first .. first+n-1 of the unit-cube stream: [n, 5] in (0, 1)."""
    out = np.empty((n, 5))
    for i in range(n):
        blk0 = philox4x64_10((first + i, 0, 0, 0), (seed, KEY1))
        blk1 = philox4x64_10((first + i, 1, 0, 0), (seed, KEY1))
        words = blk0 + blk1[:1]
        out[i] = [((w >> 11) + 0.5) * 2.0 ** -53 for w in words]
    return out


def prior_transform(u, priors):
    """Parameters (z, t0, x0, x1, c) of unit-cube points u [n, 5]; priors: five (kind, a, b)."""
    u = np.atleast_2d(u)
    th = np.empty_like(u)
    for d, (kind, a, b) in enumerate(priors):
        if kind == FIXED:
            th[:, d] = a
        elif kind == UNIFORM:
            th[:, d] = a + (b - a) * u[:, d]
        elif kind == LOG_UNIFORM:
            th[:, d] = np.exp(np.log(a) + (np.log(b) - np.log(a)) * u[:, d])
        else:
            raise ValueError("unknown prior kind")
    return th


def _finite_or_minus_inf(ll):
    """ln L with NaN (a sample the model cannot evaluate) as -inf: never above any threshold."""
    ll = np.asarray(ll, np.float64)
    return np.where(np.isnan(ll), -np.inf, ll)


def nested_sampling(loglike, priors, n_live=400, batch=1024, max_iter=100000, dlogz=0.01, enlarge=1.5, seed=1,
                    max_evals=50_000_000):
    """loglike: parameters [n, 5] -> ln L [n].  Returns dict(logz, logz_err, information, n_iter, n_eval,
    dead_theta, dead_logl, dead_logw, dead_draw, dead_margin (each iteration's decision margin, above),
    live_theta, live_logl, live_logw)."""
    u_live = unit_draws(seed, 0, n_live)
    th_live = prior_transform(u_live, priors)
    l_live = _finite_or_minus_inf(loglike(th_live))
    d_live = np.arange(n_live)
    n_draw = n_live
    n_eval = n_live
    logz, H, logx = -np.inf, 0.0, 0.0
    log_shrink = np.log(-np.expm1(-1.0 / n_live))      # ln(1 - e^{-1/N})
    dead = {"theta": [], "logl": [], "logw": [], "draw": [], "margin": []}
    pool = deque()
    n_iter = 0
    while n_iter < max_iter:
        if np.isfinite(logz) and np.logaddexp(logz, l_live.max() + logx) - logz < dlogz:
            break
        worst = int(np.argmin(l_live))
        lstar = l_live[worst]
        # the decision margin of this iteration: how far the retired point lies below the next live
        # point, and every candidate examined below from the threshold (a run in lower precision can
        # take a different decision only where this is within its rounding)
        two = np.partition(l_live, 1)[:2] if n_live > 1 else np.array([lstar, np.inf])
        margin = two[1] - two[0]
        logw = logx + log_shrink
        lz_new = np.logaddexp(logz, lstar + logw)
        H = (np.exp(lstar + logw - lz_new) * lstar
             + (np.exp(logz - lz_new) * (H + logz) if np.isfinite(logz) else 0.0) - lz_new)
        logz = lz_new
        dead["theta"].append(th_live[worst].copy())
        dead["logl"].append(lstar)
        dead["logw"].append(logw)
        dead["draw"].append(int(d_live[worst]))
        logx -= 1.0 / n_live
        n_iter += 1
        # replacement: the first kept candidate above L*, refilling the pool when it runs dry
        while True:
            while pool and not pool[0][2] > lstar:
                margin = min(margin, abs(pool[0][2] - lstar))
                pool.popleft()
            if pool:
                margin = min(margin, abs(pool[0][2] - lstar))
                break
            if n_eval >= max_evals:
                dead["margin"].append(margin)
                return _finish(dead, th_live, l_live, logz, H, logx, n_live, n_iter, n_eval, stopped=True)
            lo = u_live.min(axis=0)
            hi = u_live.max(axis=0)
            c, h = 0.5 * (lo + hi), 0.5 * (hi - lo) * enlarge
            lo, hi = np.maximum(c - h, 0.0), np.minimum(c + h, 1.0)
            u = lo + (hi - lo) * unit_draws(seed, n_draw, batch)
            th = prior_transform(u, priors)
            ll = _finite_or_minus_inf(loglike(th))
            if np.any(np.isfinite(ll)):
                margin = min(margin, float(np.min(np.abs(ll[np.isfinite(ll)] - lstar))))
            for k in range(batch):
                if ll[k] > lstar:
                    pool.append((u[k], th[k], ll[k], n_draw + k))
            n_draw += batch
            n_eval += batch
        uk, tk, lk, dk = pool.popleft()
        u_live[worst], th_live[worst], l_live[worst], d_live[worst] = uk, tk, lk, dk
        dead["margin"].append(margin)
    return _finish(dead, th_live, l_live, logz, H, logx, n_live, n_iter, n_eval, stopped=False)


def _finish(dead, th_live, l_live, logz, H, logx, n_live, n_iter, n_eval, stopped):
    """Adds the live points with weights X_final / N each to the evidence and the information."""
    logw_live = logx - np.log(n_live)
    for lj in l_live:
        lz_new = np.logaddexp(logz, lj + logw_live)
        H = (np.exp(lj + logw_live - lz_new) * lj
             + (np.exp(logz - lz_new) * (H + logz) if np.isfinite(logz) else 0.0) - lz_new)
        logz = lz_new
    return dict(logz=logz, logz_err=np.sqrt(max(H, 0.0) / n_live), information=H, n_iter=n_iter, n_eval=n_eval,
                stopped_on_evals=stopped,
                dead_theta=np.array(dead["theta"]).reshape(-1, 5), dead_logl=np.array(dead["logl"]),
                dead_logw=np.array(dead["logw"]), dead_draw=np.array(dead["draw"], np.int64),
                dead_margin=np.array(dead["margin"]),
                live_theta=th_live.copy(), live_logl=l_live.copy(), live_logw=np.full(n_live, logw_live))

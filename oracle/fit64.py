"""FP64 oracle of the light-curve fits served by the library.

TEST INFRASTRUCTURE ONLY (see ``oracle/salt64.py``).

The paper's example drivers fit the free SALT parameters x0, x1, t0, c of one
supernova to its photometry by gradient-based optimisation (section
"Implementation", the two example scripts).  The served fit is a
Levenberg-Marquardt damped Gauss-Newton iteration, written here step by step:

* unknowns q = (t0, ln x0, x1, c); z is given and held fixed;
* residuals r_i = d_i - f_i(q), weights W_i = 1/sigma_i^2, chi2 = sum W r^2;
* H = J^T W J and g = J^T W r with J = d f / d q, where d f/d ln x0 = x0 d f/d x0;
* each iteration solves (H + lambda diag(H)) delta = g by Cholesky, evaluates
  the trial q + delta, accepts it when its chi2 is finite and strictly smaller
  (lambda /= 10), otherwise keeps q (lambda *= 10); a non-positive Cholesky
  pivot counts as a rejected step; lambda stays within [1e-9, 1e9];
* exactly ``iters`` iterations (default 50) after the evaluation at the
  starting point, lambda starts at 1e-3;
* a subset of the four parameters may be held at its starting value: the
  damped system is then the one of the free parameters alone (the rows and
  columns of H and the entries of g that belong to them).

The second solver is the bounded quasi-Newton method of the paper's
optimisation example, L-BFGS-B (``oracle/lbfgsb64.py``), on the same unknowns
and objective chi2(q) with gradient -2 J^T W r, bounds on (t0, x0, x1, c)
(x0's taken to ln x0), a held parameter being one whose lower and upper bounds
equal its start, and the same budget: ``iters`` evaluations after the start.
"""
from __future__ import annotations

import numpy as np

from .lbfgsb64 import lbfgsb
from .salt64 import Oracle

LAMBDA_MIN, LAMBDA_MAX = 1e-9, 1e9


def _cholesky_solve4(A, b):
    """Solve A x = b for a symmetric n x n A (n <= 4) by Cholesky; None if a pivot is not positive."""
    n = len(b)
    L = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            s = A[i, j] - np.dot(L[i, :j], L[j, :j])
            if i == j:
                if not (s > 0.0) or not np.isfinite(s):
                    return None
                L[i, i] = np.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (b[i] - np.dot(L[i, :i], y[:i])) / L[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (y[i] - np.dot(L[i + 1:, i], x[i + 1:])) / L[i, i]
    return x


class FitOracle:
    def __init__(self, oracle: Oracle):
        self.o = oracle

    def evaluate(self, batch, z, q, data, inv_sigma2):
        """chi2, H (4x4) and g (4) at q = (t0, ln x0, x1, c) for a one-supernova batch."""
        t0, lnx0, x1, c = q
        x0 = np.exp(lnx0)
        f, J5 = self.o.jac(batch, params=np.array([[z, t0, x0, x1, c]]))
        J = np.stack([J5[:, 1], x0 * J5[:, 2], J5[:, 3], J5[:, 4]], axis=1)
        r = np.asarray(data, np.float64) - f
        w = np.asarray(inv_sigma2, np.float64)
        chi2 = float(np.sum(w * r * r))
        H = J.T @ (w[:, None] * J)
        g = J.T @ (w * r)
        return chi2, H, g

    def fit(self, batch, z, theta0, data, inv_sigma2, iters=50, lambda0=1e-3, free=(True, True, True, True)):
        """LM fit from theta0 = (t0, x0, x1, c), varying the parameters whose ``free`` flag is set.
        Returns dict(theta, chi2, n_accept, status)."""
        t0, x0, x1, c = [float(v) for v in theta0]
        fr = np.flatnonzero(np.asarray(free, bool))
        q = np.array([t0, np.log(x0), x1, c])
        chi2, H, g = self.evaluate(batch, z, q, data, inv_sigma2)
        if not np.isfinite(chi2):
            return dict(theta=np.array([t0, x0, x1, c]), chi2=chi2, n_accept=0, status="diverged")
        lam = lambda0
        n_acc = 0
        for _ in range(iters):
            Hf = H[np.ix_(fr, fr)]
            A = Hf + lam * np.diag(np.diag(Hf))
            delta = _cholesky_solve4(A, g[fr])
            if delta is None:
                lam = min(lam * 10.0, LAMBDA_MAX)
                continue
            qt = q.copy()
            qt[fr] += delta
            chi2_t, H_t, g_t = self.evaluate(batch, z, qt, data, inv_sigma2)
            if np.isfinite(chi2_t) and chi2_t < chi2:
                q, chi2, H, g = qt, chi2_t, H_t, g_t
                lam = max(lam * 0.1, LAMBDA_MIN)
                n_acc += 1
            else:
                lam = min(lam * 10.0, LAMBDA_MAX)
        theta = np.array([q[0], np.exp(q[1]), q[2], q[3]])
        return dict(theta=theta, chi2=chi2, n_accept=n_acc, status="ok")


    def fit_lbfgsb(self, batch, z, theta0, data, inv_sigma2, lower=None, upper=None, iters=50, m=5,
                   free=(True, True, True, True)):
        """L-BFGS-B fit from theta0 = (t0, x0, x1, c) within bounds on (t0, x0, x1, c) (None: none;
        x0's bounds apply to ln x0, a lower bound <= 0 meaning none).  Returns dict(theta, chi2,
        n_accept, evals, status)."""
        t0, x0, x1, c = [float(v) for v in theta0]
        q0 = np.array([t0, np.log(x0), x1, c])
        lo = np.full(4, -np.inf) if lower is None else np.asarray(lower, np.float64).copy()
        hi = np.full(4, np.inf) if upper is None else np.asarray(upper, np.float64).copy()
        lo[1] = np.log(lo[1]) if lo[1] > 0 else -np.inf
        hi[1] = np.log(hi[1]) if hi[1] > 0 else (-np.inf if hi[1] <= 0 and np.isfinite(hi[1]) else np.inf)
        for k in range(4):
            if not free[k]:
                lo[k] = hi[k] = q0[k]

        def fun(q):
            chi2, _, g = self.evaluate(batch, z, q, data, inv_sigma2)
            return chi2, -2.0 * g

        chi2_0, _, _ = self.evaluate(batch, z, np.clip(q0, lo, hi), data, inv_sigma2)
        if not np.isfinite(chi2_0):
            return dict(theta=np.array([t0, x0, x1, c]), chi2=chi2_0, n_accept=0, evals=0, status="diverged")
        r = lbfgsb(fun, q0, lo, hi, m=m, max_evals=iters)
        q = r["x"]
        theta = np.array([q[0], np.exp(q[1]) if free[1] else x0, q[2], q[3]])
        return dict(theta=theta, chi2=r["f"], n_accept=r["n_iter"], evals=r["evals"], status="ok")

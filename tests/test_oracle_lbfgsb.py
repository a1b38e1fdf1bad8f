"""Pins of the FP64 L-BFGS-B oracle (oracle/lbfgsb64.py) against what the method and the
mathematics fix, independently of the oracle's own code (CPU only).

Byrd, Lu, Nocedal and Zhu (1995) fix: the compact form of the limited-memory BFGS matrix
(their section 3), the generalized Cauchy point as the first local minimiser of the quadratic
model along the projected gradient path (section 4), the subspace step over the free variables
(section 5) and convergence to the bound-constrained minimiser; the fit wrapper is pinned against
the Levenberg-Marquardt fit, which has its own pins.
"""
import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle
import oracle.lbfgsb64 as L
import synth


def _pairs(rng, n, m):
    A = rng.normal(size=(n, n))
    H = A @ A.T + n * np.eye(n)
    out = []
    for _ in range(m):
        s = rng.normal(size=n)
        out.append((s, H @ s))          # y = H s: s^T y > 0
    return out


@pytest.mark.parametrize("m", [1, 3, 5])
def test_bfgs_matrix_equals_compact_form(m):
    """B from m BFGS updates of theta I equals theta I - W M W^T with W = [Y, theta S] and
    M = [[-D, L^T], [L, theta S^T S]]^-1, D = diag(s_i^T y_i), L_ij = s_i^T y_j for i > j."""
    rng = np.random.default_rng(m)
    n = 4
    pr = _pairs(rng, n, m)
    theta = 1.7
    S = np.stack([p[0] for p in pr], axis=1)
    Y = np.stack([p[1] for p in pr], axis=1)
    SY = S.T @ Y
    D = np.diag(np.diag(SY))
    Lo = np.tril(SY, -1)
    Mi = np.block([[-D, Lo.T], [Lo, theta * S.T @ S]])
    W = np.hstack([Y, theta * S])
    B_compact = theta * np.eye(n) - W @ np.linalg.inv(Mi) @ W.T
    B = L.bfgs_matrix(pr, theta, n)
    np.testing.assert_allclose(B, B_compact, rtol=1e-10, atol=1e-10)
    # secant condition on the newest pair, symmetry, positive definiteness
    np.testing.assert_allclose(B @ pr[-1][0], pr[-1][1], rtol=1e-10)
    np.testing.assert_allclose(B, B.T, atol=1e-10)
    assert np.all(np.linalg.eigvalsh(B) > 0)


def _model(x, g, B, xt):
    d = xt - x
    return g @ d + 0.5 * d @ B @ d


@pytest.mark.parametrize("seed", range(8))
def test_cauchy_point_is_first_local_minimiser_along_projected_path(seed):
    """Brute force: the model along x(t) = P(x - t g) on a fine grid of t; its first local minimum
    is the generalized Cauchy point."""
    rng = np.random.default_rng(100 + seed)
    n = 4
    pr = _pairs(rng, n, 2)
    B = L.bfgs_matrix(pr, 0.8, n)
    x = rng.uniform(-1, 1, n)
    g = rng.normal(size=n) * 3
    l = x - rng.uniform(0.05, 1.0, n)
    u = x + rng.uniform(0.05, 1.0, n)
    if seed % 3 == 0:
        l[1], u[1] = -np.inf, np.inf
    xc = L.cauchy_point(x, g, l, u, B)
    t = np.linspace(0.0, 5.0, 500001)
    path = np.clip(x[None, :] - t[:, None] * g[None, :], l, u)
    d = path - x
    mv = d @ g + 0.5 * np.einsum("ij,jk,ik->i", d, B, d)
    k = 0
    while k + 1 < len(t) and mv[k + 1] < mv[k]:
        k += 1
    assert np.all((xc >= l - 1e-12) & (xc <= u + 1e-12))
    np.testing.assert_allclose(xc, path[k], atol=2e-4)
    assert _model(x, g, B, xc) <= mv[k] + 1e-9


def test_subspace_step_minimises_the_model_over_the_free_variables():
    """Without truncation the step zeroes the model's gradient on the free variables at xbar."""
    rng = np.random.default_rng(7)
    n = 4
    B = L.bfgs_matrix(_pairs(rng, n, 3), 1.0, n)
    x = np.zeros(n)
    g = np.array([1.0, -2.0, 0.5, 3.0])
    l, u = np.full(n, -10.0), np.full(n, 10.0)
    l[3] = -0.1          # variable 3 reaches its bound on the Cauchy path
    xc = L.cauchy_point(x, g, l, u, B)
    xbar = L.subspace_min(x, g, l, u, B, xc)
    free = (xc > l) & (xc < u)
    grad = g + B @ (xbar - x)
    assert not free[3] and xbar[3] == xc[3]
    np.testing.assert_allclose(grad[free], 0.0, atol=1e-10)


def test_subspace_step_is_cut_back_to_the_feasible_region():
    """Where the free minimiser leaves the box, xbar is x^c + alpha (free step) with the largest
    alpha < 1 that keeps every free variable within its bounds (found here by bisection)."""
    found = 0
    for seed in range(200):
        rng = np.random.default_rng(1000 + seed)
        n = 4
        B = L.bfgs_matrix(_pairs(rng, n, 2), 0.5, n)
        x = rng.uniform(-0.2, 0.2, n)
        g = rng.normal(size=n)
        l, u = x - rng.uniform(0.01, 0.5, n), x + rng.uniform(0.01, 0.5, n)
        xc = L.cauchy_point(x, g, l, u, B)
        F = np.flatnonzero((xc > l) & (xc < u))
        if len(F) < 2:
            continue
        r = g + B @ (xc - x)
        step = np.linalg.solve(B[np.ix_(F, F)], -r[F])
        if np.all((xc[F] + step >= l[F]) & (xc[F] + step <= u[F])):
            continue
        feas = lambda a: np.all((xc[F] + a * step >= l[F] - 1e-15) & (xc[F] + a * step <= u[F] + 1e-15))
        a0, a1 = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (a0 + a1)
            a0, a1 = (mid, a1) if feas(mid) else (a0, mid)
        xbar = L.subspace_min(x, g, l, u, B, xc)
        np.testing.assert_allclose(xbar[F], xc[F] + a0 * step, atol=1e-12)
        assert np.all((xbar >= l - 1e-15) & (xbar <= u + 1e-15))
        found += 1
    assert found >= 5


def test_kept_pairs_keep_the_matrix_positive_definite():
    """A concave function in a box: steps end on bounds (the largest feasible step) where the
    curvature along them is negative; the pairs the method keeps all have s^T y > 0, so its
    quasi-Newton matrix stays positive definite, and every start ends at a vertex of the box."""
    fun = lambda x: (-x @ x + 0.3 * x[0] * x[1], -2.0 * x + 0.3 * np.array([x[1], x[0], 0.0, 0.0]))
    for seed in range(10):
        x0 = np.random.default_rng(seed).uniform(-0.9, 0.9, 4)
        res = L.lbfgsb(fun, x0, np.full(4, -1.0), np.full(4, 1.0), m=5, max_evals=30)
        for s, y in res["pairs"]:
            assert s @ y > 0.0
        assert np.all(np.abs(res["x"]) == 1.0)


@pytest.mark.parametrize("case", ["inactive", "active", "mixed", "one_sided"])
def test_bounded_linear_least_squares_matches_lsq_linear(case):
    """min ||A x - b||^2 within bounds: L-BFGS-B reaches scipy's bounded least-squares solution."""
    rng = np.random.default_rng({"inactive": 1, "active": 2, "mixed": 3, "one_sided": 4}[case])
    A = rng.normal(size=(40, 4))
    b = rng.normal(size=40)
    xu = np.linalg.lstsq(A, b, rcond=None)[0]
    if case == "inactive":
        lo, hi = xu - 1.0, xu + 1.0
    elif case == "active":
        lo, hi = xu + 0.1, xu + 1.0           # every unconstrained optimum coordinate is below its box
    elif case == "mixed":
        lo = np.array([-np.inf, xu[1] + 0.05, -np.inf, xu[3] - 2.0])
        hi = np.array([xu[0] - 0.05, np.inf, np.inf, xu[3] + 2.0])
    else:
        lo = np.array([0.0, 0.0, 0.0, 0.0])
        hi = np.full(4, np.inf)

    def fun(x):
        r = A @ x - b
        return r @ r, 2.0 * A.T @ r

    x0 = np.clip(np.zeros(4), lo, hi)
    res = L.lbfgsb(fun, x0, lo, hi, m=5, max_evals=60)
    ref = lsq_linear(A, b, bounds=(lo, hi), method="bvls", tol=1e-14)
    np.testing.assert_allclose(res["x"], ref.x, atol=1e-7)
    assert res["f"] <= 2.0 * ref.cost * (1 + 1e-12) + 1e-12
    if case == "active":
        assert np.any(res["x"] == lo)


def test_unconstrained_quadratic_reaches_the_exact_minimiser():
    rng = np.random.default_rng(11)
    A = rng.normal(size=(4, 4))
    H = A @ A.T + np.eye(4)
    c = rng.normal(size=4)
    fun = lambda x: (0.5 * x @ H @ x - c @ x, H @ x - c)
    res = L.lbfgsb(fun, np.zeros(4), np.full(4, -np.inf), np.full(4, np.inf), m=5, max_evals=40)
    # f is flat to rounding within sqrt(2 eps |f| / lambda_min) ~ 1e-8 of the minimiser
    np.testing.assert_allclose(res["x"], np.linalg.solve(H, c), atol=2e-8)


def test_rosenbrock_converges():
    """A non-quadratic valley: the iterates converge to (1, 1, 1, 1) within 150 evaluations."""
    def rosen(x):
        f = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1.0 - x[:-1]) ** 2)
        g = np.zeros_like(x)
        g[:-1] += -400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2.0 * (1.0 - x[:-1])
        g[1:] += 200.0 * (x[1:] - x[:-1] ** 2)
        return f, g
    res = L.lbfgsb(rosen, np.array([-1.2, 1.0, -0.5, 0.8]), np.full(4, -np.inf), np.full(4, np.inf),
                   max_evals=150)
    np.testing.assert_allclose(res["x"], np.ones(4), atol=1e-8)
    assert np.all(np.diff(res["history"]) <= 0)     # every accepted step lowers f


@pytest.fixture(scope="module")
def fit_case():
    model = synth.make_model()
    bands = synth.make_bands(6)
    o = oracle.Oracle(model, bands)
    out = []
    for r in synth.fit_requests(3, k=44):
        b = synth.Batch(np.float32([r.z]), np.float32([r.theta_true[0]]), np.float32([r.theta_true[1]]),
                        np.float32([r.theta_true[2]]), np.float32([r.theta_true[3]]), r.t, r.band,
                        np.int32([0, len(r.t)]))
        d, _, w = synth.make_data(o.bandflux(b), b.sn_offsets, r.normals)
        out.append((r, b, d, w))
    return oracle.FitOracle(o), out


def test_lbfgsb_fit_reaches_the_lm_minimum(fit_case):
    """Unbounded, the L-BFGS-B fit of a light curve reaches the minimum the LM fit reaches."""
    fo, items = fit_case
    for r, b, d, w in items:
        lm = fo.fit(b, r.z, r.theta_init, d, w, iters=50)
        lb = fo.fit_lbfgsb(b, r.z, r.theta_init, d, w, iters=120)
        assert abs(lb["chi2"] - lm["chi2"]) <= 1e-9 * lm["chi2"]
        q = lambda th: np.array([th[0], np.log(th[1]), th[2], th[3]])
        _, H, _ = fo.evaluate(b, r.z, q(lm["theta"]), d, w)
        sig = np.sqrt(np.diag(np.linalg.inv(H)))
        assert np.max(np.abs(q(lb["theta"]) - q(lm["theta"])) / sig) <= 1e-4


def test_lbfgsb_fit_with_an_active_bound_matches_lm_with_that_parameter_held(fit_case):
    """A bound on c that excludes the unconstrained optimum: the fit ends with c exactly on the
    bound and the other parameters at the LM fit with c held at the bound value."""
    fo, items = fit_case
    r, b, d, w = items[0]
    lm = fo.fit(b, r.z, r.theta_init, d, w, iters=50)
    c_opt = lm["theta"][3]
    bound = c_opt - 0.05
    start = np.array(r.theta_init, np.float64)
    start[3] = min(start[3], bound)
    lb = fo.fit_lbfgsb(b, r.z, start, d, w, lower=[-np.inf, 0.0, -np.inf, -np.inf],
                       upper=[np.inf, np.inf, np.inf, bound], iters=150)
    assert lb["theta"][3] == bound
    held = start.copy()
    held[3] = bound
    ref = fo.fit(b, r.z, held, d, w, iters=80, free=(True, True, True, False))
    assert abs(lb["chi2"] - ref["chi2"]) <= 1e-9 * ref["chi2"]
    np.testing.assert_allclose(lb["theta"][[0, 2]], ref["theta"][[0, 2]], atol=1e-5)
    np.testing.assert_allclose(np.log(lb["theta"][1]), np.log(ref["theta"][1]), atol=1e-6)

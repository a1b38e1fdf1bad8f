"""Pins of the FP64 nested-sampling oracle (oracle/nested64.py), CPU only: the draws' generator
against numpy's Philox, the prior transform's closed forms, and evidences, information and
posterior moments of likelihoods whose values are known analytically."""
import numpy as np
import pytest
from scipy.special import ndtr

import oracle.nested64 as N


def test_philox_matches_numpy():
    """numpy's Philox bit generator is Philox4x64-10; it increments its counter (a 256-bit integer)
    before each block, so its block after counter c - 1 is the block of counter c."""
    for ctr, key in (((1, 0, 0, 0), (7, 11)), ((123456789, 5, 0, 1 << 63), (2 ** 64 - 1, 3)),
                     ((41, 1, 0, 0), (1, N.KEY1))):
        g = np.random.Philox(counter=np.array([ctr[0] - 1, ctr[1], ctr[2], ctr[3]], np.uint64),
                             key=np.array(key, np.uint64))
        want = [int(v) for v in g.random_raw(4)]
        assert N.philox4x64_10(ctr, key) == want


def test_unit_draws_are_uniform_and_reproducible():
    u = N.unit_draws(5, 0, 4000)
    assert np.all((u > 0) & (u < 1))
    assert np.allclose(u.mean(axis=0), 0.5, atol=4 * np.sqrt(1 / 12 / 4000))
    assert np.array_equal(N.unit_draws(5, 1000, 10), u[1000:1010])
    assert not np.array_equal(N.unit_draws(6, 0, 10), u[:10])


def test_prior_transform():
    pri = [(N.FIXED, 0.3, 0.0), (N.UNIFORM, -10.0, 30.0), (N.LOG_UNIFORM, 1e-6, 1e-4), (N.UNIFORM, -3, 3),
           (N.UNIFORM, -0.3, 0.3)]
    u = np.array([[0.25, 0.25, 0.5, 0.0, 1.0]])
    th = N.prior_transform(u, pri)
    np.testing.assert_allclose(th[0], [0.3, 0.0, 1e-5, -3.0, 0.3], rtol=1e-14)


def _gauss(mu, cov):
    ic = np.linalg.inv(cov)
    lnorm = -0.5 * np.log(np.linalg.det(2 * np.pi * cov))
    d = len(mu)

    def ll(th):
        x = th[:, 3:3 + d] - mu
        return lnorm - 0.5 * np.einsum("ni,ij,nj->n", x, ic, x)
    return ll


def test_gaussian_evidence_information_and_moments():
    """A 2-D correlated Gaussian likelihood (normalised) well inside a uniform prior box of volume V:
    Z = 1 / V, H = ln V - ln(2 pi e) - ln|Sigma| / 2, posterior mean mu and covariance Sigma.  The
    estimate is held to 3 of its own error estimates, over four seeds."""
    mu = np.array([0.4, -0.05])
    cov = np.array([[0.09, 0.012], [0.012, 0.0025]])
    pri = [(N.FIXED, 0.1, 0), (N.FIXED, 0.0, 0), (N.FIXED, 1e-5, 0), (N.UNIFORM, -3.0, 3.0), (N.UNIFORM, -0.5, 0.5)]
    V = 6.0 * 1.0
    lz_true = -np.log(V)
    H_true = np.log(V) - np.log(2 * np.pi * np.e) - 0.5 * np.log(np.linalg.det(cov))
    for seed in (1, 2, 3, 4):
        r = N.nested_sampling(_gauss(mu, cov), pri, n_live=300, batch=256, seed=seed, dlogz=0.01)
        assert abs(r["logz"] - lz_true) <= 3 * r["logz_err"], (seed, r["logz"], lz_true, r["logz_err"])
        assert abs(r["information"] - H_true) <= 0.15 * H_true
        th = np.vstack([r["dead_theta"], r["live_theta"]])[:, 3:5]
        lw = np.concatenate([r["dead_logw"] + r["dead_logl"], r["live_logw"] + r["live_logl"]]) - r["logz"]
        w = np.exp(lw)
        assert abs(w.sum() - 1.0) < 1e-9
        m = w @ th
        c = (th - m).T @ ((th - m) * w[:, None])
        assert np.all(np.abs(m - mu) <= 4 * np.sqrt(np.diag(cov) / 300))
        np.testing.assert_allclose(c, cov, rtol=0.25, atol=0.003)
        # dead points rise in likelihood; the draws they came from are distinct
        assert np.all(np.diff(r["dead_logl"]) >= 0)
        assert len(set(r["dead_draw"].tolist())) == r["n_iter"]


def test_truncated_gaussian_evidence_by_erf():
    """A 1-D Gaussian likelihood cut by the prior's upper edge: Z = [Phi((b-mu)/s) - Phi((a-mu)/s)] / (b-a)."""
    mu, s, a, b = 0.8, 0.15, -1.0, 1.0
    pri = [(N.FIXED, 0.1, 0), (N.FIXED, 0.0, 0), (N.FIXED, 1e-5, 0), (N.UNIFORM, a, b), (N.FIXED, 0.0, 0)]
    ll = lambda th: -0.5 * ((th[:, 3] - mu) / s) ** 2 - np.log(s * np.sqrt(2 * np.pi))
    lz_true = np.log((ndtr((b - mu) / s) - ndtr((a - mu) / s)) / (b - a))
    errs = []
    for seed in (11, 12, 13):
        r = N.nested_sampling(ll, pri, n_live=500, batch=256, seed=seed)
        assert abs(r["logz"] - lz_true) <= 3 * r["logz_err"]
        errs.append(r["logz"] - lz_true)
    assert abs(np.mean(errs)) <= 3 * r["logz_err"] / np.sqrt(3)


def test_max_iter_and_budget_stop():
    pri = [(N.FIXED, 0.1, 0), (N.FIXED, 0.0, 0), (N.FIXED, 1e-5, 0), (N.UNIFORM, -1.0, 1.0), (N.FIXED, 0.0, 0)]
    ll = lambda th: -0.5 * (th[:, 3] / 0.01) ** 2
    r = N.nested_sampling(ll, pri, n_live=50, batch=64, max_iter=40, seed=3)
    assert r["n_iter"] == 40 and len(r["dead_logl"]) == 40
    r = N.nested_sampling(ll, pri, n_live=50, batch=64, seed=3, max_evals=300)
    assert r["stopped_on_evals"] and r["n_eval"] <= 300 + 64


def test_library_generator_matches_the_oracle_and_numpy():
    """The library's Philox4x64-10 (the driver's draws) against the oracle's and numpy's."""
    import os
    from paper_2504_08081_amd import saltbf
    if not os.path.exists(saltbf.LIB_PATH):
        pytest.fail("libsaltbf.so is not built")
    for ctr, key in (((1, 0, 0, 0), (7, 11)), ((2 ** 40 + 3, 1, 0, 0), (123, N.KEY1)), ((5, 7, 9, 2 ** 64 - 1), (0, 0))):
        assert saltbf.philox4x64_10(ctr, key) == N.philox4x64_10(ctr, key)
        g = np.random.Philox(counter=np.array([ctr[0] - 1, ctr[1], ctr[2], ctr[3]], np.uint64),
                             key=np.array(key, np.uint64))
        assert saltbf.philox4x64_10(ctr, key) == [int(v) for v in g.random_raw(4)]

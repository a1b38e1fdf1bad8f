"""GPU tests of the nested-sampling driver (sb_nested_sampling): the evidence of a light curve
whose likelihood is Gaussian in x0 against its closed form, and the whole run on a SALT light
curve against the FP64 oracle's driver with the same draws."""
import numpy as np
import pytest
from scipy.special import ndtr

import oracle
import oracle.nested64 as NS
import synth
from gpu_util import torch_or_skip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


@pytest.fixture(scope="module")
def sb(torch):
    from paper_2504_08081_amd import saltbf
    saltbf.lib()
    return saltbf


def _oracle_loglike(o, t, band, data, w, log_norm):
    """ln L of parameter rows [n, 5] by the FP64 oracle, at the float32-rounded parameters the GPU sees."""
    n_obs = len(t)

    def ll(th):
        th32 = np.float32(th)
        m = len(th32)
        b = synth.Batch(th32[:, 0], th32[:, 1], th32[:, 2], th32[:, 3], th32[:, 4], np.tile(t, m), np.tile(band, m),
                        np.arange(0, (m + 1) * n_obs, n_obs, dtype=np.int32))
        f = o.bandflux(b).reshape(m, n_obs)
        return log_norm - 0.5 * ((f - data) ** 2 * w).sum(axis=1)
    return ll


def _compare_runs(g, r, log_norm):
    """The two runs draw the same candidates, so they retire the same dead points until the first
    iteration whose decision the oracle takes with a margin (retired point to the next live one,
    examined candidates to the threshold) within the GPU's FP32 resolution of ln L (2e-6 of chi2, a
    few times the measured chi-square error).  Checks that prefix and returns its length."""
    n = min(g["n_iter"], r["n_iter"])
    chi_r = 2.0 * (log_norm - r["dead_logl"][:n])
    tol = 2e-6 * np.maximum(chi_r, 1.0)
    close = np.flatnonzero(r["dead_margin"][:n] < tol)
    i0 = int(close[0]) + 1 if len(close) else n     # decisions of iterations before i0 are unique
    i0 = min(i0, n)
    assert np.array_equal(g["dead_draw"][:i0], r["dead_draw"][:i0]), i0
    np.testing.assert_allclose(g["dead_theta"][:i0], r["dead_theta"][:i0], rtol=1e-13, atol=0)
    chi_g = 2.0 * (log_norm - g["dead_logl"][:i0])
    assert np.max(np.abs(chi_g - chi_r[:i0]) / np.maximum(chi_r[:i0], 1.0)) <= 1e-5
    same = g["dead_draw"][:n] == r["dead_draw"][:n]
    return i0, (n if same.all() else int(np.argmin(same)))


def test_gaussian_in_x0_evidence_closed_form(sb, torch):
    """Flat spectrum M0 = K through a top-hat band, only x0 free with a uniform prior: f_i = x0 C
    exactly (the trapezoid is exact for the linear integrand), so chi2 is quadratic in x0 and
    Z = exp(log_norm - chi2_min / 2) sqrt(2 pi) s [Phi((b - m)/s) - Phi((a - m)/s)] / (b - a) with
    m = sum d_i w_i / (C sum w_i), s = 1 / (C sqrt(sum w_i)).  The GPU run's ln Z is held to three of
    its error estimates; the oracle's driver on the same draws gives the same dead points."""
    K, a_band, b_band, z = 0.75, 4000.0, 5230.0, 0.2
    m0 = np.full((71, 721), K, np.float32)
    ctx = sb.Context(m0, np.zeros_like(m0), -20.0, 1.0, 2000.0, 10.0, [-0.9, 0.1, 0.01], 4302.57, 5428.55)
    tb = synth.tophat_band(a_band, b_band)
    ctx.add_band(tb.wave, tb.trans)
    zf = float(np.float32(z))
    C = K * (b_band ** 2 - a_band ** 2) / (2 * oracle.HC * (1 + zf))
    g = np.random.default_rng(4)
    n_obs = 30
    t = np.float32(np.linspace(-10.0, 40.0, n_obs))
    band = np.zeros(n_obs, np.int32)
    x0_true = 2e-5
    sig = 0.05 * x0_true * C * np.ones(n_obs)
    data = np.float32(x0_true * C + sig * g.normal(size=n_obs))
    w = np.float32(1.0 / sig ** 2)
    log_norm = float(-np.sum(np.log(np.sqrt(2 * np.pi) / np.sqrt(np.float64(w)))))
    W = np.float64(w).sum()
    m = float((np.float64(data) * np.float64(w)).sum() / (C * W))
    s = 1.0 / (C * np.sqrt(W))
    chi_min = float(((np.float64(data) - m * C) ** 2 * np.float64(w)).sum())
    lo, hi = 1.5e-5, 2.5e-5
    lz_true = (log_norm - 0.5 * chi_min + np.log(np.sqrt(2 * np.pi) * s)
               + np.log(ndtr((hi - m) / s) - ndtr((lo - m) / s)) - np.log(hi - lo))
    pri = [(0, z, 0), (0, 0.0, 0), (1, lo, hi), (0, 0.0, 0), (0, 0.0, 0)]
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    res = ctx.nested_sampling(pri, dv(t), dv(band), dv(data), dv(w), n_live=400, batch=1024, seed=21,
                              log_norm=log_norm)
    ctx.device_check()
    print(f"Gaussian in x0: ln Z {res['logz']:.4f} +- {res['logz_err']:.4f}, closed form {lz_true:.4f}, "
          f"{res['n_iter']} iterations, {res['n_eval']} evaluations")
    assert abs(res["logz"] - lz_true) <= 3 * res["logz_err"]
    o = oracle.Oracle(synth.Model(m0=m0, m1=np.zeros_like(m0), cl_coef=np.array([-0.9, 0.1, 0.01])), [tb])
    ref = NS.nested_sampling(_oracle_loglike(o, t, band, np.float64(data), np.float64(w), log_norm),
                             [(k, a, b) for k, a, b in pri], n_live=400, batch=1024, seed=21)
    i0, k = _compare_runs(res, ref, log_norm)
    print(f"oracle driver: ln Z {ref['logz']:.4f}; unique decisions up to iteration {i0}, same dead points "
          f"up to {k} of {res['n_iter']}")
    assert i0 >= 100 and k >= i0
    assert abs(res["logz"] - ref["logz"]) <= 2 * res["logz_err"]
    ctx.close()


def test_salt_light_curve_run_matches_the_oracle_driver(sb, torch, model, bands6):
    """The 120-observation light curve of the sweep, four free parameters with uniform and
    log-uniform priors around the truth: the GPU driver and the oracle's driver (same seed, same
    draws) retire the same dead points, with chi-squares within 1e-5, and agree on ln Z."""
    sw = synth.sweep_120_obs(n_samples=16)
    o6 = oracle.Oracle(model, bands6)
    n_obs = len(sw.obs_t)
    z, t0, x0, x1, c = [float(v) for v in sw.theta_true]
    f_true = o6.bandflux(synth.Batch(np.float32([z]), np.float32([t0]), np.float32([x0]), np.float32([x1]),
                                     np.float32([c]), sw.obs_t, sw.obs_band, np.int32([0, n_obs])))
    data, sig, w = synth.make_data(f_true, [0, n_obs], synth.noise_draws(n_obs, k=55))
    log_norm = float(-np.sum(np.log(np.sqrt(2 * np.pi) * np.float64(sig))))
    pri = [(0, z, 0), (1, t0 - 1.0, t0 + 1.0), (2, x0 * 0.9, x0 * 1.1), (1, x1 - 0.5, x1 + 0.5),
           (1, c - 0.05, c + 0.05)]
    ctx = sb.Context.from_model(model, bands6)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    print("case: nested sampling, 120-observation light curve", flush=True)
    res = ctx.nested_sampling(pri, dv(sw.obs_t), dv(sw.obs_band), dv(np.float32(data)), dv(np.float32(w)),
                              n_live=100, batch=256, seed=5, dlogz=0.05, log_norm=log_norm)
    ctx.device_check()
    ref = NS.nested_sampling(_oracle_loglike(o6, sw.obs_t, sw.obs_band, np.float64(data), np.float64(w), log_norm),
                             pri, n_live=100, batch=256, seed=5, dlogz=0.05)
    i0, k = _compare_runs(res, ref, log_norm)
    print(f"SALT light curve: GPU ln Z {res['logz']:.4f} +- {res['logz_err']:.4f} ({res['n_iter']} iterations, "
          f"{res['n_eval']} evaluations), oracle {ref['logz']:.4f} ({ref['n_iter']}); unique decisions up to "
          f"{i0}, same dead points up to {k}")
    assert i0 >= 100 and k >= i0
    assert abs(res["logz"] - ref["logz"]) <= 2 * res["logz_err"]
    # the posterior mean of the weighted dead and live points is within a few sigma of the truth
    th = np.vstack([res["dead_theta"], res["live_theta"]])
    lw = np.concatenate([res["dead_logw"] + res["dead_logl"], res["live_logw"] + res["live_logl"]]) - res["logz"]
    wt = np.exp(lw)
    assert abs(wt.sum() - 1.0) < 1e-6
    ctx.close()


def test_nested_sampling_argument_errors(sb, torch, model, bands6):
    ctx = sb.Context.from_model(model, bands6)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t, band = dv(np.float32([1.0, 2.0])), dv(np.int32([0, 1]))
    d, w = dv(np.float32([1.0, 1.0])), dv(np.float32([1.0, 1.0]))
    good = [(0, 0.1, 0), (1, 0.0, 1.0), (2, 1e-6, 1e-4), (1, -1, 1), (1, -0.1, 0.1)]
    for bad in ([(0, 0.1, 0), (1, 1.0, 0.0)] + good[2:], [(0, 0.1, 0), (1, 0.0, 1.0), (2, 0.0, 1e-4)] + good[3:],
                [(7, 0.1, 0)] + good[1:]):
        with pytest.raises(sb.SaltBFError) as e:
            ctx.nested_sampling(bad, t, band, d, w, n_live=10, batch=8, max_iter=5)
        assert e.value.status == sb.SB_ERR_ARG
    with pytest.raises(sb.SaltBFError):
        ctx.nested_sampling(good, t, band, d, w, n_live=1, batch=8, max_iter=5)
    r = ctx.nested_sampling(good, t, band, d, w, n_live=10, batch=8, max_iter=5)
    assert r["n_iter"] == 5
    ctx.device_check()
    ctx.close()

"""GPU tests of the continuous-batching fit server (sb_fit_submit / poll / wait / cancel).

Fits are checked against the FP64 oracle's Levenberg-Marquardt fit; a fit's
result must not depend on the other fits sharing its launches, on the byte
budget, or on how its iterations are split over launches.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import fit_resolution, torch_or_skip

pytestmark = pytest.mark.gpu

# GPU fit against the FP64 LM fit from the same start.  The minimum chi-square is held to 1e-5
# relative.  The parameters are held to 1e-2 of their statistical uncertainty sigma_q: an FP32 fit
# accepts a step only when its FP32 chi-square is lower, and near the minimum a step of
# delta sigma_q lowers chi2 by about delta^2, so steps below sqrt(eps chi2) sigma_q (eps ~ 1e-6, the
# FP32 chi-square's relative error; chi2 ~ 10-300) cannot be told apart from rounding: the FP32
# optimum is fixed to a few 1e-3 sigma_q, not to 1e-4.
CHI2_TOL = 1e-5
THETA_SIGMA_TOL = 1e-2


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


@pytest.fixture(scope="module")
def sb(torch):
    from paper_2504_08081_amd import saltbf
    saltbf.lib()
    return saltbf


@pytest.fixture(scope="module")
def o6(model, bands6):
    return oracle.Oracle(model, bands6)


@pytest.fixture(scope="module")
def requests(o6):
    """Workload-4 requests with noisy data built from the oracle's true fluxes."""
    reqs = synth.fit_requests(40, k=44)
    out = []
    for r in reqs:
        b = single_batch(r)
        f = o6.bandflux(b)
        d, sig, w = synth.make_data(f, b.sn_offsets, r.normals)
        out.append((r, d, sig, w))
    return out


def single_batch(r, theta=None):
    th = r.theta_true if theta is None else theta
    return synth.Batch(np.float32([r.z]), np.float32([th[0]]), np.float32([th[1]]), np.float32([th[2]]),
                       np.float32([th[3]]), r.t, r.band, np.int32([0, len(r.t)]))


def submit(ctx, item):
    r, d, sig, _ = item
    return ctx.fit_submit(r.t, r.band, d, sig, r.z, *r.theta_init)


def result_key(res):
    return (res.status, res.t0, res.x0, res.x1, res.c, res.chi2, res.iters, res.n_accept)


def run_all(ctx, items, timeout=60.0):
    tks = [submit(ctx, it) for it in items]
    res = [ctx.fit_wait(tk, timeout) for tk in tks]
    assert all(r is not None for r in res), "fit did not finish in time"
    return res


def test_fits_match_oracle(sb, o6, model, bands6, requests):
    """Every GPU fit of 40 requests against the FP64 LM fit from the same start: parameters within
    1e-2 of their statistical uncertainty, minimum chi2 within 1e-5."""
    ctx = sb.Context.from_model(model, bands6)
    items = requests
    res = run_all(ctx, items)
    fo = oracle.FitOracle(o6)
    worst = 0.0
    for (r, d, sig, w), g in zip(items, res):
        assert g.status == sb.SB_OK and g.iters == 50
        ref = fo.fit(single_batch(r), r.z, r.theta_init, d, w)
        th = ref["theta"]
        q64 = np.array([th[0], np.log(th[1]), th[2], th[3]])
        qg = np.array([g.t0, np.log(g.x0), g.x1, g.c])
        _, H, _ = fo.evaluate(single_batch(r), r.z, q64, d, w)
        sig_q = np.sqrt(np.diag(np.linalg.inv(H)))
        dev = np.abs(qg - q64) / sig_q
        worst = max(worst, dev.max())
        assert dev.max() <= THETA_SIGMA_TOL, (dev, g.as_dict(), ref)
        assert abs(g.chi2 - ref["chi2"]) <= CHI2_TOL * ref["chi2"]
    print(f"fit parity: max |dq|/sigma_q = {worst:.2e}")
    ctx.close()


@pytest.mark.parametrize("mask", [7, 13, 11])
def test_fits_with_held_parameters(sb, o6, model, bands6, requests, mask):
    """free_mask: the held parameters come back exactly as submitted, and the free ones match the
    FP64 LM fit over the same subset (within 1e-2 of their uncertainty, chi2 within 1e-5).  The
    fits share launches with all-free fits of the same requests."""
    ctx = sb.Context.from_model(model, bands6)
    items = requests[12:20]
    tk_held = [ctx.fit_submit(r.t, r.band, d, sig, r.z, *r.theta_init, free_mask=mask) for r, d, sig, _ in items]
    tk_all = [submit(ctx, it) for it in items]
    held = [ctx.fit_wait(tk, 60.0) for tk in tk_held]
    full = [ctx.fit_wait(tk, 60.0) for tk in tk_all]
    assert all(x is not None for x in held + full)
    fo = oracle.FitOracle(o6)
    free = [bool(mask >> k & 1) for k in range(4)]
    fr = np.flatnonzero(free)
    worst = 0.0
    for (r, d, sig, w), g, ga in zip(items, held, full):
        assert g.status == sb.SB_OK and g.iters == 50 and ga.status == sb.SB_OK
        start = np.float32(r.theta_init)
        got = np.float32([g.t0, g.x0, g.x1, g.c])
        for k in range(4):
            if not free[k]:
                assert got[k] == start[k], (k, got, start)
        ref = fo.fit(single_batch(r), r.z, r.theta_init, d, w, free=free)
        th = ref["theta"]
        q64 = np.array([th[0], np.log(th[1]), th[2], th[3]])
        qg = np.array([g.t0, np.log(g.x0), g.x1, g.c])
        _, H, _ = fo.evaluate(single_batch(r), r.z, q64, d, w)
        sig_q = np.sqrt(np.diag(np.linalg.inv(H[np.ix_(fr, fr)])))
        dev = np.abs(qg[fr] - q64[fr]) / sig_q
        worst = max(worst, dev.max())
        assert dev.max() <= THETA_SIGMA_TOL, (dev, g.as_dict(), ref)
        assert abs(g.chi2 - ref["chi2"]) <= CHI2_TOL * ref["chi2"]
        assert g.chi2 >= ga.chi2 * (1 - 1e-5)   # holding parameters cannot fit better
    print(f"free_mask {mask}: max |dq|/sigma_q = {worst:.2e}")
    with pytest.raises(sb.SaltBFError):
        r, d, sig, _ = items[0]
        ctx.fit_submit(r.t, r.band, d, sig, r.z, *r.theta_init, free_mask=16)
    ctx.close()


def test_fits_with_single_wave_workgroups(sb, o6, model, bands6, requests):
    """A 15 KiB LDS limit makes the fit kernel run one wave per fit (its eight-wave layout takes 34 KiB);
    fits still match the oracle."""
    ctx = sb.Context.from_model(model, bands6, lds_limit_bytes=15 * 1024)
    items = requests[:6]
    res = run_all(ctx, items)
    fo = oracle.FitOracle(o6)
    for (r, d, sig, w), g in zip(items, res):
        assert g.status == sb.SB_OK and g.iters == 50
        ref = fo.fit(single_batch(r), r.z, r.theta_init, d, w)
        th = ref["theta"]
        q64 = np.array([th[0], np.log(th[1]), th[2], th[3]])
        qg = np.array([g.t0, np.log(g.x0), g.x1, g.c])
        _, H, _ = fo.evaluate(single_batch(r), r.z, q64, d, w)
        sig_q = np.sqrt(np.diag(np.linalg.inv(H)))
        assert (np.abs(qg - q64) / sig_q).max() <= THETA_SIGMA_TOL
        assert abs(g.chi2 - ref["chi2"]) <= CHI2_TOL * ref["chi2"]
    ctx.close()


def test_alone_vs_in_the_mix_bitwise(sb, o6, model, bands6):
    """100 seeded requests: each fit run alone and the same fit among the other 99 sharing its
    launches (all submitted at once) give identical results."""
    items = []
    for r in synth.fit_requests(100, k=45):
        b = single_batch(r)
        d, sig, w = synth.make_data(o6.bandflux(b), b.sn_offsets, r.normals)
        items.append((r, d, sig, w))
    ctx = sb.Context.from_model(model, bands6)
    alone = [run_all(ctx, [it])[0] for it in items]
    mixed = run_all(ctx, items)
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert result_key(m) == result_key(a), i
    st = ctx.stats()
    assert st["completed"] == 200 and st["queue_depth"] == 0 and st["active_slots"] == 0
    assert st["slot_ticks"] > st["ticks"]   # the mixed fits did share launches
    ctx.close()


def test_diverged_request_is_isolated(sb, model, bands6, requests):
    """A request whose start overflows the flux (x0 = 1e30: every model flux is beyond FP32 range,
    so its chi-square at the start is not finite) ends as SB_FIT_DIVERGED after no iteration, and
    only that ticket: the twelve fits sharing its launches are bitwise their results alone."""
    ctx = sb.Context.from_model(model, bands6)
    items = requests[:12]
    alone = [run_all(ctx, [it])[0] for it in items]
    r, d, sig, _ = requests[20]
    tks = [submit(ctx, it) for it in items[:6]]
    bad = ctx.fit_submit(r.t, r.band, d, sig, r.z, r.theta_init[0], 1e30, r.theta_init[2], r.theta_init[3])
    tks += [submit(ctx, it) for it in items[6:]]
    res = [ctx.fit_wait(tk, 60.0) for tk in tks]
    rb = ctx.fit_wait(bad, 60.0)
    assert rb is not None and rb.status == sb.SB_FIT_DIVERGED and rb.iters == 0
    assert not np.isfinite(rb.chi2)
    for i, (a, m) in enumerate(zip(alone, res)):
        assert m is not None and m.status == sb.SB_OK
        assert result_key(m) == result_key(a), i
    st = ctx.stats()
    assert st["completed"] == 25 and st["active_slots"] == 0
    ctx.device_check()
    ctx.close()


def test_budget_and_tick_split_do_not_change_results(sb, model, bands6, requests):
    """A 64 KiB budget forces queueing; 7 iterations per launch splits fits differently; results match."""
    items = requests[:16]
    ref_ctx = sb.Context.from_model(model, bands6)
    ref = run_all(ref_ctx, items)
    ref_ctx.close()
    small = sb.Context.from_model(model, bands6, hbm_budget_bytes=64 * 1024)
    res = run_all(small, items)
    st = small.stats()
    small.close()
    assert [result_key(a) for a in res] == [result_key(b) for b in ref]
    assert st["ticks"] > 5
    split = sb.Context.from_model(model, bands6, iters_per_tick=7)
    res2 = run_all(split, items)
    split.close()
    assert [result_key(a) for a in res2] == [result_key(b) for b in ref]


def test_invalid_requests_rejected(sb, model, bands6, requests):
    r, d, sig, _ = requests[0]
    # a budget of 16 bytes per observation leaves no room for the fit's state: the request alone
    # exceeds it
    ctx = sb.Context.from_model(model, bands6, hbm_budget_bytes=16 * len(r.t))

    def expect(status, **kw):
        a = dict(t=r.t, band=r.band, data=d, sigma=sig, z=r.z, t0=r.theta_init[0], x0=r.theta_init[1],
                 x1=r.theta_init[2], c=r.theta_init[3])
        a.update(kw)
        with pytest.raises(sb.SaltBFError) as e:
            ctx.fit_submit(**a)
        assert e.value.status == status

    n = len(r.t)
    expect(sb.SB_ERR_ARG, band=np.full(n, 9, np.int32))
    expect(sb.SB_ERR_ARG, sigma=np.zeros(n, np.float32))
    expect(sb.SB_ERR_ARG, x0=-1.0)
    bad_t = r.t.copy()
    bad_t[0] = np.nan
    expect(sb.SB_ERR_ARG, t=bad_t)
    expect(sb.SB_ERR_ARG, t=np.zeros(300, np.float32), band=np.zeros(300, np.int32),
           data=np.zeros(300, np.float32), sigma=np.ones(300, np.float32))
    expect(sb.SB_ERR_ARG, t=np.zeros(0, np.float32), band=np.zeros(0, np.int32), data=np.zeros(0, np.float32),
           sigma=np.ones(0, np.float32))
    expect(sb.SB_ERR_ARG, z=0.95, band=np.zeros(n, np.int32))   # band 0 leaves the grid at z = 0.95
    expect(sb.SB_ERR_BUDGET)
    ctx.close()


def test_cancel(sb, model, bands6, requests):
    ctx = sb.Context.from_model(model, bands6, hbm_budget_bytes=16 * 1024)
    tks = [submit(ctx, it) for it in requests[:20]]
    for tk in tks[5:15]:
        ctx.fit_cancel(tk)
    res = [ctx.fit_wait(tk, 60.0) for tk in tks]
    st = ctx.stats()
    ctx.close()
    assert all(x is not None for x in res)
    for i, x in enumerate(res):
        if 5 <= i < 15:
            assert x.status in (sb.SB_CANCELLED, sb.SB_OK)
        else:
            assert x.status == sb.SB_OK
    assert sum(x.status == sb.SB_CANCELLED for x in res) >= 5
    assert st["completed"] + st["cancelled"] == 20
    with pytest.raises(sb.SaltBFError):
        ctx2 = sb.Context.from_model(model, bands6)
        try:
            ctx2.fit_poll(12345)
        finally:
            ctx2.close()


def test_poll_and_ticket_lifecycle(sb, model, bands6, requests):
    ctx = sb.Context.from_model(model, bands6)
    tk = submit(ctx, requests[3])
    res = None
    for _ in range(20000):
        res = ctx.fit_poll(tk)
        if res is not None:
            break
    if res is None:
        res = ctx.fit_wait(tk, 30.0)
    assert res is not None and res.status == sb.SB_OK
    assert res.t_submit <= res.t_admit <= res.t_done
    with pytest.raises(sb.SaltBFError) as e:
        ctx.fit_poll(tk)          # a result is handed out once
    assert e.value.status == sb.SB_ERR_NOTFOUND
    # one fit of 50 iterations at 5 per launch: ten launches with one fit each
    st = ctx.stats()
    assert st["submitted"] == st["admitted"] == st["completed"] == 1
    assert st["ticks"] == 10 and st["slot_ticks"] == 10
    assert st["active_slots"] == 0 and st["queue_depth"] == 0 and st["bytes_in_use"] == 0
    # the latency histogram holds the one fit in the bin of its submit-to-done time
    hist = st["latency_hist"]
    us = (res.t_done - res.t_submit) * 1e6
    assert sum(hist) == 1 and hist[max(0, min(23, int(np.floor(np.log2(max(us, 1.0))))))] == 1
    ctx.close()


# ----------------------------------------------------------------------------- L-BFGS-B solver

def test_lbfgsb_served_fits_match_oracle(sb, o6, model, bands6, requests):
    """A server running the L-BFGS-B solver: 24 fits, every third with a box on (x1, c) whose c
    upper bound excludes the unconstrained optimum, against the FP64 L-BFGS-B fit with the same
    bounds (parameters within the fit's FP32 resolution, at least 1e-2 of their uncertainty; chi2
    within 1e-5)."""
    ctx = sb.Context.from_model(model, bands6, solver=sb.SB_SOLVER_LBFGSB)
    fo = oracle.FitOracle(o6)
    items = requests[:24]
    bounds = []
    tks = []
    for i, (r, d, sig, w) in enumerate(items):
        if i % 3 == 0:
            lm = fo.fit(single_batch(r), r.z, r.theta_init, d, w)
            lo = np.float32([-np.inf, 0.0, lm["theta"][2] - 1.0, -np.inf])
            hi = np.float32([np.inf, np.inf, lm["theta"][2] + 1.0, lm["theta"][3] - 0.05])
            bounds.append((lo, hi))
            tks.append(ctx.fit_submit(r.t, r.band, d, sig, r.z, *r.theta_init, lower=lo, upper=hi))
        else:
            bounds.append(None)
            tks.append(submit(ctx, items[i]))
    res = [ctx.fit_wait(tk, 60.0) for tk in tks]
    worst = 0.0
    for (r, d, sig, w), g, bd in zip(items, res, bounds):
        assert g is not None and g.status == sb.SB_OK and 0 < g.iters <= 50
        lo = None if bd is None else np.float64(bd[0])
        hi = None if bd is None else np.float64(bd[1])
        ref = fo.fit_lbfgsb(single_batch(r), r.z, r.theta_init, d, w, lower=lo, upper=hi)
        th = ref["theta"]
        q64 = np.array([th[0], np.log(th[1]), th[2], th[3]])
        qg = np.array([g.t0, np.log(g.x0), g.x1, g.c])
        _, H, _ = fo.evaluate(single_batch(r), r.z, q64, d, w)
        dev = np.abs(qg - q64) / np.sqrt(np.diag(np.linalg.inv(H)))
        worst = max(worst, dev.max())
        # held to the fit's own FP32 resolution (see test_gpu_fit_batch), THETA_SIGMA_TOL at least
        tol = max(THETA_SIGMA_TOL, fit_resolution(o6.bandflux(single_batch(r, th)), d, w, ref["chi2"]))
        assert dev.max() <= tol, (dev, tol, g.as_dict())
        assert abs(g.chi2 - ref["chi2"]) <= CHI2_TOL * ref["chi2"]
        if bd is not None:
            assert np.float32(g.c) == bd[1][3]
    print(f"L-BFGS-B served fits: max |dq|/sigma_q = {worst:.2e}")
    ctx.close()


def test_lbfgsb_alone_vs_in_the_mix_bitwise(sb, model, bands6, requests):
    """L-BFGS-B fits alone and sharing launches with 29 others give identical results."""
    ctx = sb.Context.from_model(model, bands6, solver=sb.SB_SOLVER_LBFGSB)
    items = requests[:30]
    alone = [run_all(ctx, [it])[0] for it in items]
    mixed = run_all(ctx, items)
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert result_key(m) == result_key(a), i
    ctx.close()


def test_bounds_need_the_lbfgsb_solver_and_must_be_ordered(sb, model, bands6, requests):
    r, d, sig, _ = requests[0]
    lm = sb.Context.from_model(model, bands6)
    with pytest.raises(sb.SaltBFError) as e:
        lm.fit_submit(r.t, r.band, d, sig, r.z, *r.theta_init, lower=np.zeros(4), upper=np.ones(4))
    assert e.value.status == sb.SB_ERR_ARG
    lm.close()
    lb = sb.Context.from_model(model, bands6, solver=sb.SB_SOLVER_LBFGSB)
    for lo, hi in ((np.ones(4), np.zeros(4)), (np.zeros(4), np.float32([1, 0, 1, 1])),
                   (np.float32([np.nan, 0, 0, 0]), np.ones(4))):
        with pytest.raises(sb.SaltBFError) as e:
            lb.fit_submit(r.t, r.band, d, sig, r.z, *r.theta_init, lower=lo, upper=hi)
        assert e.value.status == sb.SB_ERR_ARG
    lb.close()

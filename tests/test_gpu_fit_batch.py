"""GPU tests of batch fits (sb_fit_batch): the fit server's Levenberg-Marquardt fit over a whole
device-resident batch of light curves, against the FP64 oracle's fit."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import fit_resolution, torch_or_skip

pytestmark = pytest.mark.gpu

CHI2_TOL = 1e-5          # minimum chi-square against the FP64 fit (relative)
THETA_SIGMA_TOL = 1e-2   # fitted parameters against the FP64 fit, in units of their uncertainty
# L-BFGS-B's line search stops on a sufficient-decrease test, chi2 + 1e-3 a g.d, that meets the FP32
# chi-square's resolution sooner than the LM's plain decrease test: its optimum is held to the fit's
# own FP32 resolution, gpu_util.fit_resolution (0.006-0.032 sigma_q here; the FP64 L-BFGS-B fits
# reach the FP64 LM optimum exactly), with THETA_SIGMA_TOL as the floor.


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
def ctx(sb, model, bands6):
    c = sb.Context.from_model(model, bands6)
    yield c
    c.close()


def single_batch(r, theta=None):
    th = r.theta_true if theta is None else theta
    return synth.Batch(np.float32([r.z]), np.float32([th[0]]), np.float32([th[1]]), np.float32([th[2]]),
                       np.float32([th[3]]), r.t, r.band, np.int32([0, len(r.t)]))


@pytest.fixture(scope="module")
def requests(o6):
    """Serving-workload requests with noisy data built from the oracle's true fluxes."""
    out = []
    for r in synth.fit_requests(40, k=44):
        b = single_batch(r)
        d, sig, w = synth.make_data(o6.bandflux(b), b.sn_offsets, r.normals)
        out.append((r, d, sig, w))
    return out


def device_batch(torch, items, free=None, x0=None, lower=None, upper=None):
    """The requests as one CSR batch of device arrays (the fit's start is the request's)."""
    dv = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).cuda()
    n = np.array([len(r.t) for r, *_ in items])
    off = np.zeros(len(items) + 1, np.int32)
    off[1:] = np.cumsum(n)
    th = np.array([r.theta_init for r, *_ in items], np.float64)
    if x0 is not None:
        th[:, 1] = x0
    args = dict(z=dv([r.z for r, *_ in items], np.float32), t0=dv(th[:, 0], np.float32),
                x0=dv(th[:, 1], np.float32), x1=dv(th[:, 2], np.float32), c=dv(th[:, 3], np.float32),
                t=dv(np.concatenate([r.t for r, *_ in items]), np.float32),
                band=dv(np.concatenate([r.band for r, *_ in items]), np.int32), fit_offsets=dv(off, np.int32),
                data=dv(np.concatenate([d for _, d, _, _ in items]), np.float32),
                inv_sigma2=dv(np.concatenate([w for *_, w in items]), np.float32))
    if free is not None:
        args["free_mask"] = dv(free, np.int32)
    if lower is not None:
        args["lower"] = dv(lower, np.float32)
    if upper is not None:
        args["upper"] = dv(upper, np.float32)
    return args


def check_against_oracle(o6, items, res, free_masks=None, solver="lm", lower=None, upper=None):
    """Each GPU fit against the FP64 fit (same solver, start, free mask and bounds): the free
    parameters within THETA_SIGMA_TOL of their uncertainty, chi2 within CHI2_TOL; held parameters and
    parameters ending on a bound exactly as given."""
    fo = oracle.FitOracle(o6)
    worst = 0.0
    for i, (r, d, sig, w) in enumerate(items):
        mask = 15 if free_masks is None or free_masks[i] == 0 else int(free_masks[i])
        free = [bool(mask >> k & 1) for k in range(4)]
        fr = np.flatnonzero(free)
        assert res["status"][i] == 0, i
        if solver == "lm":
            assert res["iters"][i] == 50, i
            ref = fo.fit(single_batch(r), r.z, r.theta_init, d, w, free=free)
        else:
            assert 0 < res["iters"][i] <= 50, i
            lo = None if lower is None else np.float64(np.float32(lower[i]))
            hi = None if upper is None else np.float64(np.float32(upper[i]))
            ref = fo.fit_lbfgsb(single_batch(r), r.z, r.theta_init, d, w, lower=lo, upper=hi, free=free)
        th = ref["theta"]
        q64 = np.array([th[0], np.log(th[1]), th[2], th[3]])
        qg = np.array([res["t0"][i], np.log(res["x0"][i]), res["x1"][i], res["c"][i]], np.float64)
        _, H, _ = fo.evaluate(single_batch(r), r.z, q64, d, w)
        sig_q = np.sqrt(np.diag(np.linalg.inv(H[np.ix_(fr, fr)])))
        dev = np.abs(qg[fr] - q64[fr]) / sig_q
        worst = max(worst, dev.max())
        tol = THETA_SIGMA_TOL
        if solver != "lm":
            f64 = o6.bandflux(single_batch(r, th))
            tol = max(tol, fit_resolution(f64, d, w, ref["chi2"]))
        assert dev.max() <= tol, (i, dev, tol)
        assert abs(res["chi2"][i] - ref["chi2"]) <= CHI2_TOL * ref["chi2"], i
        start = np.float32(r.theta_init)
        got = np.float32([res["t0"][i], res["x0"][i], res["x1"][i], res["c"][i]])
        for k in range(4):
            if not free[k]:
                assert got[k] == start[k], (i, k)
    return worst


def test_batch_fits_match_oracle(sb, ctx, o6, torch, requests):
    """40 light curves (8-256 observations, 2-6 bands) fitted in one call, each against the FP64 LM
    fit from the same start: parameters within 1e-2 of their uncertainty, minimum chi2 within 1e-5."""
    print("case: sb_fit_batch, 40 fits", flush=True)
    out = ctx.fit_batch(**device_batch(torch, requests))
    ctx.device_check()
    worst = check_against_oracle(o6, requests, sb.fit_results(out))
    print(f"batch fit parity: max |dq|/sigma_q = {worst:.2e}")


def test_batch_fits_with_held_parameters(sb, ctx, o6, torch, requests):
    """Per-fit free masks (0 = all free): held parameters come back exactly as given, the free ones
    match the oracle's fit of the free subset."""
    items = requests[:16]
    masks = np.array([7, 13, 11, 0, 14, 5, 15, 9] * 2, np.int32)
    out = ctx.fit_batch(**device_batch(torch, items, free=masks))
    ctx.device_check()
    check_against_oracle(o6, items, sb.fit_results(out), masks)


def test_batch_fit_does_not_depend_on_the_rest_of_the_batch(sb, ctx, torch, requests):
    """Each fit's result is bitwise the same in the 40-fit call and in calls on parts of it."""
    full = ctx.fit_batch(**device_batch(torch, requests)).cpu().numpy()
    for lo, hi in ((0, 1), (0, 7), (7, 40), (23, 24)):
        part = ctx.fit_batch(**device_batch(torch, requests[lo:hi])).cpu().numpy()
        assert np.array_equal(part, full[lo:hi]), (lo, hi)
    ctx.device_check()


def test_batch_fit_iteration_split_does_not_change_results(sb, model, bands6, torch, requests):
    """Seven iterations per launch instead of five (other launch boundaries): bitwise the same fits."""
    items = requests[:12]
    a = sb.Context.from_model(model, bands6)
    b = sb.Context.from_model(model, bands6, iters_per_tick=7)
    ra = a.fit_batch(**device_batch(torch, items)).cpu().numpy()
    rb = b.fit_batch(**device_batch(torch, items)).cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(ra, rb)


def test_batch_fit_bad_inputs_are_isolated(sb, ctx, torch, requests):
    """A start whose fluxes overflow (x0 = 1e30) diverges alone; malformed offsets of one fit and a
    band id beyond the registry are flagged (SB_ERR_RANGE) and affect only their own fits."""
    items = requests[:6]
    ref = ctx.fit_batch(**device_batch(torch, items)).cpu().numpy()
    x0 = np.array([r.theta_init[1] for r, *_ in items])
    x0[2] = 1e30
    res = sb.fit_results(ctx.fit_batch(**device_batch(torch, items, x0=x0)))
    ctx.device_check()
    assert res["status"][2] == sb.SB_FIT_DIVERGED and res["iters"][2] == 0 and not np.isfinite(res["chi2"][2])
    keep = [0, 1, 3, 4, 5]
    got = ctx.fit_batch(**device_batch(torch, items, x0=x0)).cpu().numpy()
    assert np.array_equal(got[keep], ref[keep])
    # fit 4's offsets run backwards
    d = device_batch(torch, items)
    off = d["fit_offsets"].cpu().numpy()
    off[5] = off[4] - 1
    d["fit_offsets"] = torch.from_numpy(off).cuda()
    r2 = ctx.fit_batch(**d)
    with pytest.raises(sb.SaltBFError) as e:
        ctx.device_check()
    assert e.value.status == sb.SB_ERR_RANGE
    r2n = r2.cpu().numpy()
    assert sb.fit_results(r2n)["status"][4] == sb.SB_FIT_DIVERGED
    assert np.array_equal(r2n[:4], ref[:4])
    # a band id beyond the registry in fit 1
    d = device_batch(torch, items)
    band = d["band"].cpu().numpy()
    band[int(off[1])] = 40
    d["band"] = torch.from_numpy(band).cuda()
    r3 = ctx.fit_batch(**d).cpu().numpy()
    with pytest.raises(sb.SaltBFError):
        ctx.device_check()
    assert sb.fit_results(r3)["status"][1] == sb.SB_FIT_DIVERGED
    assert np.array_equal(r3[[0, 2, 3, 4, 5]], ref[[0, 2, 3, 4, 5]])
    ctx.device_check()


def test_batch_fit_argument_errors(sb, ctx, torch, requests):
    import ctypes
    d = device_batch(torch, requests[:3])
    with pytest.raises(ValueError):
        ctx.fit_batch(**{**d, "t0": d["t0"][:2]})
    with pytest.raises(TypeError):
        ctx.fit_batch(**{**d, "z": d["z"].cpu()})
    L = sb.lib()
    assert L.sb_fit_batch(ctx._h, None, None, None) == sb.SB_ERR_ARG
    desc = ctx._fit_batch_desc(**{k: d[k] for k in d}, free_mask=None)
    assert L.sb_fit_batch(ctx._h, ctypes.byref(desc), None, None) == sb.SB_ERR_ARG
    desc.n_fit = 0
    assert L.sb_fit_batch(ctx._h, ctypes.byref(desc), None, None) == sb.SB_OK


# ----------------------------------------------------------------------------- L-BFGS-B

@pytest.fixture(scope="module")
def ctx_lb(sb, model, bands6):
    c = sb.Context.from_model(model, bands6, solver=sb.SB_SOLVER_LBFGSB)
    yield c
    c.close()


def test_lbfgsb_batch_fits_match_oracle(sb, ctx_lb, o6, torch, requests):
    """40 light curves fitted by L-BFGS-B in one call, each against the FP64 L-BFGS-B fit from the
    same start (50 evaluations): parameters within 1e-2 of their uncertainty, chi2 within 1e-5."""
    print("case: sb_fit_batch L-BFGS-B, 40 fits", flush=True)
    out = ctx_lb.fit_batch(**device_batch(torch, requests))
    ctx_lb.device_check()
    res = sb.fit_results(out)
    worst = check_against_oracle(o6, requests, res, solver="lbfgsb")
    print(f"L-BFGS-B batch fit parity: max |dq|/sigma_q = {worst:.2e}, evaluations {res['iters'].min()}-"
          f"{res['iters'].max()}, iterations {res['n_accept'].min()}-{res['n_accept'].max()}")


def test_lbfgsb_bounds_and_held_parameters(sb, ctx_lb, o6, torch, requests):
    """Per-fit bounds: on every other fit an upper bound on c 0.05 below the unconstrained optimum
    (active at the solution: c ends exactly on it) and a box on x1 containing its optimum; free
    masks on a few fits.  Against the FP64 L-BFGS-B fit with the same bounds."""
    items = requests[:16]
    fo = oracle.FitOracle(o6)
    lower = np.tile(np.float32([-np.inf, 0.0, -np.inf, -np.inf]), (len(items), 1))
    upper = np.tile(np.float32([np.inf, np.inf, np.inf, np.inf]), (len(items), 1))
    masks = np.array([0, 0, 0, 7, 0, 0, 11, 0] * 2, np.int32)
    active = []
    for i, (r, d, sig, w) in enumerate(items):
        lm = fo.fit(single_batch(r), r.z, r.theta_init, d, w)
        if i % 2 == 0:
            upper[i, 3] = np.float32(lm["theta"][3] - 0.05)
            if masks[i] == 0 or masks[i] & 8:
                active.append(i)
        lower[i, 2] = np.float32(lm["theta"][2] - 1.0)
        upper[i, 2] = np.float32(lm["theta"][2] + 1.0)
    out = ctx_lb.fit_batch(**device_batch(torch, items, free=masks, lower=lower, upper=upper))
    ctx_lb.device_check()
    res = sb.fit_results(out)
    check_against_oracle(o6, items, res, masks, solver="lbfgsb", lower=lower, upper=upper)
    for i in active:
        assert res["c"][i] == upper[i, 3], i


def test_lbfgsb_batch_does_not_depend_on_the_rest_of_the_batch(sb, ctx_lb, torch, requests):
    full = ctx_lb.fit_batch(**device_batch(torch, requests)).cpu().numpy()
    for lo, hi in ((0, 1), (5, 23)):
        part = ctx_lb.fit_batch(**device_batch(torch, requests[lo:hi])).cpu().numpy()
        assert np.array_equal(part, full[lo:hi]), (lo, hi)
    noalloc = ctx_lb.fit_batch_noalloc(**device_batch(torch, requests)).cpu().numpy()
    assert np.array_equal(noalloc, full)
    ctx_lb.device_check()


def test_bounds_need_the_lbfgsb_solver(sb, ctx, torch, requests):
    d = device_batch(torch, requests[:2], lower=np.zeros((2, 4)), upper=np.ones((2, 4)))
    with pytest.raises(sb.SaltBFError) as e:
        ctx.fit_batch(**d)
    assert e.value.status == sb.SB_ERR_ARG

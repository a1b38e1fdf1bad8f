"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: fluxes <= 1e-5 relative, gradients and Jacobians <= 1e-4 relative
(scaled parameters), as stated in tests/gpu_util.py.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import (FLUX_TOL, GRAD_TOL, flux_rel_err, grad_norm_err, grad_propagated_excess, grad_rel_err,
                      jac_rel_err, oracle_over_batch, to_dev, torch_or_skip)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_or_skip()


@pytest.fixture(scope="module")
def sb():
    from paper_2504_08081_amd import saltbf
    saltbf.lib()   # raises if the library is not built
    return saltbf


@pytest.fixture(scope="module")
def ctx4(sb, torch, model, bands4):
    return sb.Context.from_model(model, bands4)


@pytest.fixture(scope="module")
def ctx6(sb, torch, model, bands6):
    return sb.Context.from_model(model, bands6)


@pytest.fixture(scope="module")
def o4(model, bands4):
    return oracle.Oracle(model, bands4)


@pytest.fixture(scope="module")
def o6(model, bands6):
    return oracle.Oracle(model, bands6)


@pytest.fixture(scope="module")
def big_batch():
    return synth.batch_4096_sn()


def run_fwd(ctx, batch, torch):
    d = to_dev(batch, torch)
    f = ctx.bandflux(**d)
    ctx.device_check()
    return f.cpu().numpy()


def run_jac(ctx, batch, torch, cot=None):
    d = to_dev(batch, torch)
    if cot is None:
        cot = np.zeros(batch.n_obs, np.float32)
    r = ctx.bandflux_vjp(**d, cotangent=torch.from_numpy(np.float32(cot)).cuda(), want_flux=True, want_jac=True)
    ctx.device_check()
    return r["flux"].cpu().numpy(), r["jac"].cpu().numpy(), r["grad"].cpu().numpy()


def x0_per_obs(batch):
    return np.repeat(batch.x0.astype(np.float64), np.diff(batch.sn_offsets))


# ----------------------------------------------------------------------------- one supernova, 40 observations

def test_one_sn_forward_all_40(ctx4, o4, torch):
    b = synth.one_sn_40_obs()
    print("case: one_sn_40_obs forward, 40 obs", flush=True)
    f = run_fwd(ctx4, b, torch)
    f64 = o4.bandflux(b)
    err = flux_rel_err(f, f64, b.sn_offsets)
    print(f"one SN flux rel err max {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() <= FLUX_TOL


def test_one_sn_jacobian_rows(ctx4, o4, torch):
    b = synth.one_sn_40_obs()
    f, J, _ = run_jac(ctx4, b, torch)
    f64, J64 = o4.jac(b)
    assert flux_rel_err(f, f64, b.sn_offsets).max() <= FLUX_TOL
    err = jac_rel_err(J, J64, x0_per_obs(b), b.sn_offsets)
    print(f"one SN jacobian rel err max per param {err.max(axis=0)}")
    assert err.max() <= GRAD_TOL


# ----------------------------------------------------------------------------- small full batch

def test_small_batch_every_result(ctx6, o6, torch):
    """A 96-supernova batch (1-300 observations each): every flux, Jacobian row and cotangent
    gradient against the oracle.  With random cotangents a gradient component can cancel by
    hundreds across observations, so besides the norm-wise 1e-4 bound each component is held to
    1e-4 or to the error that the measured errors of its Jacobian rows propagate into its sum
    (plus the sum's own FP32 rounding)."""
    b = synth.random_batch(31, 96, 1, 300, synth.make_bands(6), synth.make_model())
    g = np.random.default_rng(7)
    cot = g.normal(size=b.n_obs).astype(np.float32)
    f, J, grad = run_jac(ctx6, b, torch, cot)
    f64, J64 = o6.jac(b)
    g64 = oracle.segment_sum(cot.astype(np.float64)[:, None] * J64, b.sn_offsets)
    ef = flux_rel_err(f, f64, b.sn_offsets)
    ej = jac_rel_err(J, J64, x0_per_obs(b), b.sn_offsets)
    eg = grad_rel_err(grad, g64, b.x0)
    en = grad_norm_err(grad, g64, b.x0)
    ec = grad_propagated_excess(grad, g64, b.x0, b.sn_offsets, cot, J64, J)
    print(f"small batch: flux {ef.max():.3e} jac {ej.max():.3e} grad component-wise {eg.max():.3e} "
          f"({int(np.sum(eg > GRAD_TOL))} above 1e-4) norm-wise {en.max():.3e}; "
          f"worst over the propagated bound {ec.max():.3f}")
    assert ef.max() <= FLUX_TOL and ej.max() <= GRAD_TOL
    assert en.max() <= GRAD_TOL
    assert np.all((eg <= GRAD_TOL) | (ec <= 1.0))
    f_fwd = run_fwd(ctx6, b, torch)
    assert flux_rel_err(f_fwd, f64, b.sn_offsets).max() <= FLUX_TOL


def test_adjoint_vs_central_differences(ctx6, torch):
    """The adjoint's Jacobian rows against central differences of the GPU forward kernel, step
    h_q = 1e-4 max(|theta_q|, s_q) with s = (0.1, 1 d, x0, 1, 0.1).  Both sides run in FP32: the
    forward kernel's rounding (about 1e-7 of f, 2.1e-7 at most against FP64) divided by the step
    puts the differences within about 1e-3 of the row's scale |x0 df/dx0| = |f|, so each
    observation's scaled row is held norm-wise to 1e-2 (the FP64 differences that pin the
    oracle's own gradient are a CPU test)."""
    model = synth.make_model()
    b = synth.random_batch(47, 64, 5, 120, synth.make_bands(6), model)
    f, J, _ = run_jac(ctx6, b, torch)
    P = np.stack([b.z, b.t0, b.x0, b.x1, b.c], axis=1).astype(np.float64)
    scale = np.stack([np.full(b.n_sn, 0.1), np.ones(b.n_sn), b.x0.astype(np.float64),
                      np.ones(b.n_sn), np.full(b.n_sn, 0.1)], axis=1)
    d = to_dev(b, torch)
    n_s = np.diff(b.sn_offsets)
    J_fd = np.zeros_like(J, dtype=np.float64)
    for q, name in enumerate(("z", "t0", "x0", "x1", "c")):
        h = 1e-4 * np.maximum(np.abs(P[:, q]), scale[:, q])
        vals = []
        for sign in (1.0, -1.0):
            v = np.float32(P[:, q] + sign * h)
            dd = dict(d)
            dd[name] = torch.from_numpy(v).cuda()
            vals.append(ctx6.bandflux(**dd).cpu().numpy().astype(np.float64))
            hq = (np.float64(np.float32(P[:, q] + h)) - np.float64(np.float32(P[:, q] - h)))  # steps as rounded
        J_fd[:, q] = (vals[0] - vals[1]) / np.repeat(hq, n_s)
    ctx6.device_check()
    s_obs = np.repeat(scale, n_s, axis=0)
    Jt, Jt_fd = J.astype(np.float64) * s_obs, J_fd * s_obs
    row = np.max(np.abs(Jt), axis=1)
    live = row > 0
    err = np.max(np.abs(Jt_fd - Jt), axis=1)[live] / row[live]
    print(f"adjoint vs central differences: scaled row error max {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() <= 1e-2


# ----------------------------------------------------------------------------- the 4,096-supernova batch

def sample_sns(batch, n=40, seed=3):
    n_s = np.diff(batch.sn_offsets)
    g = np.random.default_rng(seed)
    pick = set(g.choice(batch.n_sn, n, replace=False).tolist())
    pick |= {int(np.argmax(n_s)), int(np.argmin(n_s)), int(np.argmax(batch.z)), int(np.argmin(batch.z)),
             0, batch.n_sn - 1}
    return np.array(sorted(pick))


def test_batch_4096_forward_sampled(ctx6, o6, big_batch, torch):
    print(f"case: batch_4096_sn forward, {big_batch.n_sn} SN, {big_batch.n_obs} obs", flush=True)
    f = run_fwd(ctx6, big_batch, torch)
    assert np.all(np.isfinite(f))
    idx = sample_sns(big_batch)
    sub = big_batch.subset(idx)
    f64 = o6.bandflux(sub)
    sel = np.concatenate([np.arange(big_batch.sn_offsets[s], big_batch.sn_offsets[s + 1]) for s in idx])
    err = flux_rel_err(f[sel], f64, sub.sn_offsets)
    print(f"big_batch sampled {len(idx)} SN / {len(sel)} obs: flux rel err max {err.max():.3e} "
          f"p99 {np.percentile(err, 99):.3e} median {np.median(err):.3e}")
    assert err.max() <= FLUX_TOL


def test_batch_4096_chi2_gradient_sampled(ctx6, o6, big_batch, torch):
    """Chi-square gradient of the 4,096-supernova batch at perturbed parameters, full batch on the GPU,
    sampled supernovae against the oracle's analytic FP64 gradient."""
    print("case: 4096-SN chi2 gradient", flush=True)
    truth = big_batch
    ev = synth.perturb(truth)
    idx = sample_sns(truth, n=32, seed=5)
    sub_true = truth.subset(idx)
    f_true = o6.bandflux(sub_true)
    normals = synth.noise_draws(sub_true.n_obs)
    d_sub, _, w_sub = synth.make_data(f_true, sub_true.sn_offsets, normals)
    data = np.zeros(truth.n_obs, np.float32)
    w = np.ones(truth.n_obs, np.float32)
    sel = np.concatenate([np.arange(truth.sn_offsets[s], truth.sn_offsets[s + 1]) for s in idx])
    data[sel] = d_sub
    w[sel] = w_sub
    d = to_dev(ev, torch)
    r = ctx6.bandflux_vjp(**d, chi2=True, data=torch.from_numpy(data).cuda(), inv_sigma2=torch.from_numpy(w).cuda(),
                          want_flux=True)
    ctx6.device_check()
    grad = r["grad"].cpu().numpy()[idx]
    chi2 = r["chi2"].cpu().numpy()[idx]
    sub_ev = ev.subset(idx)
    f64, c64, g64 = o6.chi2_grad(sub_ev, d_sub, w_sub)
    eg = grad_rel_err(grad, g64, sub_ev.x0)
    ec = np.abs(chi2 - c64) / np.abs(c64)
    ef = flux_rel_err(r["flux"].cpu().numpy()[sel], f64, sub_ev.sn_offsets)
    en = grad_norm_err(grad, g64, sub_ev.x0)
    print(f"4096-SN chi2 gradient: grad rel err max {eg.max():.3e} (per param {eg.max(axis=0)}), norm-wise {en.max():.3e}, "
          f"chi2 {ec.max():.3e}, flux {ef.max():.3e}")
    assert eg.max() <= GRAD_TOL
    assert ec.max() <= 1e-4
    assert ef.max() <= FLUX_TOL


def test_batch_65536_forward_adjoint_sampled(ctx6, o6, torch):
    """The 65,536 x 100 batch, forward + adjoint with random cotangents on the GPU in one launch:
    sampled supernovae's fluxes, Jacobian rows and gradients against the oracle (flux 1e-5;
    Jacobian 1e-4; gradient norm-wise 1e-4, each component to 1e-4 or to the error its measured
    Jacobian errors propagate into it, as for the small batch)."""
    print("case: 65536-SN forward + adjoint", flush=True)
    b = synth.perturb(synth.batch_65536_sn(), k=7)
    cot = np.random.default_rng(23).normal(size=b.n_obs).astype(np.float32)
    r = ctx6.bandflux_vjp(**to_dev(b, torch), cotangent=torch.from_numpy(cot).cuda(), want_flux=True,
                          want_jac=True)
    ctx6.device_check()
    idx = sample_sns(b, n=24, seed=9)
    sub = b.subset(idx)
    sel = np.concatenate([np.arange(b.sn_offsets[s], b.sn_offsets[s + 1]) for s in idx])
    f64, J64 = o6.jac(sub)
    g64 = oracle.segment_sum(cot[sel].astype(np.float64)[:, None] * J64, sub.sn_offsets)
    f = r["flux"].cpu().numpy()[sel]
    J = r["jac"].cpu().numpy()[sel]
    grad = r["grad"].cpu().numpy()[idx]
    ef = flux_rel_err(f, f64, sub.sn_offsets)
    ej = jac_rel_err(J, J64, x0_per_obs(sub), sub.sn_offsets)
    en = grad_norm_err(grad, g64, sub.x0)
    eg = grad_rel_err(grad, g64, sub.x0)
    ec = grad_propagated_excess(grad, g64, sub.x0, sub.sn_offsets, cot[sel], J64, J)
    print(f"65536-SN sampled {len(idx)} SN: flux {ef.max():.3e} jac {ej.max():.3e} grad norm-wise {en.max():.3e} "
          f"component-wise {eg.max():.3e}; worst over the propagated bound {ec.max():.3f}")
    assert ef.max() <= FLUX_TOL and ej.max() <= GRAD_TOL and en.max() <= GRAD_TOL
    assert np.all((eg <= GRAD_TOL) | (ec <= 1.0))


def test_batch_4096_every_flux_chi2_and_gradient(ctx6, big_batch, torch):
    """The whole 4,096-supernova batch against the oracle (run over all supernovae on a pool of
    CPU processes): every flux at the true parameters, and every supernova's fluxes, Jacobian
    rows, chi-square and gradient at perturbed ones, data drawn around the oracle's true fluxes.
    A gradient component is a sum of terms of both signs (cotangent 2 (f - d) / sigma^2 times
    Jacobian entries) that can cancel to far below its terms, and its cotangent is formed from a
    flux whose own error is magnified by |f| / |f - d| (about twenty-fold at 5% noise).  So besides
    the norm-wise 1e-4 bound each component is held to 1e-4 or to the error that the MEASURED
    flux and Jacobian-row errors of its own supernova propagate into it; the fluxes themselves are
    held here to 1e-6, a tenth of the flux tolerance and about 2.5 times their measured worst."""
    print("case: 4096-SN batch, every result", flush=True)
    f_true64 = oracle_over_batch("flux", big_batch, 6)
    f_gpu = ctx6.bandflux(**to_dev(big_batch, torch)).cpu().numpy()
    ef = flux_rel_err(f_gpu, f_true64, big_batch.sn_offsets)
    data, _, w = synth.make_data(f_true64, big_batch.sn_offsets, synth.noise_draws(big_batch.n_obs))
    ev = synth.perturb(big_batch)
    f64, c64, g64 = oracle_over_batch("chi2", ev, 6, data=data, w=w)
    r = ctx6.bandflux_vjp(**to_dev(ev, torch), chi2=True, data=torch.from_numpy(data).cuda(),
                          inv_sigma2=torch.from_numpy(w).cuda(), want_flux=True, want_jac=True)
    ctx6.device_check()
    grad, chi2 = r["grad"].cpu().numpy(), r["chi2"].cpu().numpy()
    fg, Jg = r["flux"].cpu().numpy(), r["jac"].cpu().numpy()
    ef2 = flux_rel_err(fg, f64, ev.sn_offsets)
    eg = grad_rel_err(grad, g64, ev.x0)
    en = grad_norm_err(grad, g64, ev.x0)
    ec = np.abs(chi2 - c64) / np.abs(c64)
    _, J64 = oracle_over_batch("jac", ev, 6)
    ej = jac_rel_err(Jg, J64, x0_per_obs(ev), ev.sn_offsets)
    cot64 = 2.0 * (f64 - data.astype(np.float64)) * w
    cot_err = 2.0 * w.astype(np.float64) * np.abs(fg.astype(np.float64) - f64)
    ek = grad_propagated_excess(grad, g64, ev.x0, ev.sn_offsets, cot64, J64, Jg, cot_err=cot_err)
    print(f"4096-SN every result: flux {ef.max():.3e} (perturbed {ef2.max():.3e}), jac {ej.max():.3e}, "
          f"chi2 {ec.max():.3e}, grad component-wise {eg.max():.3e} (p99 {np.percentile(eg, 99):.3e}, "
          f"{int(np.sum(eg > GRAD_TOL))} of {eg.size} above 1e-4), norm-wise {en.max():.3e}; "
          f"worst over the propagated bound {ek.max():.3f}")
    assert ef.max() <= 1e-6 and ef2.max() <= 1e-6
    assert ej.max() <= GRAD_TOL
    assert ec.max() <= 1e-5
    assert en.max() <= GRAD_TOL
    assert np.all((eg <= GRAD_TOL) | (ek <= 1.0))


def test_run_twice_bitwise(ctx6, big_batch, torch):
    d = to_dev(big_batch, torch)
    cot = torch.ones(big_batch.n_obs, dtype=torch.float32, device="cuda")
    a = ctx6.bandflux_vjp(**d, cotangent=cot, want_flux=True)
    b = ctx6.bandflux_vjp(**d, cotangent=cot, want_flux=True)
    torch.cuda.synchronize()
    assert torch.equal(a["grad"], b["grad"]) and torch.equal(a["flux"], b["flux"])
    f = ctx6.bandflux(**d)
    torch.cuda.synchronize()
    # forward-only and forward+adjoint kernels agree to rounding
    rel = ((f - a["flux"]).abs() / a["flux"].abs().clamp_min(1e-30)).max().item()
    assert rel < 1e-6


def test_prepared_calls_match_plain_calls(ctx6, big_batch, torch):
    """A prepared call launches the same kernel on the same buffers: bitwise equal to the plain call,
    also after the parameter buffers are updated in place between launches."""
    d = to_dev(big_batch, torch)
    cot = torch.ones(big_batch.n_obs, dtype=torch.float32, device="cuda")
    pv = ctx6.prepare_bandflux_vjp(**d, cotangent=cot, want_flux=True)
    pf = ctx6.prepare_bandflux(**d)
    for step in range(2):
        pv()
        pf()
        a = ctx6.bandflux_vjp(**d, cotangent=cot, want_flux=True)
        f = ctx6.bandflux(**d)
        torch.cuda.synchronize()
        assert torch.equal(pv.outputs["grad"], a["grad"]) and torch.equal(pv.outputs["flux"], a["flux"])
        assert torch.equal(pf.outputs["out"], f)
        d["x1"].add_(0.25)   # in-place update seen by the next launch of both prepared calls
    ctx6.device_check()


def test_graph_replays_match_eager(ctx6, big_batch, torch):
    """Prepared calls captured in a HIP graph (torch.cuda.CUDAGraph on a side stream): every replay
    equals the eager call bitwise, with eager work and synchronisations between replays, and a
    replay sees parameter buffers updated in place."""
    d = to_dev(big_batch, torch)
    data = torch.ones(big_batch.n_obs, dtype=torch.float32, device="cuda")
    w = torch.ones(big_batch.n_obs, dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    pv = ctx6.prepare_bandflux_vjp(**d, data=data, inv_sigma2=w, chi2=True, stream=side)
    pf = ctx6.prepare_bandflux(**d, stream=side)
    with torch.cuda.stream(side):
        pv()
        pf()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        pv()
        pf()
        pv()
    for rep in range(4):
        g.replay()
        torch.cuda.synchronize()
        grad_g, chi_g, f_g = pv.outputs["grad"].clone(), pv.outputs["chi2"].clone(), pf.outputs["out"].clone()
        a = ctx6.bandflux_vjp(**d, data=data, inv_sigma2=w, chi2=True)
        f = ctx6.bandflux(**d)
        torch.cuda.synchronize()
        assert torch.equal(grad_g, a["grad"]) and torch.equal(chi_g, a["chi2"]), rep
        assert torch.equal(f_g, f), rep
        assert torch.isfinite(grad_g).all()
        d["c"].add_(0.01)    # the next replay reads the updated colours
    ctx6.device_check()


def test_single_wave_workgroups_when_lds_is_short(sb, model, bands6, big_batch, torch):
    """With a 15 KiB LDS limit the adjoint runs one wave per workgroup instead of three (its one-wave
    layout takes 14.0 KiB, the three-wave one 25.4 KiB; the forward's three-wave layout, 9.1 KiB, still
    fits): the per-observation results are bitwise those of the multi-wave kernels (each band's
    projections are built by one wave either way) and the per-supernova gradient differs only by
    reduction order."""
    small = sb.Context.from_model(model, bands6, lds_limit_bytes=15 * 1024)
    full = sb.Context.from_model(model, bands6)
    ev = synth.perturb(big_batch)
    d = to_dev(ev, torch)
    cot = torch.from_numpy(np.random.default_rng(11).normal(size=ev.n_obs).astype(np.float32)).cuda()
    a = small.bandflux_vjp(**d, cotangent=cot, want_flux=True)
    b = full.bandflux_vjp(**d, cotangent=cot, want_flux=True)
    fa, fb = small.bandflux(**d), full.bandflux(**d)
    small.device_check()
    full.device_check()
    assert torch.equal(a["flux"], b["flux"]) and torch.equal(fa, fb)
    en = grad_norm_err(a["grad"].cpu().numpy(), b["grad"].cpu().numpy().astype(np.float64), ev.x0)
    assert en.max() <= 1e-5, en.max()
    small.close()
    full.close()


def test_many_bands_and_a_long_light_curve(sb, model, torch):
    """Twelve bands (two forward groups, three adjoint groups per supernova) and a 1,500-observation
    light curve (many passes of the observation loops), against the oracle."""
    bands12 = synth.make_bands(12)
    ctx = sb.Context.from_model(model, bands12)
    o12 = oracle.Oracle(model, bands12)
    g = np.random.default_rng(12)
    n0 = 1500
    ph = np.sort(g.uniform(-18.0, 48.0, n0))
    t_a = np.float32(100.0 + 1.3 * ph)
    band_a = g.integers(0, 12, n0).astype(np.int32)
    b = synth.Batch(np.float32([0.3, 0.05]), np.float32([100.0, 50.0]), np.float32([2e-5, 1e-4]),
                    np.float32([0.7, -1.2]), np.float32([-0.08, 0.15]),
                    np.concatenate([t_a, np.float32([52.0, 60.0, 71.0])]),
                    np.concatenate([band_a, np.int32([11, 0, 5])]), np.int32([0, n0, n0 + 3]))
    cot = g.normal(size=b.n_obs).astype(np.float32)
    f, J, grad = run_jac(ctx, b, torch, cot)
    f64, J64 = o12.jac(b)
    g64 = oracle.segment_sum(cot.astype(np.float64)[:, None] * J64, b.sn_offsets)
    assert flux_rel_err(f, f64, b.sn_offsets).max() <= FLUX_TOL
    assert jac_rel_err(J, J64, x0_per_obs(b), b.sn_offsets).max() <= GRAD_TOL
    assert grad_norm_err(grad, g64, b.x0).max() <= GRAD_TOL
    assert flux_rel_err(run_fwd(ctx, b, torch), f64, b.sn_offsets).max() <= FLUX_TOL
    ctx.close()


def test_results_do_not_depend_on_the_rest_of_the_batch(ctx6, big_batch, torch):
    """Every supernova's flux, gradient and chi-square are bitwise the same whether it is evaluated
    in the full 4,096-supernova batch or in a chunk of 1,000 (other neighbours, other workgroup
    indices, a differently filled device)."""
    ev = synth.perturb(big_batch)
    g = np.random.default_rng(21)
    data = g.normal(size=ev.n_obs).astype(np.float32)
    w = np.abs(g.normal(size=ev.n_obs)).astype(np.float32)
    run = lambda b, dd, ww: ctx6.bandflux_vjp(**to_dev(b, torch), chi2=True, data=torch.from_numpy(dd).cuda(),
                                               inv_sigma2=torch.from_numpy(ww).cuda(), want_flux=True)
    full = run(ev, data, w)
    torch.cuda.synchronize()
    for lo in range(0, ev.n_sn, 1000):
        idx = np.arange(lo, min(ev.n_sn, lo + 1000))
        sel = np.arange(ev.sn_offsets[lo], ev.sn_offsets[idx[-1] + 1])
        part = run(ev.subset(idx), data[sel], w[sel])
        torch.cuda.synchronize()
        assert torch.equal(part["grad"], full["grad"][lo:lo + len(idx)])
        assert torch.equal(part["chi2"], full["chi2"][lo:lo + len(idx)])
        assert torch.equal(part["flux"], full["flux"][sel[0]:sel[-1] + 1])
    ctx6.device_check()


def test_few_supernova_calls_match_the_batch_kernel(ctx6, big_batch, torch):
    """Calls on at most 64 supernovae run more waves per supernova (forward: one per band; adjoint:
    one per band of a group); their fluxes, and the adjoint's gradients and chi-squares, are bitwise
    those of the same supernovae in the 4,096-supernova batch."""
    ev = synth.perturb(big_batch)
    g = np.random.default_rng(29)
    data = g.normal(size=ev.n_obs).astype(np.float32)
    w = np.abs(g.normal(size=ev.n_obs)).astype(np.float32)
    full = ctx6.bandflux(**to_dev(big_batch, torch)).cpu()
    run = lambda bb, dd, ww: ctx6.bandflux_vjp(**to_dev(bb, torch), chi2=True, data=torch.from_numpy(dd).cuda(),
                                                inv_sigma2=torch.from_numpy(ww).cuda(), want_flux=True)
    fullv = run(ev, data, w)
    for idx in (np.array([7]), np.arange(100, 110), np.arange(4032, 4096)):
        sel = np.concatenate([np.arange(big_batch.sn_offsets[i], big_batch.sn_offsets[i + 1]) for i in idx])
        part = ctx6.bandflux(**to_dev(big_batch.subset(idx), torch)).cpu()
        assert torch.equal(part, full[torch.from_numpy(sel)]), len(idx)
        pv = run(ev.subset(idx), data[sel], w[sel])
        ti = torch.from_numpy(idx).cuda()
        assert torch.equal(pv["grad"], fullv["grad"][ti]), len(idx)
        assert torch.equal(pv["chi2"], fullv["chi2"][ti]), len(idx)
        assert torch.equal(pv["flux"], fullv["flux"][torch.from_numpy(sel).cuda()]), len(idx)
    ctx6.device_check()


# ----------------------------------------------------------------------------- autograd

def test_autograd_function(ctx6, torch):
    from paper_2504_08081_amd.saltbf import salt_bandflux
    b = synth.random_batch(33, 20, 5, 60, synth.make_bands(6), synth.make_model())
    d = to_dev(b, torch)
    params = [d[k].clone().requires_grad_(True) for k in ("z", "t0", "x0", "x1", "c")]
    f = salt_bandflux(ctx6, *params, d["t"], d["band"], d["sn_offsets"])
    g = torch.randn_like(f)
    f.backward(g)
    r = ctx6.bandflux_vjp(**d, cotangent=g.contiguous())
    torch.cuda.synchronize()
    for q, p in enumerate(params):
        assert torch.equal(p.grad, r["grad"][:, q])
    # loose finite-difference sanity check in FP32 (FP32 differences cannot reach 1e-4)
    for q, h in ((3, 1e-2), (4, 1e-3)):
        pp = [x.detach().clone() for x in params]
        pm = [x.detach().clone() for x in params]
        pp[q] += h
        pm[q] -= h
        fp = ctx6.bandflux(*pp, d["t"], d["band"], d["sn_offsets"])
        fm = ctx6.bandflux(*pm, d["t"], d["band"], d["sn_offsets"])
        fd = ((fp - fm) * g).cpu().numpy().astype(np.float64)
        fd = oracle.segment_sum(fd, b.sn_offsets) / (2 * h)
        an = params[q].grad.cpu().numpy()
        assert np.max(np.abs(fd - an)) <= 1e-2 * np.max(np.abs(an))


# ----------------------------------------------------------------------------- closed forms through the GPU

def test_tiny_exact_case_gpu(sb, torch):
    import json
    import os
    from fractions import Fraction
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tiny_exact.json")))
    S = fx["surface"]
    ctx = sb.Context(np.float32(S["m0"]), np.float32(S["m1"]), S["phase0"], S["dphase"], S["wave0"], S["dwave"],
                     [0.0], 0.0, 1.0, max_spacing=fx["band"]["spacing"])
    ctx.add_band(fx["band"]["wave"], fx["band"]["trans"])
    P = fx["params"]
    b = synth.Batch(np.float32([P["z"]]), np.float32([P["t0"]]), np.float32([P["x0"]]), np.float32([P["x1"]]),
                    np.float32([P["c"]]), np.float32([fx["obs_t"]]), np.int32([0]), np.int32([0, 1]))
    f = run_fwd(ctx, b, torch)
    gold = Fraction(fx["expected_flux_times_hc"]["num"], fx["expected_flux_times_hc"]["den"])
    want = float(gold) / oracle.HC
    assert abs(f[0] - want) <= 2e-6 * want
    ctx.close()


@pytest.mark.parametrize("z", [0.05, 0.4, 0.9])
def test_flat_spectrum_tophat_gpu(sb, torch, z):
    """M0 = K, top-hat band: f = x0 K (b^2 - a^2) / (2 hc (1+z)) and df/dz = -f/(1+z)."""
    K = 0.75
    m0 = np.full((71, 721), K, np.float32)
    ctx = sb.Context(m0, np.zeros_like(m0), -20.0, 1.0, 2000.0, 10.0, [-0.9, 0.1, 0.01], 4302.57, 5428.55)
    a, bnd = 4000.0, 5230.0
    tb = synth.tophat_band(a, bnd)
    ctx.add_band(tb.wave, tb.trans)
    t = np.float32([3.0, 17.25, -9.5, 40.0])
    b = synth.Batch(np.float32([z]), np.float32([1.0]), np.float32([3e-5]), np.float32([0.0]), np.float32([0.0]),
                    t, np.zeros(4, np.int32), np.int32([0, 4]))
    f, J, _ = run_jac(ctx, b, torch)
    zf, x0f = float(np.float32(z)), float(np.float32(3e-5))
    want = x0f * K * (bnd ** 2 - a ** 2) / (2 * oracle.HC * (1 + zf))
    assert np.max(np.abs(f - want)) <= 1e-5 * want
    assert np.max(np.abs(J[:, 0] + want / (1 + zf))) <= 1e-4 * want
    ctx.close()


def test_midpoint_rule_context(sb, torch, model, bands6):
    """A context built with the midpoint quadrature rule against the oracle on the same rule:
    every flux, Jacobian row and gradient of a 64-supernova batch; and, on a flat spectrum with
    a top-hat band (linear integrand, where the midpoint rule is exact), the closed form."""
    ctx = sb.Context.from_model(model, bands6, quad_rule=sb.SB_QUAD_MIDPOINT)
    om = oracle.Oracle(model, bands6, rule="midpoint")
    b = synth.random_batch(43, 64, 1, 200, bands6, model)
    g = np.random.default_rng(11)
    cot = g.normal(size=b.n_obs).astype(np.float32)
    f, J, grad = run_jac(ctx, b, torch, cot)
    f64, J64 = om.jac(b)
    g64 = oracle.segment_sum(cot.astype(np.float64)[:, None] * J64, b.sn_offsets)
    ef = flux_rel_err(f, f64, b.sn_offsets)
    ej = jac_rel_err(J, J64, x0_per_obs(b), b.sn_offsets)
    en = grad_norm_err(grad, g64, b.x0)
    print(f"midpoint rule: flux {ef.max():.3e} jac {ej.max():.3e} grad norm-wise {en.max():.3e}")
    assert ef.max() <= FLUX_TOL and ej.max() <= GRAD_TOL and en.max() <= GRAD_TOL
    # the two rules differ by the quadrature error, far above FP32 rounding
    ft = oracle.Oracle(model, bands6).bandflux(b)
    assert np.max(np.abs(ft - f64) / np.abs(f64).max()) > 1e-5
    ctx.close()

    K = 0.75
    m0 = np.full((71, 721), K, np.float32)
    ctx = sb.Context(m0, np.zeros_like(m0), -20.0, 1.0, 2000.0, 10.0, [-0.9, 0.1, 0.01], 4302.57, 5428.55,
                     quad_rule=sb.SB_QUAD_MIDPOINT)
    a, bnd = 4000.0, 5230.0
    tb = synth.tophat_band(a, bnd)
    ctx.add_band(tb.wave, tb.trans)
    z = 0.4
    t = np.float32([3.0, 17.25, -9.5, 40.0])
    tb1 = synth.Batch(np.float32([z]), np.float32([1.0]), np.float32([3e-5]), np.float32([0.0]), np.float32([0.0]),
                      t, np.zeros(4, np.int32), np.int32([0, 4]))
    f, J, _ = run_jac(ctx, tb1, torch)
    zf, x0f = float(np.float32(z)), float(np.float32(3e-5))
    want = x0f * K * (bnd ** 2 - a ** 2) / (2 * oracle.HC * (1 + zf))
    assert np.max(np.abs(f - want)) <= 1e-5 * want
    assert np.max(np.abs(J[:, 0] + want / (1 + zf))) <= 1e-4 * want
    ctx.close()


# ----------------------------------------------------------------------------- edge cases

def test_edge_cases(ctx6, o6, torch, sb, model):
    """Empty supernovae, phases outside and on the edges of the grid, edge cells."""
    bands = synth.make_bands(6)
    zs = [0.0, 0.2, 0.5, 0.1]
    t_lists = [
        [-30.0, -20.0, -19.5, -19.0, 0.0, 49.5, 50.0, 50.5, 80.0],   # z=0: phases exact in FP32
        [],                                                        # empty supernova
        [-19.99, 49.99, 10.0],
        [5.0],
    ]
    ts, bs = [], []
    for z, tl in zip(zs, t_lists):
        ts.append(np.float32(np.array(tl) * (1 + np.float32(z))))
        bs.append(np.full(len(tl), 3, np.int32))
    off = np.zeros(len(zs) + 1, np.int32)
    off[1:] = np.cumsum([len(x) for x in ts])
    b = synth.Batch(np.float32(zs), np.float32(np.zeros(4)), np.float32([1e-5] * 4), np.float32([0.3, 0, -1, 2]),
                    np.float32([0.05, 0, -0.1, 0.2]), np.concatenate(ts).astype(np.float32),
                    np.concatenate(bs), off)
    f, J, grad = run_jac(ctx6, b, torch, np.ones(b.n_obs, np.float32))
    f64, J64 = o6.jac(b)
    assert np.all(f[f64 == 0] == 0)
    assert flux_rel_err(f, f64, b.sn_offsets).max() <= FLUX_TOL
    assert jac_rel_err(J, J64, x0_per_obs(b), b.sn_offsets).max() <= GRAD_TOL
    assert np.all(grad[1] == 0)
    ff = run_fwd(ctx6, b, torch)
    assert flux_rel_err(ff, f64, b.sn_offsets).max() <= FLUX_TOL
    # no supernova: nothing to do
    e = synth.Batch(np.float32([]), np.float32([]), np.float32([]), np.float32([]), np.float32([]),
                    np.float32([]), np.int32([]), np.int32([0]))
    d = to_dev(e, torch)
    ctx6.bandflux(**d)
    ctx6.device_check()


def test_band_windows_at_the_wavelength_edges(sb, model, torch):
    """Rest-frame band windows that reach the first and last wavelength cells of the surface, where
    the interpolation is linear (edge cells), against the oracle element by element: top-hat bands
    (full weight at their ends) starting exactly at 2,000 A and ending exactly at 9,200 A (z = 0, so
    the end nodes sit on the grid's first and last node), and at z = 0.05 bands whose rest windows
    end inside 9,190-9,200 A and start inside 2,000-2,010 A; forward, Jacobian rows and gradients."""
    bands = [synth.tophat_band(2000.0, 2900.0), synth.tophat_band(8500.0, 9200.0),
             synth.tophat_band(8400.0, 9650.0), synth.tophat_band(2105.0, 3000.0),
             synth.make_bands(1, 8350.0, 9655.0)[0]]
    ctx = sb.Context.from_model(model, bands)
    o = oracle.Oracle(model, bands)
    ph = np.array([-18.5, -15.0, -5.0, 0.0, 10.0, 25.0, 40.0, 49.0])
    ts, bs = [], []
    for z, bl in ((0.0, (0, 1)), (0.05, (2, 3, 4))):
        for bd in bl:
            ts.append(np.float32(30.0 + (1.0 + np.float32(z)) * ph))
            bs.append(np.full(len(ph), bd, np.int32))
    n0 = 2 * len(ph)
    b = synth.Batch(np.float32([0.0, 0.05]), np.float32([30.0, 30.0]), np.float32([2e-5, 1e-5]),
                    np.float32([0.4, -0.7]), np.float32([0.08, -0.05]), np.concatenate(ts), np.concatenate(bs),
                    np.int32([0, n0, n0 + 3 * len(ph)]))
    mu_hi = 9650.0 / (1.0 + float(np.float32(0.05)))
    assert 9190.0 < mu_hi < 9200.0 and 2000.0 < 2105.0 / (1.0 + float(np.float32(0.05))) < 2010.0
    cot = np.random.default_rng(41).normal(size=b.n_obs).astype(np.float32)
    f, J, grad = run_jac(ctx, b, torch, cot)
    f64, J64 = o.jac(b)
    g64 = oracle.segment_sum(cot.astype(np.float64)[:, None] * J64, b.sn_offsets)
    ef = flux_rel_err(f, f64, b.sn_offsets)
    ej = jac_rel_err(J, J64, x0_per_obs(b), b.sn_offsets)
    en = grad_norm_err(grad, g64, b.x0)
    print(f"edge windows: flux {ef.max():.3e} jac {ej.max():.3e} grad norm-wise {en.max():.3e}")
    assert np.all(np.isfinite(f)) and ef.max() <= FLUX_TOL
    assert ej.max() <= GRAD_TOL and en.max() <= GRAD_TOL
    assert flux_rel_err(run_fwd(ctx, b, torch), f64, b.sn_offsets).max() <= FLUX_TOL
    ctx.close()


def test_range_errors_are_flagged(ctx6, torch, sb):
    """A band id beyond the registry, or a rest window outside the surface, gives NaN and SB_ERR_RANGE."""
    ctx6.device_check()
    b = synth.Batch(np.float32([0.2, 0.95]), np.float32([0, 0]), np.float32([1e-5, 1e-5]), np.float32([0, 0]),
                    np.float32([0, 0]), np.float32([1.0, 2.0, 1.0, 2.0]), np.int32([1, 17, 0, 1]),
                    np.int32([0, 2, 4]))
    f = ctx6.bandflux(**to_dev(b, torch)).cpu().numpy()
    with pytest.raises(sb.SaltBFError) as e:
        ctx6.device_check()
    assert e.value.status == sb.SB_ERR_RANGE
    assert np.isfinite(f[0]) and np.isnan(f[1])     # band 17 does not exist
    assert np.isnan(f[2]) and np.isfinite(f[3])     # band 0 at z = 0.95 leaves the grid
    ctx6.device_check()                              # flags were cleared
    # malformed CSR offsets
    b2 = synth.Batch(np.float32([0.2]), np.float32([0]), np.float32([1e-5]), np.float32([0]), np.float32([0]),
                     np.float32([1.0]), np.int32([1]), np.int32([0, 5]))
    r = ctx6.bandflux_vjp(**to_dev(b2, torch), cotangent=torch.ones(1, device="cuda"))
    with pytest.raises(sb.SaltBFError):
        ctx6.device_check()
    assert np.all(np.isnan(r["grad"].cpu().numpy()))


def test_blueshifted_window_capacity(ctx6, o6, torch, sb):
    """Rest windows are sized for z >= -1/20: z = -0.04 matches the oracle; at z = -0.2 band 1's window
    (about 119 columns against a capacity of 105) exceeds it, which is flagged like any other range error."""
    ctx6.device_check()
    t = np.float32([-10.0, 0.0, 15.0, 30.0, -5.0, 5.0, 20.0])
    band = np.int32([1, 1, 3, 3, 1, 3, 1])
    b = synth.Batch(np.float32([-0.04]), np.float32([0.0]), np.float32([2e-5]), np.float32([0.4]),
                    np.float32([-0.05]), t, band, np.int32([0, 7]))
    f = ctx6.bandflux(**to_dev(b, torch)).cpu().numpy()
    ctx6.device_check()
    err = flux_rel_err(f, o6.bandflux(b), b.sn_offsets)
    assert err.max() <= FLUX_TOL, err
    b2 = synth.Batch(np.float32([-0.2]), np.float32([0.0]), np.float32([2e-5]), np.float32([0.0]),
                     np.float32([0.0]), np.float32([0.0]), np.int32([1]), np.int32([0, 1]))
    f2 = ctx6.bandflux(**to_dev(b2, torch)).cpu().numpy()
    with pytest.raises(sb.SaltBFError) as e:
        ctx6.device_check()
    assert e.value.status == sb.SB_ERR_RANGE and np.isnan(f2[0])


def test_host_argument_errors(ctx6, torch, sb):
    import ctypes
    b = synth.one_sn_40_obs()
    d = to_dev(b, torch)
    with pytest.raises(TypeError):
        ctx6.bandflux(**{**d, "t": d["t"].cpu()})
    with pytest.raises(TypeError):
        ctx6.bandflux_vjp(**d, cotangent=None)
    L = sb.lib()
    assert L.sb_bandflux(ctx6._h, None, None, None) == sb.SB_ERR_ARG
    batch = ctx6._batch(d["z"], d["t0"], d["x0"], d["x1"], d["c"], d["t"], d["band"], d["sn_offsets"],
                        False, None, None, False)
    assert L.sb_bandflux(ctx6._h, ctypes.byref(batch), None, None) == sb.SB_ERR_ARG
    batch.flags = 64
    out = torch.empty(b.n_obs, device="cuda")
    assert L.sb_bandflux(ctx6._h, ctypes.byref(batch), ctypes.c_void_p(out.data_ptr()), None) == sb.SB_ERR_ARG
    assert len(L.sb_last_error()) > 0


# ----------------------------------------------------------------------------- sweep (one observation table, many samples)

def _sweep_data(sw, o6):
    n_obs = len(sw.obs_t)
    f_true = o6.bandflux(synth.Batch(np.float32([sw.theta_true[0]]), np.float32([sw.theta_true[1]]),
                                     np.float32([sw.theta_true[2]]), np.float32([sw.theta_true[3]]),
                                     np.float32([sw.theta_true[4]]), sw.obs_t, sw.obs_band, np.int32([0, n_obs])))
    data, _, w = synth.make_data(f_true, [0, n_obs], synth.noise_draws(n_obs, k=55))
    return data, w


def _sweep_batch(sw, idx):
    """The samples idx of a sweep as a plain batch (the shared observation table repeated)."""
    smp, no, m = sw.samples, len(sw.obs_t), len(idx)
    return synth.Batch(smp.z[idx], smp.t0[idx], smp.x0[idx], smp.x1[idx], smp.c[idx], np.tile(sw.obs_t, m),
                       np.tile(sw.obs_band, m), np.arange(0, (m + 1) * no, no, dtype=np.int32))


def test_sweep_matches_plain_kernel_and_oracle(ctx6, o6, torch):
    """Broadcast sweep == per-supernova kernel on the materialised batch (bitwise), and on 16,384
    seeded samples every flux and chi-square against the oracle (run over all samples on a pool of
    CPU processes)."""
    sw = synth.sweep_120_obs(n_samples=16384)
    smp = sw.samples
    n_obs = len(sw.obs_t)
    data, w = _sweep_data(sw, o6)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P = dict(z=dv(smp.z), t0=dv(smp.t0), x0=dv(smp.x0), x1=dv(smp.x1), c=dv(smp.c))
    t, band = dv(sw.obs_t), dv(sw.obs_band)
    chi_sw = ctx6.bandflux(**P, t=t, band=band, broadcast=True, chi2=True, data=dv(data), inv_sigma2=dv(w))
    flux_sw = ctx6.bandflux(**P, t=t, band=band, broadcast=True)
    # the same work as a plain CSR batch
    n = smp.n_sn
    tt = t.repeat(n)
    bb = band.repeat(n)
    off = torch.arange(0, (n + 1) * n_obs, n_obs, dtype=torch.int32, device="cuda")
    chi_pl = ctx6.bandflux(**P, t=tt, band=bb, sn_offsets=off, chi2=True, data=dv(data).repeat(n),
                           inv_sigma2=dv(w).repeat(n))
    flux_pl = ctx6.bandflux(**P, t=tt, band=bb, sn_offsets=off)
    ctx6.device_check()
    assert torch.equal(chi_sw, chi_pl)
    assert torch.equal(flux_sw.reshape(-1), flux_pl)
    # every sample against the oracle
    mb = _sweep_batch(sw, np.arange(n))
    f64 = oracle_over_batch("flux", mb, 6, chunk=256)
    F = flux_sw.cpu().numpy().reshape(-1)
    C = chi_sw.cpu().numpy()
    ef = flux_rel_err(F, f64, mb.sn_offsets)
    c64 = ((f64.reshape(n, n_obs) - data) ** 2 * w).sum(axis=1)
    ec = np.abs(C - c64) / c64
    print(f"sweep, {n} samples x {n_obs} obs: flux {ef.max():.3e} (p99 {np.percentile(ef, 99):.3e}), "
          f"chi2 {ec.max():.3e}")
    assert ef.max() <= FLUX_TOL
    assert ec.max() <= 1e-5
    # adjoint sweep against the per-supernova adjoint
    g_sw = ctx6.bandflux_vjp(**P, t=t, band=band, broadcast=True, chi2=True, data=dv(data), inv_sigma2=dv(w))
    g_pl = ctx6.bandflux_vjp(**P, t=tt, band=bb, sn_offsets=off, chi2=True, data=dv(data).repeat(n),
                             inv_sigma2=dv(w).repeat(n))
    torch.cuda.synchronize()
    assert torch.equal(g_sw["grad"], g_pl["grad"]) and torch.equal(g_sw["chi2"], g_pl["chi2"])
    # the persistent launch (each workgroup striding over several samples): bitwise the same
    chi_ps = ctx6.bandflux(**P, t=t, band=band, broadcast="persistent", chi2=True, data=dv(data), inv_sigma2=dv(w))
    flux_ps = ctx6.bandflux(**P, t=t, band=band, broadcast="persistent")
    g_ps = ctx6.bandflux_vjp(**P, t=t, band=band, broadcast="persistent", chi2=True, data=dv(data),
                             inv_sigma2=dv(w))
    ctx6.device_check()
    assert torch.equal(chi_ps, chi_sw) and torch.equal(flux_ps, flux_sw)
    assert torch.equal(g_ps["grad"], g_sw["grad"]) and torch.equal(g_ps["chi2"], g_sw["chi2"])


def test_persistent_sweep_with_fewer_samples_than_workgroups(ctx6, torch, sb):
    """Seven and 4,099 samples (grids of one workgroup per sample, the grid's cap not reached): the
    persistent sweep equals the one-workgroup-per-sample sweep; SB_PERSISTENT without
    SB_OBS_BROADCAST is an argument error.  Workgroups striding over several samples are checked at
    full size (test_sweep_full_size_sampled: 1,048,576 samples, 16 per workgroup on an MI355X)."""
    sw = synth.sweep_120_obs(n_samples=4099)
    smp = sw.samples
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    t, band = dv(sw.obs_t), dv(sw.obs_band)
    for n in (7, 4099):
        P = dict(z=dv(smp.z[:n]), t0=dv(smp.t0[:n]), x0=dv(smp.x0[:n]), x1=dv(smp.x1[:n]), c=dv(smp.c[:n]))
        a = ctx6.bandflux(**P, t=t, band=band, broadcast=True)
        b = ctx6.bandflux(**P, t=t, band=band, broadcast="persistent")
        ctx6.device_check()
        assert torch.equal(a, b), n
    import ctypes
    P = dict(z=dv(smp.z[:7]), t0=dv(smp.t0[:7]), x0=dv(smp.x0[:7]), x1=dv(smp.x1[:7]), c=dv(smp.c[:7]))
    off = torch.zeros(8, dtype=torch.int32, device="cuda")
    batch = ctx6._batch(P["z"], P["t0"], P["x0"], P["x1"], P["c"], t, band, off, False, None, None, False)
    batch.flags = sb.SB_PERSISTENT
    out = torch.empty(len(sw.obs_t), device="cuda")
    assert sb.lib().sb_bandflux(ctx6._h, ctypes.byref(batch), ctypes.c_void_p(out.data_ptr()), None) == sb.SB_ERR_ARG


def test_sweep_full_size_sampled(ctx6, o6, torch):
    """The full sweep (1,048,576 samples x 120 observations) as the benchmark launches it, chi-square
    and flux outputs: 256 seeded samples against the oracle, every chi-square finite, and the
    persistent launch's chi-squares bitwise those of the one-workgroup-per-sample launch."""
    print("case: full sweep 1048576 x 120", flush=True)
    sw = synth.sweep_120_obs()
    smp = sw.samples
    n, n_obs = smp.n_sn, len(sw.obs_t)
    data, w = _sweep_data(sw, o6)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P = dict(z=dv(smp.z), t0=dv(smp.t0), x0=dv(smp.x0), x1=dv(smp.x1), c=dv(smp.c))
    t, band = dv(sw.obs_t), dv(sw.obs_band)
    chi = ctx6.bandflux(**P, t=t, band=band, broadcast=True, chi2=True, data=dv(data), inv_sigma2=dv(w))
    chi_ps = ctx6.bandflux(**P, t=t, band=band, broadcast="persistent", chi2=True, data=dv(data), inv_sigma2=dv(w))
    flux = ctx6.bandflux(**P, t=t, band=band, broadcast=True)
    ctx6.device_check()
    assert torch.equal(chi, chi_ps)
    C = chi.cpu().numpy()
    assert np.all(np.isfinite(C))
    pick = np.sort(np.random.default_rng(77).choice(n, 256, replace=False))
    F = flux[torch.from_numpy(pick).cuda()].cpu().numpy().reshape(-1)
    mb = _sweep_batch(sw, pick)
    f64 = o6.bandflux(mb)
    ef = flux_rel_err(F, f64, mb.sn_offsets)
    c64 = ((f64.reshape(len(pick), n_obs) - data) ** 2 * w).sum(axis=1)
    ec = np.abs(C[pick] - c64) / c64
    print(f"full sweep sampled 256: flux {ef.max():.3e} chi2 {ec.max():.3e}")
    assert ef.max() <= FLUX_TOL and ec.max() <= 1e-5

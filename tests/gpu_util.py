"""Helpers of the GPU tests: moving synthetic batches to the device, error metrics."""
import numpy as np
import pytest

FLUX_TOL = 1e-5    # max relative error of an FP32 flux against the FP64 oracle
GRAD_TOL = 1e-4    # max relative error of an FP32 (scaled) gradient against the FP64 oracle
PARAM_SCALE = np.array([0.1, 1.0, 1.0, 1.0, 0.1])   # z, t0 [d], x0 (times x0), x1, c


def torch_or_skip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def to_dev(batch, torch):
    d = "cuda"
    return dict(z=torch.from_numpy(np.ascontiguousarray(batch.z, np.float32)).to(d),
                t0=torch.from_numpy(np.ascontiguousarray(batch.t0, np.float32)).to(d),
                x0=torch.from_numpy(np.ascontiguousarray(batch.x0, np.float32)).to(d),
                x1=torch.from_numpy(np.ascontiguousarray(batch.x1, np.float32)).to(d),
                c=torch.from_numpy(np.ascontiguousarray(batch.c, np.float32)).to(d),
                t=torch.from_numpy(np.ascontiguousarray(batch.t, np.float32)).to(d),
                band=torch.from_numpy(np.ascontiguousarray(batch.band, np.int32)).to(d),
                sn_offsets=torch.from_numpy(np.ascontiguousarray(batch.sn_offsets, np.int32)).to(d))


def flux_rel_err(f_gpu, f64, offsets):
    """|f - f64| / max(|f64|, 1e-3 max_{j in SN} |f64_j|), per observation."""
    f_gpu = np.asarray(f_gpu, np.float64)
    f64 = np.asarray(f64, np.float64)
    floor = np.zeros_like(f64)
    for s in range(len(offsets) - 1):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        if hi > lo:
            floor[lo:hi] = 1e-3 * np.abs(f64[lo:hi]).max()
    den = np.maximum(np.abs(f64), floor)
    den = np.where(den > 0, den, 1.0)
    return np.abs(f_gpu - f64) / den


def grad_rel_err(g_gpu, g64, x0):
    """Scaled gradients g * (0.1, 1 d, x0, 1, 0.1); per supernova and component, relative to
    max(|g64|, 1e-3 * max over the supernova's components)."""
    sc = PARAM_SCALE[None, :] * np.ones((len(x0), 1))
    sc[:, 2] = np.asarray(x0, np.float64)
    a = np.asarray(g_gpu, np.float64) * sc
    b = np.asarray(g64, np.float64) * sc
    floor = 1e-3 * np.abs(b).max(axis=1, keepdims=True)
    den = np.maximum(np.abs(b), floor)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - b) / den


def jac_rel_err(j_gpu, j64, x0_per_obs, offsets=None):
    """Per-observation scaled Jacobian rows: relative error with a floor at 1e-2 of the row's largest
    scaled partial.  Each partial of the bandflux is a signed combination of terms bounded by that
    row scale (the z partial, for one, cancels an amplitude term against a wavelength-stretch term),
    and FP32 sums of node values give those terms ~1e-6 of the row scale; the floor turns the 1e-4
    relative bound into a 1e-6 row-scale bound for entries that cancel to near zero."""
    sc = PARAM_SCALE[None, :] * np.ones((len(x0_per_obs), 1))
    sc[:, 2] = x0_per_obs
    a = np.asarray(j_gpu, np.float64) * sc
    b = np.asarray(j64, np.float64) * sc
    floor = 1e-2 * np.abs(b).max(axis=1, keepdims=True)
    den = np.maximum(np.abs(b), floor)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - b) / den


def grad_norm_err(g_gpu, g64, x0):
    """Norm-wise error per supernova: max_q |g~ - g~64| / max_q |g~64| on scaled gradients."""
    sc = PARAM_SCALE[None, :] * np.ones((len(x0), 1))
    sc[:, 2] = np.asarray(x0, np.float64)
    a = np.asarray(g_gpu, np.float64) * sc
    b = np.asarray(g64, np.float64) * sc
    den = np.abs(b).max(axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.abs(a - b).max(axis=1) / den


U32 = 2.0 ** -24


def grad_propagated_excess(g_gpu, g64, x0, offsets, cot64, J64, J_gpu, cot_err=None, c=4.0):
    """Component error of a gradient g_q = sum_i cot_i J_iq over the error that the MEASURED errors
    of its inputs propagate into it, plus the rounding of the FP32 sum itself:
        B_q = sum_i |dcot_i| |J~_iq| + sum_i |cot_i| |J~_gpu,iq - J~_64,iq| + c u sum_i |cot_i J~_iq|
    on scaled parameters, with dcot_i the cotangent's own error (0 for a cotangent given exactly;
    2 w_i |f_gpu,i - f_64,i| for a chi-square cotangent 2 (f_i - d_i) w_i formed from the GPU flux).
    Each Jacobian row and flux is held to its own bound elsewhere; this checks that the gradient
    adds no error beyond what those rows and fluxes carry.  Values <= 1 pass."""
    sc = PARAM_SCALE[None, :] * np.ones((len(x0), 1))
    sc[:, 2] = np.asarray(x0, np.float64)
    n_s = np.diff(offsets)
    sc_obs = np.repeat(sc, n_s, axis=0)
    Jt = np.asarray(J64, np.float64) * sc_obs
    dJ = np.abs(np.asarray(J_gpu, np.float64) * sc_obs - Jt)
    cot = np.abs(np.asarray(cot64, np.float64))
    dc = np.zeros_like(cot) if cot_err is None else np.abs(np.asarray(cot_err, np.float64))
    off = np.asarray(offsets, np.int64)

    def seg(v):   # per-supernova sums of the rows of v
        cs = np.vstack([np.zeros((1, v.shape[1])), np.cumsum(v, axis=0)])
        return cs[off[1:]] - cs[off[:-1]]

    bound = seg(dc[:, None] * np.abs(Jt)) + seg(cot[:, None] * dJ) + c * U32 * seg(cot[:, None] * np.abs(Jt))
    err = np.abs((np.asarray(g_gpu, np.float64) - np.asarray(g64, np.float64)) * sc)
    return err / np.maximum(bound, 1e-300)


# ----------------------------------------------------------------------------- the oracle over a whole batch

def _oracle_chunk(args):
    """Worker: the oracle's fluxes, or chi-square and its gradient, for one chunk of supernovae."""
    import oracle
    import synth
    kind, batch, data, w, n_bands = args
    o = oracle.Oracle(synth.make_model(), synth.make_bands(n_bands))
    if kind == "flux":
        return o.bandflux(batch)
    if kind == "jac":
        return o.jac(batch)
    return o.chi2_grad(batch, data, w)


def oracle_over_batch(kind, batch, n_bands, data=None, w=None, workers=16, chunk=128):
    """The FP64 oracle over every supernova of a batch, in chunks on a pool of CPU worker
    processes (started with spawn, so they share nothing with the GPU process).
    kind "flux": fluxes [n_obs]; kind "jac": (fluxes [n_obs], Jacobian rows [n_obs, 5]);
    kind "chi2": (fluxes [n_obs], chi2 [n_sn], gradient [n_sn, 5])."""
    import multiprocessing as mp
    import os
    jobs = []
    for lo in range(0, batch.n_sn, chunk):
        idx = np.arange(lo, min(batch.n_sn, lo + chunk))
        sub = batch.subset(idx)
        a, b = batch.sn_offsets[lo], batch.sn_offsets[idx[-1] + 1]
        jobs.append((kind, sub, None if data is None else data[a:b], None if w is None else w[a:b], n_bands))
    n = max(1, min(workers, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(n) as pool:
        out = pool.map(_oracle_chunk, jobs)
    if kind == "flux":
        return np.concatenate(out)
    if kind == "jac":
        return np.concatenate([o[0] for o in out]), np.concatenate([o[1] for o in out])
    return (np.concatenate([o[0] for o in out]), np.concatenate([o[1] for o in out]),
            np.concatenate([o[2] for o in out]))


# Worst relative FP32 flux error measured against the oracle: 3.85e-7 over all 447,402 fluxes of the
# 4,096-supernova batch (test_batch_4096_every_flux_chi2_and_gradient).
FLUX_ERR_MEASURED = 4e-7


def fit_resolution(f64, data, w, chi2, flux_err=FLUX_ERR_MEASURED):
    """How closely an FP32 fit can place its optimum, in units of the parameters' uncertainty (R27).
    The FP32 chi-square carries an error e of about sqrt(n) 2^-24 chi2 from its sum and
    2 flux_err sqrt(sum_i (r_i w_i f_i)^2) from the fluxes' relative error (independent signs; r, f at
    the FP64 optimum), and a step of u sigma changes chi2 by u^2, so the fit cannot order two points
    closer than u = sqrt(2 e)."""
    f64 = np.asarray(f64, np.float64)
    r = np.asarray(data, np.float64) - f64
    w = np.asarray(w, np.float64)
    e = np.sqrt(len(f64)) * 2.0 ** -24 * chi2 + 2.0 * flux_err * np.sqrt(np.sum((r * w * f64) ** 2))
    return float(np.sqrt(2.0 * e))

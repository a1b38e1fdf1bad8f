"""Seeded synthetic inputs for the SALT bandflux path.

This module only draws inputs: model surfaces on their grid, filter
transmission samples, supernova parameters, observation times and band ids,
noise draws and request streams.  It contains none of the method's
arithmetic (no interpolation, no colour law evaluation, no quadrature, no
flux).  Both the FP64 oracle (``oracle/``) and the GPU library are fed from
here; quantities that need a model flux (noisy data, flux errors) are built
by the caller from a flux it computed itself, through :func:`make_data`.

All random numbers come from ``numpy.random.Generator(PCG64(SEED + k))``:
k = 0 draws the model, k = 1..5 draw the five workloads below, larger k are free for
tests.  Every floating value the GPU receives is first rounded to float32
here, so both sides start from identical numbers.

Workload recipes (sizes, distributions) follow the paper's statement of the
model (section "Implementation": model equation with free parameters
x0, x1, t0, c; bandflux integral through a filter T) with synthetic stand-ins
for the trained SALT surfaces and the built-in filters, which are not public
inputs of this project.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

SEED = 250408081

# Surface grid: phase -20..50 d at 1 d, rest wavelength 2000..9200 A at 10 A.
PHASE0, DPHASE, NPHASE = -20.0, 1.0, 71
WAVE0, DWAVE, NWAVE = 2000.0, 10.0, 721
# Reference wavelengths of the colour-law variable r = (mu - B)/(V - B).
CL_WAVE_B, CL_WAVE_V = 4302.57, 5428.55
# Quadrature spacing bound of the observer-frame grid (Angstrom).
MAX_SPACING = 5.0
# Keep a band's rest-frame window this far (Angstrom) inside the surface grid,
# so that float32 and float64 agree on eligibility and the redshift steps of
# perturb() (|dz| <= 3e-3, which move the window's blue end by at most 3.5 A
# where a band can reach the grid's edge) keep every window on the grid.
ELIG_MARGIN = 6.0


def rng(k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED + k))


def f32(a):
    return np.asarray(a, dtype=np.float32)


def f32r(a):
    """Round to float32 but keep a float64 container (exactly representable)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclass
class Model:
    m0: np.ndarray  # float32 [n_phase, n_wave]
    m1: np.ndarray  # float32 [n_phase, n_wave]
    phase0: float = PHASE0
    dphase: float = DPHASE
    wave0: float = WAVE0
    dwave: float = DWAVE
    cl_coef: np.ndarray = field(default_factory=lambda: np.zeros(3))  # float32-exact, float64 container
    cl_wave_b: float = CL_WAVE_B
    cl_wave_v: float = CL_WAVE_V

    @property
    def n_phase(self):
        return self.m0.shape[0]

    @property
    def n_wave(self):
        return self.m0.shape[1]

    @property
    def wave_max(self):
        return self.wave0 + (self.n_wave - 1) * self.dwave

    @property
    def phase_max(self):
        return self.phase0 + (self.n_phase - 1) * self.dphase


@dataclass
class Band:
    wave: np.ndarray   # float64 [n] increasing (Angstrom)
    trans: np.ndarray  # float64 [n] in [0, 1]

    @property
    def lo(self):
        return float(self.wave[0])

    @property
    def hi(self):
        return float(self.wave[-1])


@dataclass
class Batch:
    """Structure-of-arrays batch: per-supernova parameters and CSR observations."""
    z: np.ndarray
    t0: np.ndarray
    x0: np.ndarray
    x1: np.ndarray
    c: np.ndarray
    t: np.ndarray
    band: np.ndarray
    sn_offsets: np.ndarray

    @property
    def n_sn(self):
        return int(self.z.shape[0])

    @property
    def n_obs(self):
        return int(self.t.shape[0])

    def params(self):
        return np.stack([self.z, self.t0, self.x0, self.x1, self.c], axis=1)

    def subset(self, sn_idx):
        """Batch made of the listed supernovae (in the given order)."""
        sn_idx = np.asarray(sn_idx, dtype=np.int64)
        lo = self.sn_offsets[sn_idx].astype(np.int64)
        hi = self.sn_offsets[sn_idx + 1].astype(np.int64)
        sel = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]) if len(sn_idx) else np.zeros(0, np.int64)
        off = np.zeros(len(sn_idx) + 1, np.int32)
        off[1:] = np.cumsum(hi - lo)
        return Batch(self.z[sn_idx], self.t0[sn_idx], self.x0[sn_idx], self.x1[sn_idx], self.c[sn_idx],
                     self.t[sel], self.band[sel], off)

    def with_params(self, z=None, t0=None, x0=None, x1=None, c=None):
        return Batch(f32(self.z if z is None else z), f32(self.t0 if t0 is None else t0),
                     f32(self.x0 if x0 is None else x0), f32(self.x1 if x1 is None else x1),
                     f32(self.c if c is None else c), self.t, self.band, self.sn_offsets)


# ----------------------------------------------------------------------------- model

def _smooth_field(g: np.random.Generator, p, mu, n_modes=64):
    """Unit-variance smooth random field on the (phase, wavelength) grid."""
    wp = g.normal(0.0, 1.0 / 10.0, n_modes)
    wm = g.normal(0.0, 1.0 / 400.0, n_modes)
    ph = g.uniform(0.0, 2.0 * np.pi, n_modes)
    arg = wp[:, None, None] * p[None, :, None] + wm[:, None, None] * mu[None, None, :] + ph[:, None, None]
    return np.sqrt(2.0 / n_modes) * np.cos(arg).sum(axis=0)


def make_model(k: int = 0, n_wave: int = NWAVE) -> Model:
    """Synthetic SALT-shaped surfaces M0 > 0, M1 ~ 0.1*M0*N(0,1), cubic colour law; n_wave columns
    at 10 A from 2000 A (721: to 9200 A; 2001: to 22000 A, a near-infrared-wide grid)."""
    g = rng(k)
    p = PHASE0 + DPHASE * np.arange(NPHASE)
    mu = WAVE0 + DWAVE * np.arange(n_wave)
    x = 14387.77 / mu                         # 1e4 K black-body shape
    planck = mu ** -5 / np.expm1(x)
    planck /= planck.max()
    g0 = _smooth_field(g, p, mu)
    g1 = _smooth_field(g, p, mu)
    lc = np.exp(-0.5 * (p / 10.0) ** 2) + 0.05
    m0 = planck[None, :] * lc[:, None] * np.exp(0.1 * g0)
    m1 = 0.1 * m0 * g1
    a1 = -0.4 * np.log(10.0) * (1.0 + 0.1 * g.normal())
    a2 = 0.05 * g.normal()
    a3 = 0.005 * g.normal()
    return Model(m0=f32(m0), m1=f32(m1), cl_coef=f32r([a1, a2, a3]))


def make_bands(n_b: int, lo: float = 3500.0, hi: float = 9000.0, n_samples: int = 200,
               edge_sigma: float = 25.0) -> List[Band]:
    """n_b Gaussian-edged top-hats with equal supports tiling [lo, hi]."""
    bands = []
    width = (hi - lo) / n_b
    for b in range(n_b):
        L = lo + b * width
        U = L + width
        w = np.linspace(L, U, n_samples)
        core_lo, core_hi = L + 4 * edge_sigma, U - 4 * edge_sigma
        tr = np.ones_like(w)
        m = w < core_lo
        tr[m] = np.exp(-0.5 * ((w[m] - core_lo) / edge_sigma) ** 2)
        m = w > core_hi
        tr[m] = np.exp(-0.5 * ((w[m] - core_hi) / edge_sigma) ** 2)
        bands.append(Band(wave=w, trans=tr))
    return bands


def nir_bands() -> List[Band]:
    """Stand-ins for near-infrared filters (Y, J, H-like supports), Gaussian-edged like make_bands."""
    out = []
    for lo, hi in ((9400.0, 11200.0), (11200.0, 13800.0), (14600.0, 18200.0)):
        out += make_bands(1, lo, hi, n_samples=300, edge_sigma=40.0)
    return out


def write_band_file(path, band: Band, header: str = "") -> None:
    """A two-column text file of the band's samples at full float64 precision (what a filter file
    on disk looks like: comments, then wavelength and transmission per line)."""
    with open(path, "w") as fh:
        if header:
            fh.write("".join(f"# {ln}\n" for ln in header.splitlines()))
        for w, t in zip(band.wave, band.trans):
            fh.write(f"{float(w)!r} {float(t)!r}\n")


def tophat_band(a: float, b: float, n_samples: int = 200) -> Band:
    return Band(wave=np.linspace(a, b, n_samples), trans=np.ones(n_samples))


def eligible_bands(z: float, bands: List[Band], model: Model, margin: float = ELIG_MARGIN):
    """Bands whose rest-frame window [lo/(1+z), hi/(1+z)] lies inside the surface grid."""
    out = []
    for i, bd in enumerate(bands):
        if bd.lo / (1.0 + z) >= model.wave0 + margin and bd.hi / (1.0 + z) <= model.wave_max - margin:
            out.append(i)
    return out


# ----------------------------------------------------------------------------- workloads

def _finish(z, t0, x0, x1, c, per_sn_t, per_sn_band):
    n = np.array([len(a) for a in per_sn_t], dtype=np.int64)
    off = np.zeros(len(n) + 1, np.int32)
    off[1:] = np.cumsum(n)
    t = np.concatenate(per_sn_t) if len(n) else np.zeros(0)
    b = np.concatenate(per_sn_band) if len(n) else np.zeros(0)
    return Batch(f32(z), f32(t0), f32(x0), f32(x1), f32(c), f32(t), np.asarray(b, np.int32), off)


def _sorted_obs(t, b):
    order = np.lexsort((t, b))
    return t[order], b[order]


def one_sn_40_obs() -> Batch:
    """1 supernova, 40 observations: 4 bands x 10 rest phases -15..45."""
    z, t0, x0, x1, c = 0.1, 0.0, 1e-5, 0.5, 0.05
    zf = float(np.float32(z))
    ph = np.linspace(-15.0, 45.0, 10)
    ts, bs = [], []
    for b in range(4):
        ts.append(t0 + (1.0 + zf) * ph)
        bs.append(np.full(10, b))
    t, bb = _sorted_obs(f32(np.concatenate(ts)).astype(np.float64), np.concatenate(bs))
    return _finish([z], [t0], [x0], [x1], [c], [t], [bb])


def draw_params(g: np.random.Generator, n: int, zlo=0.01, zhi=1.0):
    z = g.uniform(zlo, zhi, n)
    x1 = g.normal(0.0, 1.0, n)
    c = g.normal(0.0, 0.1, n)
    x0 = 10.0 ** g.uniform(-6.0, -4.0, n)
    t0 = g.uniform(0.0, 365.0, n)
    return z, t0, x0, x1, c


def random_batch(k: int, n_sn: int, nobs_lo: int, nobs_hi: int, bands: List[Band], model: Model,
                 phase_lo=-15.0, phase_hi=45.0, fixed_nobs=None, zlo=0.01, zhi=1.0) -> Batch:
    """Uneven light curves: n_s ~ U{lo..hi}, rest phases ~ U(phase_lo, phase_hi), eligible bands."""
    g = rng(k)
    z, t0, x0, x1, c = draw_params(g, n_sn, zlo, zhi)
    zf = f32r(z)
    ts, bs = [], []
    for s in range(n_sn):
        ns = fixed_nobs if fixed_nobs is not None else int(g.integers(nobs_lo, nobs_hi + 1))
        el = np.array(eligible_bands(zf[s], bands, model))
        ph = g.uniform(phase_lo, phase_hi, ns)
        bb = el[g.integers(0, len(el), ns)]
        tt = f32(t0[s]).astype(np.float64) + (1.0 + zf[s]) * ph
        tt, bb = _sorted_obs(f32(tt).astype(np.float64), bb)
        ts.append(tt)
        bs.append(bb)
    return _finish(z, t0, x0, x1, c, ts, bs)


def batch_4096_sn(n_sn: int = 4096, k: int = 2) -> Batch:
    """4,096 supernovae, n_s ~ U{20..200} observations, 6 bands, broad priors."""
    return random_batch(k, n_sn, 20, 200, make_bands(6), make_model())


def perturb(batch: Batch, k: int = 3, scale: float = 1.0) -> Batch:
    """Parameters moved off the truth: the point where workload-3 gradients are taken."""
    g = rng(k)
    n = batch.n_sn
    dz = np.clip(g.normal(0.0, 1e-3, n), -3e-3, 3e-3) * scale
    dt0 = g.normal(0.0, 1.0, n) * scale
    dx1 = g.normal(0.0, 0.2, n) * scale
    dc = g.normal(0.0, 0.02, n) * scale
    fx0 = 1.0 + g.normal(0.0, 0.05, n) * scale
    return batch.with_params(z=batch.z.astype(np.float64) + dz, t0=batch.t0.astype(np.float64) + dt0,
                             x0=batch.x0.astype(np.float64) * fx0, x1=batch.x1.astype(np.float64) + dx1,
                             c=batch.c.astype(np.float64) + dc)


def noise_draws(n_obs: int, k: int = 13) -> np.ndarray:
    return rng(k).normal(0.0, 1.0, n_obs)


def make_data(f_true, sn_offsets, normals):
    """Noisy data d = f + sigma*n with sigma = 5% of the flux, floored at 1% of the SN's peak flux.

    The caller supplies the true flux (from its own model evaluation).  Returns
    float32 arrays (data, sigma, inv_sigma2)."""
    f_true = np.asarray(f_true, np.float64)
    sig = np.empty_like(f_true)
    for s in range(len(sn_offsets) - 1):
        lo, hi = int(sn_offsets[s]), int(sn_offsets[s + 1])
        if hi <= lo:
            continue
        fa = np.abs(f_true[lo:hi])
        sig[lo:hi] = 0.05 * np.maximum(fa, 0.01 * fa.max())
    sig = np.where(sig > 0, sig, 1.0)
    d = f_true + sig * np.asarray(normals, np.float64)[: len(f_true)]
    sig32 = f32(sig)
    return f32(d), sig32, f32(1.0 / sig32.astype(np.float64) ** 2)


@dataclass
class FitRequest:
    arrival: float
    z: float
    theta_true: np.ndarray   # (t0, x0, x1, c)
    theta_init: np.ndarray   # (t0, x0, x1, c)
    t: np.ndarray
    band: np.ndarray
    normals: np.ndarray


def fit_requests(n_req: int, rate: float = 2000.0, k: int = 4, nobs_lo=8, nobs_hi=256) -> List[FitRequest]:
    """Poisson-arriving single-supernova fit requests with 8-256 observations in 2-6 bands."""
    g = rng(k)
    bands = make_bands(6)
    model = make_model()
    arr = np.cumsum(g.exponential(1.0 / rate, n_req))
    out = []
    for r in range(n_req):
        z, t0, x0, x1, c = (a[0] for a in draw_params(g, 1))
        zf = float(np.float32(z))
        el = eligible_bands(zf, bands, model)
        nb = int(g.integers(2, 7))
        nb = min(nb, len(el))
        chosen = np.sort(g.choice(el, nb, replace=False))
        ns = int(g.integers(nobs_lo, nobs_hi + 1))
        ph = g.uniform(-15.0, 45.0, ns)
        bb = chosen[g.integers(0, nb, ns)]
        tt = float(np.float32(t0)) + (1.0 + zf) * ph
        tt, bb = _sorted_obs(f32(tt).astype(np.float64), bb)
        th = f32r([t0, x0, x1, c])
        init = f32r([t0 + 3 * g.normal(0, 1.0), x0 * (1 + 3 * g.normal(0, 0.05)),
                     x1 + 3 * g.normal(0, 0.2), c + 3 * g.normal(0, 0.02)])
        init[1] = abs(init[1])
        out.append(FitRequest(float(arr[r]), zf, th, init, f32(tt), bb.astype(np.int32), g.normal(0, 1, ns)))
    return out


@dataclass
class Sweep:
    obs_t: np.ndarray       # float32 [n_obs]
    obs_band: np.ndarray    # int32 [n_obs]
    theta_true: np.ndarray  # (z, t0, x0, x1, c)
    samples: Batch          # n_sn = n_samples, no observations of its own (t, band empty)


def sweep_120_obs(n_samples: int = 1 << 20, k: int = 5) -> Sweep:
    """1 supernova with 120 observations in 6 bands, evaluated at many parameter samples."""
    g = rng(k)
    z, t0 = 0.1, 100.0
    zf = float(np.float32(z))
    ph = np.linspace(-10.0, 40.0, 20)
    ts, bs = [], []
    for b in range(6):
        ts.append(t0 + (1.0 + zf) * ph)
        bs.append(np.full(20, b))
    t, bb = _sorted_obs(f32(np.concatenate(ts)).astype(np.float64), np.concatenate(bs))
    zs = g.uniform(0.01, 0.74, n_samples)
    t0s = t0 + g.uniform(-5.0, 5.0, n_samples)
    x1s = g.normal(0.0, 1.0, n_samples)
    cs = g.normal(0.0, 0.1, n_samples)
    x0s = 10.0 ** g.uniform(-6.0, -4.0, n_samples)
    smp = Batch(f32(zs), f32(t0s), f32(x0s), f32(x1s), f32(cs), f32([]), np.zeros(0, np.int32),
                np.zeros(n_samples + 1, np.int32))
    return Sweep(f32(t), bb.astype(np.int32), f32r([z, t0, 1e-5, 0.5, 0.05]), smp)


def batch_65536_sn(n_sn: int = 65536, k: int = 6) -> Batch:
    """65,536 supernovae x 100 observations, broad priors."""
    return random_batch(k, n_sn, 100, 100, make_bands(6), make_model(), fixed_nobs=100)

"""FP64 oracle of the SALT bandflux, its parameter derivatives and the chi-square gradient.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library: it builds its own band quadrature grids, evaluates the
full 16-node bicubic at every quadrature point in Catmull-Rom cubic-Hermite
form, and sums the integral point by point with no reordering or factorisation.

Definitions (paper, section "Implementation"):

* model equation: F(p, lam) = x0 [M0(p, lam) + x1 M1(p, lam)] exp(c CL(lam));
  the free parameters are x0, x1, t0, c.
* bandflux equation: the integral of F(lam) T(lam) lam / (h c) over the band;
  the implementation paragraph states that the integral is taken with the
  trapezoidal rule along wavelength.

Readings where the paper is silent or garbled:

* phase p = (t - t0)/(1+z) and the amplitude x0/(1+z) (the phase sentence of
  the model paragraph is garbled);
* the surfaces are evaluated at the rest wavelength mu = lam/(1+z) of a fixed
  observer-frame quadrature grid lam_k; lam/(hc) uses the observer-frame lam;
* bicubic = Catmull-Rom (Keys, a = -1/2) cubic convolution on the uniform grid,
  linear in the first and last cell of each axis;
* a phase outside the surface grid contributes zero flux; a rest-frame band
  window outside the wavelength grid is an error (NaN result);
* CL(mu) = sum_n a_n r^n, r = (mu - lam_B)/(lam_V - lam_B), used as exp(c CL);
* band grid: N = ceil((U - L)/spacing) intervals of width (U - L)/N between the
  first and last tabulated wavelength, T linearly interpolated;
* h and c are the exact SI values, lam in Angstrom.
"""
from __future__ import annotations

import numpy as np

H_PLANCK = 6.62607015e-27       # erg s
C_LIGHT_AA = 2.99792458e18      # Angstrom / s
HC = H_PLANCK * C_LIGHT_AA      # erg Angstrom
FNU_AB = 10.0 ** (-0.4 * 48.60)  # AB reference source, erg s^-1 cm^-2 Hz^-1 (m_AB = 0)

PARAM_NAMES = ("z", "t0", "x0", "x1", "c")


# ----------------------------------------------------------------------------- band grid

def band_grid(wave, trans, spacing=5.0, rule="trapezoid"):
    """Quadrature grid of one band: nodes lam_k, transmission T_k, weights w_k.

    N = ceil((U - L)/spacing) equal intervals of width Delta between the first (L)
    and last (U) tabulated wavelengths; T is linearly interpolated from the samples.
    rule "trapezoid" (the paper's rule, section "Implementation"): the N + 1 interval
    ends, weights Delta/2 at both ends and Delta inside.  rule "midpoint": the N
    interval midpoints, weight Delta each.
    """
    wave = np.asarray(wave, dtype=np.float64)
    trans = np.asarray(trans, dtype=np.float64)
    L, U = wave[0], wave[-1]
    n = max(1, int(np.ceil((U - L) / spacing - 1e-9)))
    delta = (U - L) / n
    if rule == "trapezoid":
        lam = L + delta * np.arange(n + 1)
        lam[-1] = U
        w = np.full(n + 1, delta)
        w[0] = w[-1] = 0.5 * delta
    elif rule == "midpoint":
        lam = L + delta * (np.arange(n) + 0.5)
        w = np.full(n, delta)
    else:
        raise ValueError(f"unknown quadrature rule {rule!r}")
    T = np.interp(lam, wave, trans)
    return lam, T, w


def ab_zeropoint(wave, trans, spacing=5.0, rule="trapezoid"):
    """Bandflux of the AB reference source (f_nu = FNU_AB at every frequency) through the band, with
    the band's own quadrature: the photon weight lam/(hc) times f_lam = f_nu c / lam^2, summed with
    the trapezoid (or midpoint) weights.  m_AB = -2.5 log10(f / this)."""
    lam, T, w = band_grid(wave, trans, spacing, rule)
    f_lam = FNU_AB * C_LIGHT_AA / lam ** 2
    return float(np.sum(w * T * f_lam * lam / HC))


# ----------------------------------------------------------------------------- interpolation

def _cell(x, n):
    """Cell index a in [0, n-2] and fraction in [0, 1] of grid coordinate x; inside-grid mask."""
    inside = (x >= 0.0) & (x <= n - 1)
    a = np.clip(np.floor(x), 0, n - 2).astype(np.int64)
    return a, x - a, inside


def _hermite(mm, m0, m1, m2, f, edge):
    """Cubic Hermite on [node0, node1] with Catmull-Rom tangents; linear in edge cells."""
    t0 = 0.5 * (m1 - mm)
    t1 = 0.5 * (m2 - m0)
    f2 = f * f
    f3 = f2 * f
    cub = (2 * f3 - 3 * f2 + 1) * m0 + (f3 - 2 * f2 + f) * t0 + (-2 * f3 + 3 * f2) * m1 + (f3 - f2) * t1
    lin = (1.0 - f) * m0 + f * m1
    return np.where(edge, lin, cub)


def _hermite_df(mm, m0, m1, m2, f, edge):
    """Derivative with respect to the fraction f of :func:`_hermite`."""
    t0 = 0.5 * (m1 - mm)
    t1 = 0.5 * (m2 - m0)
    f2 = f * f
    cub = (6 * f2 - 6 * f) * m0 + (3 * f2 - 4 * f + 1) * t0 + (-6 * f2 + 6 * f) * m1 + (3 * f2 - 2 * f) * t1
    lin = m1 - m0
    return np.where(edge, lin, cub)


def interp2(M, u, v, deriv=False):
    """Bicubic value of surface M at grid coordinates (u, v) (phase index, wavelength index).

    u and v broadcast against each other.  Returns I, and with ``deriv`` also
    dI/du and dI/dv (per grid unit).  Points with u outside [0, n_phase-1]
    give 0; points with v outside [0, n_wave-1] give NaN.
    """
    M = np.asarray(M, dtype=np.float64)
    n_p, n_w = M.shape
    u, v = np.broadcast_arrays(np.asarray(u, np.float64), np.asarray(v, np.float64))
    a, x, in_u = _cell(u, n_p)
    j, y, in_v = _cell(v, n_w)
    edge_u = (a == 0) | (a == n_p - 2)
    edge_v = (j == 0) | (j == n_w - 2)
    rows = [np.clip(a + d, 0, n_p - 1) for d in (-1, 0, 1, 2)]
    cols = [np.clip(j + d, 0, n_w - 1) for d in (-1, 0, 1, 2)]
    nodes = [[M[r, cc] for cc in cols] for r in rows]
    along = [_hermite(*nd, y, edge_v) for nd in nodes]
    val = _hermite(*along, x, edge_u)
    zero = ~in_u
    bad = ~in_v
    val = np.where(zero, 0.0, val)
    val = np.where(bad, np.nan, val)
    if not deriv:
        return val
    d_u = _hermite_df(*along, x, edge_u)
    along_dv = [_hermite_df(*nd, y, edge_v) for nd in nodes]
    d_v = _hermite(*along_dv, x, edge_u)
    d_u = np.where(bad, np.nan, np.where(zero, 0.0, d_u))
    d_v = np.where(bad, np.nan, np.where(zero, 0.0, d_v))
    return val, d_u, d_v


# ----------------------------------------------------------------------------- colour law

def colour_law(model, mu, deriv=False):
    """CL(mu) = sum_n a_n r^n with r = (mu - lam_B)/(lam_V - lam_B); optionally dCL/dmu."""
    coef = np.asarray(model.cl_coef, dtype=np.float64)
    span = model.cl_wave_v - model.cl_wave_b
    r = (np.asarray(mu, np.float64) - model.cl_wave_b) / span
    cl = np.zeros_like(r)
    dcl = np.zeros_like(r)
    for n, a in enumerate(coef, start=1):
        cl = cl + a * r ** n
        dcl = dcl + n * a * r ** (n - 1)
    return (cl, dcl / span) if deriv else cl


# ----------------------------------------------------------------------------- bandflux

class Oracle:
    """Model surfaces (float32 nodes held in float64) and band grids, evaluated in FP64."""

    def __init__(self, model, bands, spacing=5.0, rule="trapezoid"):
        self.model = model
        self.m0 = np.asarray(model.m0, dtype=np.float64)
        self.m1 = np.asarray(model.m1, dtype=np.float64)
        self.grids = [band_grid(b.wave, b.trans, spacing, rule) for b in bands]

    def _group(self, b, z, t0, x0, x1, c, t, jac):
        """Flux (and five partials) of the observations t of one supernova in band b."""
        md = self.model
        lam, T, w = self.grids[b]
        s = 1.0 / (1.0 + z)
        A = x0 * s
        p = (t - t0) * s
        mu = lam * s
        u = (p - md.phase0) / md.dphase
        v = (mu - md.wave0) / md.dwave
        Wk = w * lam * T / HC
        cl, dcl = colour_law(md, mu, deriv=True)
        E = np.exp(c * cl)
        om = (Wk * E)[None, :]
        uu = u[:, None]
        vv = v[None, :]
        if not jac:
            I = interp2(self.m0, uu, vv) + x1 * interp2(self.m1, uu, vv)
            return A * (om * I).sum(axis=1)
        i0, i0u, i0v = interp2(self.m0, uu, vv, deriv=True)
        i1, i1u, i1v = interp2(self.m1, uu, vv, deriv=True)
        I = i0 + x1 * i1
        Ip = (i0u + x1 * i1u) / md.dphase
        Imu = (i0v + x1 * i1v) / md.dwave
        S_f = (om * I).sum(axis=1)
        S_1 = (om * i1).sum(axis=1)
        S_c = (om * cl[None, :] * I).sum(axis=1)
        S_p = (om * Ip).sum(axis=1)
        S_l = (om * mu[None, :] * (Imu + c * dcl[None, :] * I)).sum(axis=1)
        f = A * S_f
        J = np.empty((len(t), 5))
        J[:, 0] = -s * f - A * s * (p * S_p + S_l)   # d/dz
        J[:, 1] = -A * s * S_p                        # d/dt0
        J[:, 2] = s * S_f                             # d/dx0
        J[:, 3] = A * S_1                             # d/dx1
        J[:, 4] = A * S_c                             # d/dc
        return f, J

    def _run(self, batch, jac, params=None):
        P = batch.params().astype(np.float64) if params is None else np.asarray(params, np.float64)
        t_all = batch.t.astype(np.float64)
        f = np.zeros(batch.n_obs)
        J = np.zeros((batch.n_obs, 5)) if jac else None
        off = batch.sn_offsets
        for s in range(batch.n_sn):
            lo, hi = int(off[s]), int(off[s + 1])
            if hi <= lo:
                continue
            bs = batch.band[lo:hi]
            for b in np.unique(bs):
                idx = lo + np.nonzero(bs == b)[0]
                r = self._group(int(b), *P[s], t_all[idx], jac)
                if jac:
                    f[idx], J[idx] = r
                else:
                    f[idx] = r
        return (f, J) if jac else f

    def bandflux(self, batch, params=None):
        """Flux of every observation of the batch (float64 [n_obs])."""
        return self._run(batch, False, params)

    def jac(self, batch, params=None):
        """Flux and d f_i / d(z, t0, x0, x1, c) of every observation: ([n_obs], [n_obs, 5])."""
        return self._run(batch, True, params)

    def vjp(self, batch, cot, params=None):
        """Per-supernova sum_i cot_i d f_i / d theta  ->  [n_sn, 5] (z, t0, x0, x1, c)."""
        f, J = self.jac(batch, params)
        g = segment_sum(np.asarray(cot, np.float64)[:, None] * J, batch.sn_offsets)
        return f, g

    def chi2_grad(self, batch, data, inv_sigma2, params=None):
        """chi2_s = sum_i (f_i - d_i)^2 / sigma_i^2 and its gradient with sigma held fixed."""
        f, J = self.jac(batch, params)
        r = f - np.asarray(data, np.float64)
        w = np.asarray(inv_sigma2, np.float64)
        chi2 = segment_sum(r * r * w, batch.sn_offsets)
        g = segment_sum((2.0 * r * w)[:, None] * J, batch.sn_offsets)
        return f, chi2, g


def segment_sum(x, offsets):
    """Sum of rows of x within each CSR segment [offsets[s], offsets[s+1])."""
    x = np.asarray(x, np.float64)
    n = len(offsets) - 1
    out = np.zeros((n,) + x.shape[1:])
    for s in range(n):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        if hi > lo:
            out[s] = x[lo:hi].sum(axis=0)
    return out

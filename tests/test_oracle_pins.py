"""Pins of the FP64 oracle against what the model and mathematics fix (CPU only).

Each test names the part of the definition it pins.  None re-uses the oracle's
own formula for its expected value: expectations come from closed forms,
exact rational arithmetic with the Keys convolution kernel (the oracle uses the
cubic-Hermite form), invariances, scipy quadrature, or finite differences.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from oracle.salt64 import HC

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Colour-law reference wavelengths (Angstrom), written here as literals.
LAM_B, LAM_V = 4302.57, 5428.55
# h c in erg Angstrom: the CODATA value 1.98644586e-25 J m, written here as a literal.
HC_LITERAL = 1.98644586e-8


# ----------------------------------------------------------------------------- helpers

def keys(d):
    """Keys cubic-convolution kernel, a = -1/2 (works on floats and Fractions)."""
    ad = abs(d)
    if ad < 1:
        return Fraction(3, 2) * ad ** 3 - Fraction(5, 2) * ad ** 2 + 1
    if ad < 2:
        return Fraction(-1, 2) * ad ** 3 + Fraction(5, 2) * ad ** 2 - 4 * ad + 2
    return 0 * ad


def keys_interp_1d(nodes, x):
    """Brute-force convolution over all nodes of an interior cell (no Hermite form)."""
    return sum(keys(x - j) * m for j, m in enumerate(nodes))


def one_sn_batch(t, band, z=0.1, t0=0.0, x0=1e-5, x1=0.5, c=0.05):
    t = np.atleast_1d(np.asarray(t, np.float32))
    band = np.broadcast_to(np.asarray(band, np.int32), t.shape).copy()
    return synth.Batch(np.float32([z]), np.float32([t0]), np.float32([x0]), np.float32([x1]),
                       np.float32([c]), t, band, np.int32([0, len(t)]))


def const_model(K, n_phase=71, n_wave=721, cl=(0.0,), m1=None, **kw):
    m0 = np.full((n_phase, n_wave), K, np.float32)
    m1 = np.zeros_like(m0) if m1 is None else m1
    return synth.Model(m0=m0, m1=m1, cl_coef=np.asarray(cl, np.float64), **kw)


# ----------------------------------------------------------------------------- P1-P3 interpolation

def test_p1_nodes_reproduced():
    """Interpolation reproduces every grid node, interior and edge (bicubic definition)."""
    g = np.random.default_rng(1)
    M = g.normal(size=(9, 12))
    a, j = np.meshgrid(np.arange(9), np.arange(12), indexing="ij")
    val = oracle.interp2(M, a.astype(float), j.astype(float))
    assert np.array_equal(val, M)


def test_p2_quadratic_interior_bilinear_edge():
    """Catmull-Rom reproduces quadratics in interior cells; edge cells reproduce bilinear data."""
    n_p, n_w = 8, 10
    a, j = np.meshgrid(np.arange(n_p, dtype=float), np.arange(n_w, dtype=float), indexing="ij")
    q = lambda u, v: 1.5 + 0.3 * u - 0.2 * v + 0.07 * u * u - 0.05 * v * v + 0.11 * u * v
    M = q(a, j)
    g = np.random.default_rng(2)
    u = g.uniform(1.0, n_p - 2.0, 500)
    v = g.uniform(1.0, n_w - 2.0, 500)
    np.testing.assert_allclose(oracle.interp2(M, u, v), q(u, v), rtol=1e-13, atol=1e-13)
    # a cubic in u is not reproduced (the scheme is Catmull-Rom, not a cubic spline)
    Mc = a ** 3
    assert abs(oracle.interp2(Mc, 3.25, 4.0) - 3.25 ** 3) > 1e-2
    # edge cells: bilinear data reproduced, in the first and last cell of each axis
    bl = lambda u, v: 2.0 + 0.5 * u - 0.25 * v + 0.125 * u * v
    Mb = bl(a, j)
    ue = np.r_[g.uniform(0, 1, 50), g.uniform(n_p - 2, n_p - 1, 50), g.uniform(0, n_p - 1, 100)]
    ve = np.r_[g.uniform(0, n_w - 1, 100), g.uniform(0, 1, 50), g.uniform(n_w - 2, n_w - 1, 50)]
    np.testing.assert_allclose(oracle.interp2(Mb, ue, ve), bl(ue, ve), rtol=1e-13, atol=1e-13)


def test_p3_hermite_equals_keys_convolution():
    """The oracle's Hermite form equals the Keys (a=-1/2) convolution, value and derivatives."""
    g = np.random.default_rng(3)
    n_p, n_w = 7, 9
    M = g.normal(size=(n_p, n_w))
    for _ in range(200):
        u = g.uniform(1.0, n_p - 2.0)
        v = g.uniform(1.0, n_w - 2.0)
        want = sum(float(keys(u - a)) * float(keys(v - j)) * M[a, j] for a in range(n_p) for j in range(n_w))
        val, du, dv = oracle.interp2(M, u, v, deriv=True)
        assert abs(val - want) < 1e-12
        h = 1e-6
        fd_u = (oracle.interp2(M, u + h, v) - oracle.interp2(M, u - h, v)) / (2 * h)
        fd_v = (oracle.interp2(M, u, v + h) - oracle.interp2(M, u, v - h)) / (2 * h)
        assert abs(du - fd_u) < 1e-7 and abs(dv - fd_v) < 1e-7


def test_out_of_range_policy():
    """Phase outside the grid gives zero flux; a wavelength outside gives NaN."""
    M = np.ones((5, 5))
    assert oracle.interp2(M, -0.01, 2.0) == 0.0 and oracle.interp2(M, 4.01, 2.0) == 0.0
    assert oracle.interp2(M, 0.0, 2.0) == 1.0 and oracle.interp2(M, 4.0, 2.0) == 1.0
    assert np.isnan(oracle.interp2(M, 2.0, -0.01)) and np.isnan(oracle.interp2(M, 2.0, 4.01))


# ----------------------------------------------------------------------------- P10 exact tiny case

def test_p10_tiny_exact_fraction():
    """Brute-force exact rational bandflux of a tiny case equals the hand-derived golden value,
    and the FP64 oracle matches it to rounding."""
    fx = json.load(open(os.path.join(GOLDEN, "tiny_exact.json")))
    S = fx["surface"]
    M0 = [[Fraction(v) for v in r] for r in S["m0"]]
    M1 = [[Fraction(v) for v in r] for r in S["m1"]]
    P = fx["params"]
    z, t0, x0, x1 = (Fraction(P[k]) for k in ("z", "t0", "x0", "x1"))
    s = 1 / (1 + z)
    p = (Fraction(fx["obs_t"]) - t0) * s
    # band grid by hand: nodes 3..7, linear transmission between the three samples
    lam = [Fraction(v) for v in (3, 4, 5, 6, 7)]
    T = [Fraction(1, 2), Fraction(3, 4), Fraction(1), Fraction(5, 8), Fraction(1, 4)]
    w = [Fraction(1, 2), 1, 1, 1, Fraction(1, 2)]
    total = Fraction(0)
    for lk, Tk, wk in zip(lam, T, w):
        mu = lk * s
        I = sum(keys(p - a) * keys(mu - j) * (M0[a][j] + x1 * M1[a][j]) for a in range(6) for j in range(6))
        total += wk * lk * Tk * I
    exact = x0 * s * total
    gold = Fraction(fx["expected_flux_times_hc"]["num"], fx["expected_flux_times_hc"]["den"])
    assert exact == gold
    md = synth.Model(m0=np.float32(S["m0"]), m1=np.float32(S["m1"]), phase0=S["phase0"], dphase=S["dphase"],
                     wave0=S["wave0"], dwave=S["dwave"], cl_coef=np.zeros(1), cl_wave_b=0.0, cl_wave_v=1.0)
    band = synth.Band(np.array(fx["band"]["wave"]), np.array(fx["band"]["trans"]))
    o = oracle.Oracle(md, [band], spacing=fx["band"]["spacing"])
    f = o.bandflux(one_sn_batch([fx["obs_t"]], 0, z=P["z"], t0=P["t0"], x0=P["x0"], x1=P["x1"], c=P["c"]))
    assert abs(f[0] * HC - float(gold)) <= 1e-13 * float(gold)


# ----------------------------------------------------------------------------- band grid (D3)

def test_band_grid_construction():
    b = synth.make_bands(6)[2]
    lam, T, w = oracle.band_grid(b.wave, b.trans, 5.0)
    n = len(lam) - 1
    assert n == int(np.ceil((b.hi - b.lo) / 5.0))
    assert lam[0] == b.lo and lam[-1] == b.hi
    assert np.all(np.diff(lam) <= 5.0 + 1e-9)
    assert abs(w.sum() - (b.hi - b.lo)) < 1e-9
    assert np.all(T >= 0) and np.all(T <= 1)
    # exact integer division keeps N exact (4 bands of 1375 A -> 275 intervals)
    b4 = synth.make_bands(4)[0]
    assert len(oracle.band_grid(b4.wave, b4.trans, 5.0)[0]) == 276
    assert len(oracle.band_grid(b.wave, b.trans, 5.0)[0]) == 185


# ----------------------------------------------------------------------------- P4-P6 invariants

@pytest.fixture(scope="module")
def o4(model, bands4):
    return oracle.Oracle(model, bands4)


def test_p4_linear_in_x0_affine_in_x1(o4):
    b = synth.one_sn_40_obs()
    f = o4.bandflux(b)
    f2 = o4.bandflux(b.with_params(x0=b.x0 * 2))
    np.testing.assert_allclose(f2, 2 * f, rtol=1e-14)
    fa = o4.bandflux(b.with_params(x1=[0.0]))
    fb = o4.bandflux(b.with_params(x1=[1.0]))
    fc = o4.bandflux(b.with_params(x1=[-2.5]))
    np.testing.assert_allclose(fc, fa + (-2.5) * (fb - fa), rtol=1e-12)
    fj, J = o4.jac(b)
    np.testing.assert_allclose(J[:, 2], fj / b.x0[0].astype(float), rtol=1e-13)
    np.testing.assert_allclose(J[:, 3], fb - fa, rtol=1e-12)


def test_p5_c_zero_reduction(model, bands4):
    """At c = 0 the colour law drops out: same flux for any colour-law coefficients."""
    b = synth.one_sn_40_obs().with_params(c=[0.0])
    o1 = oracle.Oracle(model, bands4)
    other = synth.Model(m0=model.m0, m1=model.m1, cl_coef=np.array([3.0, -1.0, 0.5]))
    o2 = oracle.Oracle(other, bands4)
    np.testing.assert_allclose(o1.bandflux(b), o2.bandflux(b), rtol=1e-15)
    # and a zero colour law makes c irrelevant
    zero = synth.Model(m0=model.m0, m1=model.m1, cl_coef=np.zeros(3))
    o3 = oracle.Oracle(zero, bands4)
    np.testing.assert_allclose(o3.bandflux(b.with_params(c=[0.3])), o1.bandflux(b), rtol=1e-15)
    _, J = o3.jac(b.with_params(c=[0.3]))
    assert np.all(J[:, 4] == 0.0)


def test_p6_time_shift_and_z0(o4):
    """f depends on t - t0 only; at z = 0 the amplitude is x0 and phases are t - t0."""
    b = synth.one_sn_40_obs()
    f = o4.bandflux(b)
    # shift in float64 so that t - t0 stays exact
    sh = synth.Batch(b.z, b.t0, b.x0, b.x1, b.c, b.t.astype(np.float64) + 64.25, b.band, b.sn_offsets)
    P = b.params().astype(np.float64)
    P[:, 1] += 64.25
    np.testing.assert_allclose(o4.bandflux(sh, P), f, rtol=1e-13)
    # z=0: a supernova observed at t equals the rest-frame evaluation with s = 1, which for a
    # surface constant in wavelength reduces to x0 * M(p) * sum_k w_k lam_k T_k / hc
    K = np.exp(-0.5 * ((np.arange(71) - 20.0) / 10.0) ** 2)[:, None] * np.ones((1, 721))
    md = synth.Model(m0=np.float32(K), m1=np.zeros((71, 721), np.float32), cl_coef=np.zeros(1))
    band = synth.tophat_band(4000.0, 5000.0)
    o = oracle.Oracle(md, [band])
    t = np.float32([-7.0, 0.0, 13.0])        # nodes of the phase grid
    bz = one_sn_batch(t, 0, z=0.0, t0=0.0, x0=2e-5, x1=0.0, c=0.0)
    want = float(np.float32(2e-5)) * np.float32(K)[(t + 20).astype(int), 0].astype(float) * (5000.0 ** 2 - 4000.0 ** 2) / (2 * HC)
    np.testing.assert_allclose(o.bandflux(bz), want, rtol=1e-13)


# ----------------------------------------------------------------------------- P7 closed forms

@pytest.mark.parametrize("z", [0.0, 0.1, 0.37, 0.9])
def test_p7_flat_spectrum_tophat(z):
    """M0 = K, x1 = 0, top-hat T on [a,b]: f = x0 K (b^2 - a^2) / (2 hc (1+z)) exactly."""
    K = 0.75
    md = const_model(K, cl=(-0.9, 0.1, 0.01))
    a, bnd = 4000.0, 5230.0
    o = oracle.Oracle(md, [synth.tophat_band(a, bnd)])
    t = np.float32([3.0, 17.25, -9.5])
    x0 = 3e-5
    bt = one_sn_batch(t, 0, z=z, t0=1.0, x0=x0, x1=0.0, c=0.0)
    zf = float(np.float32(z))
    want = float(np.float32(x0)) * K * (bnd ** 2 - a ** 2) / (2 * HC * (1 + zf))
    f, J = o.jac(bt)
    np.testing.assert_allclose(f, want, rtol=1e-13)
    np.testing.assert_allclose(J[:, 0], -want / (1 + zf), rtol=1e-10)   # d/dz
    np.testing.assert_allclose(J[:, 1], 0.0, atol=1e-12 * want)        # d/dt0


def test_p7_phase_quadratic():
    """M0 = K q(p), q quadratic: f and df/dt0, df/dz follow the closed form for interior phases."""
    K = 1.25
    al, be, ga = 1.0, 0.02, -0.001
    p = np.arange(71) - 20.0
    m0 = (K * (al + be * p + ga * p * p))[:, None] * np.ones((1, 721))
    # float64 nodes: exactly on the quadratic up to float64 rounding
    md = synth.Model(m0=m0, m1=np.zeros((71, 721)), cl_coef=np.zeros(1))
    a, bnd = 3600.0, 4700.0
    o = oracle.Oracle(md, [synth.tophat_band(a, bnd)])
    z, t0, x0 = 0.25, 2.0, 1e-5
    t = np.float32([-8.3, 5.55, 30.7])
    bt = one_sn_batch(t, 0, z=z, t0=t0, x0=x0, x1=0.0, c=0.0)
    zf, t0f, x0f = (float(np.float32(v)) for v in (z, t0, x0))
    s = 1 / (1 + zf)
    pp = (t.astype(float) - t0f) * s
    B = (bnd ** 2 - a ** 2) / (2 * HC)
    q = K * (al + be * pp + ga * pp * pp)
    dq = K * (be + 2 * ga * pp)
    f, J = o.jac(bt)
    np.testing.assert_allclose(f, x0f * s * q * B, rtol=1e-12)
    np.testing.assert_allclose(J[:, 1], -x0f * s * s * dq * B, rtol=1e-10)
    np.testing.assert_allclose(J[:, 0], -s * s * x0f * B * (q + pp * dq), rtol=1e-10)


def test_p7_wavelength_linear_trapezoid_error():
    """M0 = K (al + be mu): trapezoid = exact integral + (b-a) Delta^2 g''/12 (quadratic integrand)."""
    K, al, be = 1.0, 0.5, 2e-4
    mu = 2000.0 + 10.0 * np.arange(721)
    m0 = (K * (al + be * mu))[None, :] * np.ones((71, 1))
    # float64 model (nodes exactly on the line up to float64 rounding)
    md = synth.Model(m0=m0, m1=np.zeros((71, 721)), cl_coef=np.zeros(1))
    a, bnd = 4100.0, 5350.0
    spacing = 5.0
    o = oracle.Oracle(md, [synth.tophat_band(a, bnd)], spacing=spacing)
    z, x0 = 0.3, 1e-5
    bt = one_sn_batch([4.0], 0, z=z, t0=0.0, x0=x0, x1=0.0, c=0.0)
    zf, x0f = float(np.float32(z)), float(np.float32(x0))
    s = 1 / (1 + zf)
    A = x0f * s
    N = int(np.ceil((bnd - a) / spacing))
    D = (bnd - a) / N
    exact = A * K / HC * (al * (bnd ** 2 - a ** 2) / 2 + be * s * (bnd ** 3 - a ** 3) / 3)
    corr = (bnd - a) * D ** 2 * (2 * A * K * be * s / HC) / 12
    f = o.bandflux(bt)
    np.testing.assert_allclose(f[0], exact + corr, rtol=1e-12)


def test_p7_midpoint_rule_closed_forms():
    """Midpoint rule (the quadrature option): exact on the flat top-hat (linear integrand), and on a
    quadratic integrand its error is -1/2 of the trapezoid's: midpoint = exact - (b-a) Delta^2 g''/24."""
    K = 0.75
    md = const_model(K, cl=(-0.9, 0.1, 0.01))
    a, bnd = 4000.0, 5230.0
    o = oracle.Oracle(md, [synth.tophat_band(a, bnd)], rule="midpoint")
    x0, z = 3e-5, 0.4
    bt = one_sn_batch(np.float32([3.0, 17.25]), 0, z=z, t0=1.0, x0=x0, x1=0.0, c=0.0)
    zf = float(np.float32(z))
    want = float(np.float32(x0)) * K * (bnd ** 2 - a ** 2) / (2 * HC * (1 + zf))
    np.testing.assert_allclose(o.bandflux(bt), want, rtol=1e-13)
    # quadratic integrand: M0 linear in the rest wavelength
    Kl, al, be = 1.0, 0.5, 2e-4
    mu = 2000.0 + 10.0 * np.arange(721)
    m0 = (Kl * (al + be * mu))[None, :] * np.ones((71, 1))
    ml = synth.Model(m0=m0, m1=np.zeros((71, 721)), cl_coef=np.zeros(1))
    a, bnd, spacing = 4100.0, 5350.0, 5.0
    zq, x0q = 0.3, 1e-5
    bq = one_sn_batch([4.0], 0, z=zq, t0=0.0, x0=x0q, x1=0.0, c=0.0)
    zf, x0f = float(np.float32(zq)), float(np.float32(x0q))
    s = 1 / (1 + zf)
    A = x0f * s
    N = int(np.ceil((bnd - a) / spacing))
    D = (bnd - a) / N
    exact = A * Kl / HC * (al * (bnd ** 2 - a ** 2) / 2 + be * s * (bnd ** 3 - a ** 3) / 3)
    g2 = 2 * A * Kl * be * s / HC            # second derivative of the integrand in lambda
    mid = oracle.Oracle(ml, [synth.tophat_band(a, bnd)], spacing=spacing, rule="midpoint").bandflux(bq)[0]
    trap = oracle.Oracle(ml, [synth.tophat_band(a, bnd)], spacing=spacing).bandflux(bq)[0]
    np.testing.assert_allclose(mid, exact - (bnd - a) * D ** 2 * g2 / 24, rtol=1e-12)
    np.testing.assert_allclose(trap - exact, -2 * (mid - exact), rtol=1e-8)


def test_midpoint_grid_nodes_and_weights():
    """Midpoint grid: the N interval midpoints, weight Delta each, summing to U - L."""
    b = synth.make_bands(6)[2]
    lam, T, w = oracle.band_grid(b.wave, b.trans, 5.0, rule="midpoint")
    lt, _, wt = oracle.band_grid(b.wave, b.trans, 5.0)
    assert len(lam) == len(lt) - 1
    np.testing.assert_allclose(lam, 0.5 * (lt[:-1] + lt[1:]), rtol=0, atol=1e-9)
    np.testing.assert_allclose(w.sum(), b.wave[-1] - b.wave[0], rtol=1e-14)
    np.testing.assert_allclose(T, np.interp(lam, b.wave, b.trans), rtol=0, atol=0)


# ----------------------------------------------------------------------------- P8 quadrature convergence

def test_p8_quadrature_converges_to_quad(model):
    """Trapezoid results converge at second order to the adaptive-quadrature integral.

    A top-hat transmission keeps the integrand free of kinks from the sampled
    filter curve, so the only non-smoothness left is that of the C1 bicubic
    surface at its nodes; quad is split at those nodes."""
    a_lo, a_hi = 4503.3, 5711.9
    band = synth.tophat_band(a_lo, a_hi)
    z, t0, x0, x1, c = 0.3, 0.0, 1e-5, 0.7, 0.08
    bt = one_sn_batch([6.2], 0, z=z, t0=t0, x0=x0, x1=x1, c=c)
    zf, x0f, x1f, cf, tf = (float(np.float32(v)) for v in (z, x0, x1, c, 6.2))
    vals = []
    for sp in (5.0, 2.5, 1.25, 0.625):
        vals.append(oracle.Oracle(model, [band], spacing=sp).bandflux(bt)[0])
    d = np.diff(vals)
    ratios = d[:-1] / d[1:]
    assert np.all((ratios > 3.5) & (ratios < 4.5)), ratios
    s = 1 / (1 + zf)
    u = (tf * s + 20.0)
    m0 = model.m0.astype(np.float64)
    m1 = model.m1.astype(np.float64)

    def integrand(lam):
        mu = lam * s
        v = (mu - 2000.0) / 10.0
        I = oracle.interp2(m0, u, v) + x1f * oracle.interp2(m1, u, v)
        r = (mu - LAM_B) / (LAM_V - LAM_B)           # the colour law written out here
        a1, a2, a3 = (float(v) for v in model.cl_coef)
        cl = a1 * r + a2 * r * r + a3 * r * r * r
        return x0f * s * I * np.exp(cf * cl) * lam / HC

    nodes = (2000.0 + 10.0 * np.arange(721)) / s
    knots = np.r_[a_lo, nodes[(nodes > a_lo) & (nodes < a_hi)], a_hi]
    ref = sum(integrate.quad(integrand, p, q, epsabs=0, epsrel=1e-13)[0] for p, q in zip(knots[:-1], knots[1:]))
    rich = vals[-1] + (vals[-1] - vals[-2]) / 3.0
    assert abs(rich - ref) / ref < 1e-9
    assert 1e-9 < abs(vals[0] - ref) / ref < 1e-4


# ----------------------------------------------------------------------------- P9 analytic gradient

def test_p9_gradient_vs_central_differences(model, bands6):
    """Analytic d f/d(z, t0, x0, x1, c) against FP64 central differences."""
    o = oracle.Oracle(model, bands6)
    b = synth.batch_4096_sn(n_sn=6)
    P = b.params().astype(np.float64)
    f, J = o.jac(b, P)
    scale = np.array([0.1, 1.0, 1.0, 1.0, 0.1])
    for q in range(5):
        h = 1e-5 * scale[q] if q != 2 else 1e-5 * P[:, 2]
        Pp, Pm = P.copy(), P.copy()
        Pp[:, q] += h
        Pm[:, q] -= h
        fd = (o.bandflux(b, Pp) - o.bandflux(b, Pm))
        hh = np.repeat(2 * np.broadcast_to(h, (b.n_sn,)), np.diff(b.sn_offsets))
        fd = fd / hh
        sc = np.abs(J[:, q]).max()
        assert np.max(np.abs(fd - J[:, q])) <= 2e-6 * sc, (q, np.max(np.abs(fd - J[:, q])) / sc)


def test_vjp_and_chi2_gradient(model, bands6):
    o = oracle.Oracle(model, bands6)
    b = synth.batch_4096_sn(n_sn=5)
    g = np.random.default_rng(5)
    cot = g.normal(size=b.n_obs)
    f, J = o.jac(b)
    _, v = o.vjp(b, cot)
    for s in range(b.n_sn):
        lo, hi = b.sn_offsets[s], b.sn_offsets[s + 1]
        np.testing.assert_allclose(v[s], cot[lo:hi] @ J[lo:hi], rtol=1e-12)
    # chi2 gradient vs FD of chi2 in x1 and c
    d = f * (1 + 0.05 * g.normal(size=b.n_obs))
    w = 1.0 / (0.05 * np.abs(f)) ** 2
    _, chi2, gr = o.chi2_grad(b, d, w)
    P = b.params().astype(np.float64)
    for q, h in ((3, 1e-6), (4, 1e-7)):
        Pp, Pm = P.copy(), P.copy()
        Pp[:, q] += h
        Pm[:, q] -= h
        cp = oracle.segment_sum((o.bandflux(b, Pp) - d) ** 2 * w, b.sn_offsets)
        cm = oracle.segment_sum((o.bandflux(b, Pm) - d) ** 2 * w, b.sn_offsets)
        np.testing.assert_allclose((cp - cm) / (2 * h), gr[:, q], rtol=1e-5)


# ----------------------------------------------------------------------------- P11 fit

def test_p11_fit_recovers_truth(model, bands6):
    """LM fit of noise-free data recovers the true parameters with chi2 -> 0."""
    o = oracle.Oracle(model, bands6)
    fo = oracle.FitOracle(o)
    reqs = synth.fit_requests(3, k=41)
    for r in reqs:
        b = synth.Batch(np.float32([r.z]), np.float32([r.theta_true[0]]), np.float32([r.theta_true[1]]),
                        np.float32([r.theta_true[2]]), np.float32([r.theta_true[3]]), r.t, r.band,
                        np.int32([0, len(r.t)]))
        f = o.bandflux(b)
        _, sig, w = synth.make_data(f, b.sn_offsets, np.zeros(len(f)))
        res = fo.fit(b, r.z, r.theta_init, f, w)
        th = res["theta"]
        tt = r.theta_true
        assert res["chi2"] < 1e-8
        assert abs(th[0] - tt[0]) < 1e-5 and abs(th[1] / tt[1] - 1) < 1e-6
        assert abs(th[2] - tt[2]) < 1e-5 and abs(th[3] - tt[3]) < 1e-6


@pytest.mark.parametrize("held", [3, 2, 0])
def test_p11_fit_with_a_held_parameter(model, bands6, held):
    """A parameter held at its true value stays there exactly and the free ones are recovered
    from noise-free data, as with all four free."""
    o = oracle.Oracle(model, bands6)
    fo = oracle.FitOracle(o)
    r = synth.fit_requests(1, k=43)[0]
    b = synth.Batch(np.float32([r.z]), np.float32([r.theta_true[0]]), np.float32([r.theta_true[1]]),
                    np.float32([r.theta_true[2]]), np.float32([r.theta_true[3]]), r.t, r.band,
                    np.int32([0, len(r.t)]))
    f = o.bandflux(b)
    _, sig, w = synth.make_data(f, b.sn_offsets, np.zeros(len(f)))
    start = np.array(r.theta_init, np.float64)
    start[held] = r.theta_true[held]
    free = [k != held for k in range(4)]
    res = fo.fit(b, r.z, start, f, w, free=free)
    th, tt = res["theta"], np.asarray(r.theta_true, np.float64)
    assert th[held] == start[held] or (held == 1 and abs(th[1] / start[1] - 1) < 1e-15)
    assert res["chi2"] < 1e-8
    assert abs(th[0] - tt[0]) < 1e-5 and abs(th[1] / tt[1] - 1) < 1e-6
    assert abs(th[2] - tt[2]) < 1e-5 and abs(th[3] - tt[3]) < 1e-6


def test_p11_held_parameters_on_linear_least_squares():
    """On a linear model the fit with some parameters held converges to the weighted
    least-squares solution over the free columns, the held values moved to the data side
    (numpy.linalg.lstsq)."""
    g = np.random.default_rng(12)
    X = g.normal(size=(40, 4))
    d = g.normal(size=40)
    w = g.uniform(0.5, 2.0, 40)

    class Lin(oracle.FitOracle):
        def __init__(self):
            pass

        def evaluate(self, batch, z, q, data, inv_sigma2):
            r = d - X @ q
            return float(np.sum(w * r * r)), X.T @ (w[:, None] * X), X.T @ (w * r)

    q0 = np.array([0.3, np.log(2.0), -1.0, 0.5])
    for free in ([True, True, False, True], [False, True, True, False], [True, False, False, False]):
        fr = np.flatnonzero(free)
        hd = np.flatnonzero(~np.asarray(free))
        sw = np.sqrt(w)
        rhs = d - X[:, hd] @ q0[hd]
        sol = np.linalg.lstsq(sw[:, None] * X[:, fr], sw * rhs, rcond=None)[0]
        res = Lin().fit(None, 0.0, [q0[0], np.exp(q0[1]), q0[2], q0[3]], d, w, iters=60, free=free)
        q = np.array([res["theta"][0], np.log(res["theta"][1]), res["theta"][2], res["theta"][3]])
        np.testing.assert_allclose(q[fr], sol, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(q[hd], q0[hd], rtol=1e-15, atol=0)


def test_p11_lm_iterates_on_linear_least_squares():
    """On a linear model every LM iterate has a closed form: q1 = q0 + (H + lam0 diag H)^-1 g,
    lambda shrinks by 10 after an accepted step and grows by 10 after a rejected one."""
    g = np.random.default_rng(11)
    X = g.normal(size=(30, 4))
    d = g.normal(size=30)
    w = g.uniform(0.5, 2.0, 30)

    class Lin(oracle.FitOracle):
        def __init__(self):
            pass

        def evaluate(self, batch, z, q, data, inv_sigma2):
            r = d - X @ q
            return float(np.sum(w * r * r)), X.T @ (w[:, None] * X), X.T @ (w * r)

    fo = Lin()
    H = X.T @ (w[:, None] * X)
    q0 = np.array([0.3, np.log(2.0), -1.0, 0.5])
    chi = lambda q: float(np.sum(w * (d - X @ q) ** 2))
    # expected sequence, computed with numpy.linalg.solve (not the oracle's Cholesky)
    q, lam, seq = q0.copy(), 1e-3, []
    for _ in range(4):
        gq = X.T @ (w * (d - X @ q))
        qt = q + np.linalg.solve(H + lam * np.diag(np.diag(H)), gq)
        if chi(qt) < chi(q):
            q, lam = qt, lam * 0.1
        else:
            lam = lam * 10.0
        seq.append(q.copy())
    for n in range(1, 5):
        res = fo.fit(None, 0.0, [q0[0], 2.0, q0[2], q0[3]], None, None, iters=n)
        th = res["theta"]
        got = np.array([th[0], np.log(th[1]), th[2], th[3]])
        np.testing.assert_allclose(got, seq[n - 1], rtol=1e-10, atol=1e-12)
    # the first step differs from the undamped Gauss-Newton step by the damping term
    gn = q0 + np.linalg.solve(H, X.T @ (w * (d - X @ q0)))
    assert np.max(np.abs(seq[0] - gn)) > 1e-6


def test_tiny_exact_fixture_is_its_own_exact_derivation():
    """The stored P10 value equals an exact rational re-derivation (no oracle, no GPU involved)."""
    import importlib.util
    import json
    from fractions import Fraction
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_exact_derivation.py")
    spec = importlib.util.spec_from_file_location("tiny_exact_derivation", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(mod.PATH) as fh:
        fx = json.load(fh)
    stored = Fraction(fx["expected_flux_times_hc"]["num"], fx["expected_flux_times_hc"]["den"])
    assert mod.derive(fx) == stored


# ----------------------------------------------------------------------------- D6 colour law, D8 hc, R7 edge cells



def test_colour_law_polynomial_values_and_slopes():
    """CL(mu) = a1 r + a2 r^2 + a3 r^3 with r = (mu - lam_B)/(lam_V - lam_B), evaluated by hand at
    r = 0, 1, 2 and -1 (values) and its mu-slope at the same points."""
    a1, a2, a3 = -0.93, 0.047, -0.0061
    md = synth.Model(m0=np.ones((4, 4), np.float32), m1=np.zeros((4, 4), np.float32),
                     cl_coef=np.array([a1, a2, a3]))
    span = 1125.98                                   # lam_V - lam_B, by hand
    mu = np.array([LAM_B, LAM_V, LAM_B + 2 * span, LAM_B - span])
    cl, dcl = oracle.colour_law(md, mu, deriv=True)
    want = [0.0, a1 + a2 + a3, 2 * a1 + 4 * a2 + 8 * a3, -a1 + a2 - a3]
    np.testing.assert_allclose(cl, want, rtol=1e-12, atol=1e-15)
    want_d = np.array([a1, a1 + 2 * a2 + 3 * a3, a1 + 4 * a2 + 12 * a3, a1 - 2 * a2 + 3 * a3]) / span
    np.testing.assert_allclose(dcl, want_d, rtol=1e-12)


@pytest.mark.parametrize("z,c", [(0.0, 0.3), (0.25, -0.2), (0.6, 0.45)])
def test_colour_closed_form_linear_law(z, c):
    """c != 0 closed form: flat M0 = K, top-hat T on [a, b], linear colour law a1 r.  The integrand
    K x0 s exp(c a1 (lam s - lam_B)/(lam_V - lam_B)) lam / hc integrates exactly to
    e^{beta} [e^{kappa lam}(lam/kappa - 1/kappa^2)]_a^b; trapezoid values on refined grids,
    Richardson-extrapolated, reach it, and the 5 A value is within its O(Delta^2) error."""
    K, a1 = 0.75, -0.92              # K exact in float32 (the surface is stored in float32)
    md = const_model(K, cl=(a1,))
    a, bnd = 3900.0, 5150.0
    x0 = 2e-5
    bt = one_sn_batch(np.float32([2.5]), 0, z=z, t0=0.0, x0=x0, x1=0.0, c=c)
    zf, cf, x0f = (float(np.float32(v)) for v in (z, c, x0))
    s = 1.0 / (1.0 + zf)
    kap = cf * a1 * s / (LAM_V - LAM_B)
    beta = -cf * a1 * LAM_B / (LAM_V - LAM_B)
    prim = lambda L: np.exp(kap * L) * (L / kap - 1.0 / kap ** 2)
    exact = x0f * s * K * np.exp(beta) * (prim(bnd) - prim(a)) / HC_LITERAL
    vals = [oracle.Oracle(md, [synth.tophat_band(a, bnd)], spacing=sp).bandflux(bt)[0] for sp in (5.0, 2.5, 1.25)]
    rich = (4 * vals[2] - vals[1]) / 3
    np.testing.assert_allclose(rich, exact, rtol=1e-8)
    # the plain 5 A trapezoid differs by its Euler-Maclaurin term Delta^2 [g'(b) - g'(a)] / 12,
    # g(lam) = lam e^{kappa lam}, g' = (1 + kappa lam) e^{kappa lam}
    gp = lambda L: (1.0 + kap * L) * np.exp(kap * L)
    scale = x0f * s * K * np.exp(beta) / HC_LITERAL
    em = 25.0 / 12.0 * (gp(bnd) - gp(a)) * scale
    np.testing.assert_allclose(vals[0] - exact, em, rtol=2e-3, atol=2e-9 * abs(exact))
    bound = abs(em)
    # and the colour term is really present: the c = 0 flux differs by far more than that
    f0 = oracle.Oracle(md, [synth.tophat_band(a, bnd)]).bandflux(one_sn_batch([2.5], 0, z=z, x0=x0, x1=0.0, c=0.0))
    assert abs(f0[0] - exact) > 100 * bound


def test_colour_cubic_law_against_adaptive_quadrature(model):
    """c != 0 with the cubic colour law written out in this test (not through the oracle):
    Richardson-extrapolated trapezoid values equal scipy.quad on the continuous integrand."""
    a_lo, a_hi = 4210.0, 5570.0
    band = synth.tophat_band(a_lo, a_hi)
    z, x0, c = 0.2, 1e-5, 0.35
    K = 1.25
    a1, a2, a3 = (float(v) for v in model.cl_coef)
    md = const_model(K, cl=(a1, a2, a3))
    bt = one_sn_batch([0.0], 0, z=z, x0=x0, x1=0.0, c=c)
    zf, x0f, cf = (float(np.float32(v)) for v in (z, x0, c))
    s = 1.0 / (1.0 + zf)

    def integrand(lam):
        r = (lam * s - LAM_B) / (LAM_V - LAM_B)
        cl = a1 * r + a2 * r * r + a3 * r * r * r
        return x0f * s * K * np.exp(cf * cl) * lam / HC_LITERAL

    ref = integrate.quad(integrand, a_lo, a_hi, epsabs=0, epsrel=1e-13)[0]
    vals = [oracle.Oracle(md, [band], spacing=sp).bandflux(bt)[0] for sp in (5.0, 2.5, 1.25)]
    rich = (4 * vals[2] - vals[1]) / 3
    np.testing.assert_allclose(rich, ref, rtol=1e-8)


def test_hc_is_the_physical_constant():
    """Flat spectrum through a top-hat with hc written as the literal CODATA value: the oracle's
    flux equals x0 K (b^2 - a^2) / (2 hc (1+z)) to the literal's 9 digits."""
    K = 0.5
    md = const_model(K)
    a, bnd = 4400.0, 6100.0
    o = oracle.Oracle(md, [synth.tophat_band(a, bnd)])
    bt = one_sn_batch(np.float32([1.0, 11.0]), 0, z=0.5, t0=0.0, x0=1e-5, x1=0.0, c=0.0)
    want = float(np.float32(1e-5)) * K * (bnd ** 2 - a ** 2) / (2 * HC_LITERAL * 1.5)
    np.testing.assert_allclose(o.bandflux(bt), want, rtol=5e-9)
    assert abs(oracle.HC / HC_LITERAL - 1.0) < 5e-9


def _edge_points(n, g, m):
    """m points in each of the first and last cells (0, 1) and (n-2, n-1), kept off the nodes."""
    return np.r_[g.uniform(0.05, 0.95, m), g.uniform(n - 1.95, n - 1.05, m)]


def test_edge_cell_derivatives_vs_central_differences():
    """dI/du and dI/dv in the first and last cell of each axis (linear there) against FP64 central
    differences taken inside the cell."""
    g = np.random.default_rng(21)
    n_p, n_w = 9, 11
    M = g.normal(size=(n_p, n_w))
    h = 1e-6
    # phase edge cells, wavelength interior and edge
    for u, v in ((_edge_points(n_p, g, 20), g.uniform(1.0, n_w - 2.0, 40)),
                 (g.uniform(1.0, n_p - 2.0, 40), _edge_points(n_w, g, 20)),
                 (_edge_points(n_p, g, 20), _edge_points(n_w, g, 20))):
        _, du, dv = oracle.interp2(M, u, v, deriv=True)
        fd_u = (oracle.interp2(M, u + h, v) - oracle.interp2(M, u - h, v)) / (2 * h)
        fd_v = (oracle.interp2(M, u, v + h) - oracle.interp2(M, u, v - h)) / (2 * h)
        np.testing.assert_allclose(du, fd_u, rtol=0, atol=1e-8)
        np.testing.assert_allclose(dv, fd_v, rtol=0, atol=1e-8)
        # in an edge cell the derivative along that axis is the node difference (linear piece)
    u = np.array([0.3, n_p - 1.7])
    _, du, _ = oracle.interp2(M, u, np.array([4.0, 4.0]), deriv=True)
    np.testing.assert_allclose(du, [M[1, 4] - M[0, 4], M[n_p - 1, 4] - M[n_p - 2, 4]], rtol=1e-13)


def test_edge_cell_partials_of_the_bandflux(model):
    """d f/d t0 for observations in the first and last phase cell, and d f/dz for bands whose rest
    window reaches the first or last wavelength cell, against FP64 central differences."""
    lo_band = synth.tophat_band(2004.0 * 1.3, 2600.0 * 1.3)     # rest window starts in cell 0 at z = 0.3
    hi_band = synth.tophat_band(8600.0 * 1.3, 9197.0 * 1.3)     # rest window ends in the last cell
    o = oracle.Oracle(model, [lo_band, hi_band])
    t = np.float32([-19.6 * 1.3, -19.2 * 1.3, 49.3 * 1.3, 49.8 * 1.3, 10.0 * 1.3])
    for bd in (0, 1):
        b = one_sn_batch(t, bd, z=0.3, t0=0.0, x0=1e-5, x1=0.4, c=0.1)
        P = b.params().astype(np.float64)
        f, J = o.jac(b, P)
        for q, h in ((1, 1e-5), (0, 1e-7)):
            Pp, Pm = P.copy(), P.copy()
            Pp[:, q] += h
            Pm[:, q] -= h
            fd = (o.bandflux(b, Pp) - o.bandflux(b, Pm)) / (2 * h)
            sc = np.abs(J[:, q]).max()
            assert np.max(np.abs(fd - J[:, q])) <= 1e-6 * sc, (bd, q, np.max(np.abs(fd - J[:, q])) / sc)

"""Input generators: determinism, sizes and eligibility (CPU only)."""
import numpy as np
import pytest

import synth


def test_deterministic_and_shapes():
    a = synth.batch_4096_sn(n_sn=50)
    b = synth.batch_4096_sn(n_sn=50)
    assert np.array_equal(a.t, b.t) and np.array_equal(a.band, b.band) and np.array_equal(a.z, b.z)
    assert a.sn_offsets[0] == 0 and a.sn_offsets[-1] == a.n_obs
    n = np.diff(a.sn_offsets)
    assert n.min() >= 20 and n.max() <= 200
    for arr in (a.z, a.t0, a.x0, a.x1, a.c, a.t):
        assert arr.dtype == np.float32
    assert a.band.dtype == np.int32 and a.sn_offsets.dtype == np.int32


def test_batch_4096_size_and_eligibility(model, bands6):
    b = synth.batch_4096_sn()
    assert b.n_sn == 4096 and 400_000 < b.n_obs < 500_000
    # every observation's band keeps its rest window inside the surface grid
    for s in range(0, b.n_sn, 97):
        lo, hi = b.sn_offsets[s], b.sn_offsets[s + 1]
        el = set(synth.eligible_bands(float(b.z[s]), bands6, model))
        assert set(np.unique(b.band[lo:hi])) <= el
        # sorted by (band, t)
        assert np.all(np.diff(b.band[lo:hi]) >= 0)


def test_one_sn_and_sweep():
    c1 = synth.one_sn_40_obs()
    assert c1.n_sn == 1 and c1.n_obs == 40 and set(c1.band) == {0, 1, 2, 3}
    sw = synth.sweep_120_obs(n_samples=1000)
    assert len(sw.obs_t) == 120 and sw.samples.n_sn == 1000
    assert sw.samples.z.max() < 0.75


def test_make_data_sigma_rule():
    f = np.array([1.0, -2.0, 100.0, 0.0, 5.0])
    off = np.array([0, 3, 5])
    d, sig, w = synth.make_data(f, off, np.zeros(5))
    np.testing.assert_allclose(sig, np.float32([0.05, 0.1, 5.0, 0.05 * 0.05, 0.25]), rtol=1e-6)
    np.testing.assert_allclose(d, f)


@pytest.mark.parametrize("which", ["batch_4096_sn", "batch_65536_sn"])
def test_perturbed_batches_keep_every_band_window_on_the_grid(which):
    """The gradient workloads evaluate at perturbed parameters: after the redshift steps every
    observed band's rest-frame window [lo/(1+z), hi/(1+z)] (z as the float32 the GPU gets) still
    lies on the surface grid, so no evaluation is a range error."""
    model, bands = synth.make_model(), synth.make_bands(6)
    base = getattr(synth, which)()
    for k in (3, 7):
        b = synth.perturb(base, k=k)
        z = b.z.astype(np.float64)
        n_s = np.diff(b.sn_offsets)
        sn_of = np.repeat(np.arange(b.n_sn), n_s)
        lo = np.array([bd.lo for bd in bands])[b.band] / (1.0 + z[sn_of])
        hi = np.array([bd.hi for bd in bands])[b.band] / (1.0 + z[sn_of])
        assert lo.min() >= model.wave0 and hi.max() <= model.wave_max, (which, k)

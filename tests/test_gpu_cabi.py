"""The C ABI driven from a plain C++ program (tests/c_abi/sb_cabi_check.cpp), without Python or
torch in the process: its fluxes and cotangent gradients against the FP64 oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from gpu_util import FLUX_TOL, GRAD_TOL, flux_rel_err, grad_norm_err

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "sb_cabi_check")


def write_input(path, model, bands, b, cot):
    with open(path, "wb") as f:
        np.array([model.m0.shape[0], model.m0.shape[1], len(model.cl_coef), len(bands), b.n_sn, b.n_obs],
                 np.int32).tofile(f)
        np.array([model.phase0, model.dphase, model.wave0, model.dwave, model.cl_wave_b, model.cl_wave_v],
                 np.float64).tofile(f)
        np.asarray(model.cl_coef, np.float64).tofile(f)
        np.ascontiguousarray(model.m0, np.float32).tofile(f)
        np.ascontiguousarray(model.m1, np.float32).tofile(f)
        for bd in bands:
            np.array([len(bd.wave)], np.int32).tofile(f)
            np.asarray(bd.wave, np.float64).tofile(f)
            np.asarray(bd.trans, np.float64).tofile(f)
        for a in (b.z, b.t0, b.x0, b.x1, b.c, b.t):
            np.asarray(a, np.float32).tofile(f)
        np.asarray(b.band, np.int32).tofile(f)
        np.asarray(b.sn_offsets, np.int32).tofile(f)
        np.asarray(cot, np.float32).tofile(f)


def test_c_program_matches_oracle(tmp_path, model, bands6):
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi/sb_cabi_check is not built (run the package build)")
    b = synth.random_batch(41, 24, 1, 120, bands6, model)
    cot = np.random.default_rng(41).normal(size=b.n_obs).astype(np.float32)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    write_input(inp, model, bands6, b, cot)
    print(f"case: C ABI program, {b.n_sn} SN, {b.n_obs} obs", flush=True)
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    res = np.fromfile(out, np.float32)
    flux, grad = res[:b.n_obs], res[b.n_obs:].reshape(b.n_sn, 5)
    o6 = oracle.Oracle(model, bands6)
    f64, J64 = o6.jac(b)
    g64 = oracle.segment_sum(cot.astype(np.float64)[:, None] * J64, b.sn_offsets)
    assert flux_rel_err(flux, f64, b.sn_offsets).max() <= FLUX_TOL
    assert grad_norm_err(grad, g64, b.x0).max() <= GRAD_TOL

"""Exact re-derivation of tests/golden/tiny_exact.json's expected value with rational arithmetic.

It follows the fixture's hand derivation step by step (phase and amplitude from the model
equation, trapezoid quadrature on the band grid, Catmull-Rom weights at a half-cell and at a
node) and uses neither the oracle nor the HIP library, so the stored value pins both.

    python tests/golden/tiny_exact_derivation.py          # check the stored value
    python tests/golden/tiny_exact_derivation.py --write  # rewrite it
"""
import json
import math
import os
import sys
from fractions import Fraction as Fr

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "tiny_exact.json")


def catmull_rom(x: Fr):
    """Weights of nodes a-1..a+2 at fraction x of an interior cell (Keys, a = -1/2)."""
    return [((-Fr(1, 2) * x + 1) * x - Fr(1, 2)) * x,
            (Fr(3, 2) * x - Fr(5, 2)) * x * x + 1,
            ((-Fr(3, 2) * x + 2) * x + Fr(1, 2)) * x,
            (Fr(1, 2) * x - Fr(1, 2)) * x * x]


def derive(fx):
    srf, prm, bnd = fx["surface"], fx["params"], fx["band"]
    assert srf["phase0"] == 0 and srf["dphase"] == 1 and srf["wave0"] == 0 and srf["dwave"] == 1
    assert fx["colour_law"]["coef"] == [0.0] and prm["c"] == 0.0   # E = exp(c CL) = 1
    s = 1 / (1 + Fr(prm["z"]))
    amp = Fr(prm["x0"]) * s
    x1 = Fr(prm["x1"])
    mx = [[Fr(a) + x1 * Fr(b) for a, b in zip(r0, r1)] for r0, r1 in zip(srf["m0"], srf["m1"])]
    n_phase, n_wave = srf["n_phase"], srf["n_wave"]

    def interp1(vals, u):
        """Catmull-Rom along one axis at grid coordinate u, in an interior cell."""
        a = math.floor(u)
        assert 1 <= a <= len(vals) - 3, "interior cells only"
        w = catmull_rom(u - a)
        return sum(wi * vals[a - 1 + i] for i, wi in enumerate(w))

    u = (Fr(fx["obs_t"]).limit_denominator(1 << 20) - Fr(prm["t0"]).limit_denominator(1 << 20)) * s
    rows = [interp1([mx[a][j] for a in range(n_phase)], u) for j in range(n_wave)]

    # band grid: N = ceil((U - L)/spacing) equal intervals, T linear between samples, trapezoid weights
    wave, trans = [Fr(w) for w in bnd["wave"]], [Fr(t).limit_denominator(1 << 20) for t in bnd["trans"]]
    lo, hi = wave[0], wave[-1]
    n = math.ceil((hi - lo) / Fr(bnd["spacing"]).limit_denominator(1 << 20))
    dl = (hi - lo) / n
    total = Fr(0)
    for k in range(n + 1):
        lam = lo + k * dl
        i = max(i for i in range(len(wave) - 1) if wave[i] <= lam) if lam < hi else len(wave) - 2
        t = trans[i] + (trans[i + 1] - trans[i]) * (lam - wave[i]) / (wave[i + 1] - wave[i])
        wk = dl / 2 if k in (0, n) else dl
        mu = lam * s
        v = rows[int(mu)] if mu.denominator == 1 else interp1(rows, mu)
        total += wk * lam * t * v
    return amp * total


def main():
    with open(PATH) as fh:
        fx = json.load(fh)
    val = derive(fx)
    stored = Fr(fx["expected_flux_times_hc"]["num"], fx["expected_flux_times_hc"]["den"])
    if "--write" in sys.argv:
        fx["expected_flux_times_hc"] = {"num": val.numerator, "den": val.denominator}
        with open(PATH, "w") as fh:
            json.dump(fx, fh, indent=2)
        print("written", val)
        return 0
    print("derived", val, "stored", stored)
    return 0 if val == stored else 1


if __name__ == "__main__":
    sys.exit(main())

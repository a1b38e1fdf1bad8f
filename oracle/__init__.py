"""Plain FP64 CPU oracle of the SALT bandflux path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``, never by the library.  It shares
no code with the HIP path; both are fed from the input generators in ``synth``.

Every function is pinned by the ``-m "not gpu"`` tests against closed forms,
invariants and brute-force exact rational evaluation (tests/test_oracle_pins.py).
"""
from .salt64 import FNU_AB, HC, Oracle, ab_zeropoint, band_grid, colour_law, interp2, segment_sum  # noqa: F401
from .fit64 import FitOracle  # noqa: F401
from .lbfgsb64 import lbfgsb  # noqa: F401

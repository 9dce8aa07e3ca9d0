"""Plain FP64 CPU oracle for the DMPT Bethe-Salpeter (TDA) force path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the only
module both sides use is ``synth`` (seeded inputs, no method arithmetic).

Everything is written for readability against the paper, not for speed:

* ``basis``   the real plane-wave basis of the Gamma-point wavefunction sphere
              and the grid transforms (numpy FFT), plus an explicit cos/sin
              basis matrix used as an independent route.
* ``model``   the synthetic Kohn-Sham Hamiltonian, the screened interaction W
              of Eq. 3 and the DMPT operator D + s K1e - K1d of Eqs. 1-2.
* ``dense``   the conventional electron-hole BSE matrix built from explicit
              DFT and basis matrices and every conduction state (the plain
              definition the DMPT operator must reproduce exactly).
* ``solvers`` Davidson, the U vector (SM Sec. I), the Z-vector CG (Eq. 7),
              the force contraction (Eqs. 4-6) and central finite differences.

Pins (tests/test_oracle_*.py) fix each function against closed forms, the
dense electron-hole matrix, special cases of the Table S-I kind and finite
differences.  Functions without such a pin say so in their docstring with
the phrase "parity unpinned".
"""
from . import basis, model, dense, solvers  # noqa: F401

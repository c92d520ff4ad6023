"""CPU oracle for the liquid-vapour lattice Boltzmann update (FP64, slow, plain).

TEST INFRASTRUCTURE ONLY.  Only tests/, the package smoke check and the
CPU-baseline leg of bench.py may import, call or execute anything under oracle/.
The product library (paper_2106_01557_amd) must never import it, link it or fall
back to it; the two share no code.

Modules
  thermo  equation of state, Maxwell coexistence, square-gradient sigma and W,
          derived model constants (mpmath, arbitrary precision)
  lbm     the lattice update in moment space with explicit 9x9 matrices (numpy FP64)

Parity status of each function is recorded in the test suite; every function
here is pinned by at least one check that does not re-use its own formula.
"""
from . import thermo, lbm  # noqa: F401

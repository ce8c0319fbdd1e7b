"""FP64 CPU oracle for the adaptively compressed exchange (ACE) build.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it, links it or falls back to it, and the two share no code.

Everything here is plain NumPy/SciPy in float64 / complex128, written from
the paper (L. Lin, "Adaptively Compressed Exchange Operator", J. Chem. Theory
Comput. 2016) for a reader to check by eye:

* exchange operator applied by pair Poisson solves     Section 2, Eq. (applyVX2)
* exchange kernel and its Hadamard (dense) form         Section 2, Eq. (VXkernel)
* screened short-range kernel erfc(mu r)/r               Section 2, Eq. (EXSR)
* W_i = V_X[phi] phi_i                                  Section 3, Eq. (W)
* M, Cholesky -M = L L^H, xi = W L^{-H}                  Section 3, Eqs. (ACEconstruct2), (Wtilde)
* V_ACE = -xi xi^H                                      Section 3, Eq. (ACE)
* E_X directly and from the projection vectors           Eqs. (EX), (EX_ACE)
* oversampling N_band > N_occ                            end of Section 3
* the self-consistent loops around the exchange          Alg. 1 (V_X), Alg. 2 (V_ACE),
  operator with a linear eigensolver (oracle.scf_oracle)  Eq. (HFlineig)

Pins against facts fixed outside this package live in tests/test_oracle_*.py.
"""
from .ace_oracle import *  # noqa: F401,F403

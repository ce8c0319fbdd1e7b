"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Run from the repository root:  python tests/golden/make_golden.py
Only the oracle and the seeded input generator are called.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_1601_07159_amd import synth  # noqa: E402


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    psi = synth.smooth_orbitals(24, 10.0, 8, seed=0)
    g = O.Grid.cubic(24, 10.0)
    ge = O.Grid.cubic(24, 10.0, "erfc", 0.106)
    W = O.build_W(psi, psi, g)
    M, L, xi = O.compress(psi, W, g)
    out = {
        "case": "24^3 grid, cubic L=10 bohr, 8 smooth orthonormal orbitals "
                "(Ecut 10 Ha, seed 0), N_occ = N_band = 8",
        "E_X_coulomb": O.exchange_energy_direct(psi, g),
        "E_X_erfc_mu0.106": O.exchange_energy_direct(psi, ge),
        "eig_minus_M": [float(v) for v in np.linalg.eigvalsh(-M)],
        "W_fro": float(np.linalg.norm(W)),
        "planewaves_in_sphere": int(np.count_nonzero(np.abs(np.fft.fftn(psi[0])) > 1e-12)),
    }
    with open(os.path.join(here, "smooth24_seed0.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")

    # 48^3, L = 20.5 bohr, 80 orbitals (seed 0), N_occ = 64: exchange energy
    psi = synth.smooth_orbitals(48, 20.5, 80, seed=0)
    g = O.Grid.cubic(48, 20.5)
    out = {
        "case": "48^3 grid, cubic L=20.5 bohr, 80 smooth orthonormal orbitals (Ecut 10 Ha, "
                "seed 0); occupied = first 64",
        "E_X_coulomb_nocc64": O.exchange_energy_direct(psi[:64], g),
    }
    with open(os.path.join(here, "smooth48_seed0.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()

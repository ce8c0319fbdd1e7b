"""Pins of the oracle's self-consistent loops (Alg. 1 with V_X applied
directly, Alg. 2 with V_ACE; Section 2 Eq. HFlineig with a fixed local
potential) against facts fixed outside the loop code:

* a constant potential without exchange has the plane-wave spectrum
  1/2 |k|^2 + V_0 (the spectral Laplacian and the whole eigensolver);
* the Chebyshev filter multiplies an eigenvector by T_m((t - c)/e) /
  T_m((a0 - c)/e) (numpy's Chebyshev series);
* the loops with V_X and with V_ACE converge to the same fixed point (the
  paper's claim that ACE does not change the self-consistent solution);
* that fixed point solves the Hartree-Fock-like equations with the exact
  exchange operator of its own occupied orbitals (oracle build_W).
"""
import numpy as np
import pytest

import oracle as O
from oracle import scf_oracle as S
from paper_1601_07159_amd import synth


def test_constant_potential_gives_planewave_levels():
    n, L, v0 = 12, 7.0, -0.4
    g = O.Grid.cubic(n, L)
    X0 = synth.smooth_orbitals(n, L, 10, seed=1)
    r = S.scf(g, np.full((n, n, n), v0), X0, 7, 0.0, "none", 8, 12, 1)
    k2 = (2.0 * np.pi / L) ** 2
    exact = np.array([v0] + [v0 + 0.5 * k2] * 6)
    assert np.max(np.abs(r["ritz"][-1][:7] - exact)) <= 1e-8


def test_filter_scales_an_eigenvector_by_the_chebyshev_ratio():
    n, L, v0 = 8, 5.0, 0.3
    g = O.Grid.cubic(n, L)
    m = (1, -2, 0)
    pw = synth.planewave_orbitals(n, L, [m])
    lam = v0 + 0.5 * (2 * np.pi / L) ** 2 * sum(x * x for x in m)
    vloc = np.full((n, n, n), v0)
    a, b, a0, deg = lam + 0.7, 40.0, lam - 0.2, 7
    Y = S.chebyshev_filter(pw, lambda Z: S.apply_h(Z, g, vloc), deg, a, b, a0)
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    coef = np.zeros(deg + 1)
    coef[-1] = 1.0
    ratio = np.polynomial.chebyshev.chebval((lam - c) / e, coef) / \
        np.polynomial.chebyshev.chebval((a0 - c) / e, coef)
    assert np.max(np.abs(Y - ratio * pw)) <= 1e-12 * np.max(np.abs(pw)) * max(1.0, abs(ratio))


@pytest.fixture(scope="module")
def loops():
    n, L = 12, 7.0
    g = O.Grid.cubic(n, L, "erfc", 0.3)
    vloc = synth.local_potential(n, L, 5, depth=1.5)
    X0 = synth.smooth_orbitals(n, L, 8, seed=2)
    out = {m: S.scf(g, vloc, X0, 4, 0.25, m, 8, 4, 16, n_band=6) for m in ("vx", "ace")}
    return g, vloc, out


def test_ace_and_direct_exchange_reach_the_same_fixed_point(loops):
    _, _, r = loops
    ev, ea = r["vx"]["E_X"][-1], r["ace"]["E_X"][-1]
    assert abs(ev - ea) <= 1e-9 * abs(ev)
    assert np.max(np.abs(r["vx"]["ritz"][-1][:6] - r["ace"]["ritz"][-1][:6])) <= 1e-9
    # and the outer loop did converge
    assert abs(r["vx"]["E_X"][-1] - r["vx"]["E_X"][-2]) <= 1e-9 * abs(ev)


def test_fixed_point_solves_the_exchange_equations(loops):
    g, vloc, r = loops
    X = r["vx"]["X"]
    phi = X[:4]
    HX = S.apply_h(phi, g, vloc) + O.build_W(phi, phi, g, scale=0.25)
    nb = phi.shape[0]
    S_ = g.dV * (phi.reshape(nb, -1).conj() @ HX.reshape(nb, -1).T)
    res = HX.reshape(nb, -1) - S_.T @ phi.reshape(nb, -1)
    assert np.linalg.norm(res) * np.sqrt(g.dV) <= 1e-6
    # the projected Hamiltonian is diagonal in the Ritz basis
    off = S_ - np.diag(np.diag(S_))
    assert np.max(np.abs(off)) <= 1e-8

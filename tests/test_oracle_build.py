"""Pins of the oracle's W = V_X[phi] psi (Eqs. applyVX2, W) against facts
fixed outside its FFT arithmetic:

* the plane-wave closed form (eigenvalues summed from the kernel formula)
* the dense real-space form -(Phi Phi^H) o C built from explicit DFT sums
  (Eq. VXkernel), on tiny non-cubic grids
* invariants: unitary mixing of phi (V_X depends on the density matrix only),
  linearity in psi, Hermitian projected matrix, negative semidefiniteness.
"""
import numpy as np
import pytest

import oracle as O
from paper_1601_07159_amd import synth


def _pw_set(nocc, nband, n, seed=0):
    rng = np.random.default_rng(seed)
    seen, out = set(), []
    while len(out) < nband:
        m = tuple(int(v) for v in rng.integers(-(n // 2), n // 2, size=3))
        if m not in seen:
            seen.add(m)
            out.append(m)
    return out[:nocc], out


@pytest.mark.parametrize("kind,mu,g0", [("coulomb", 0.0, 0.0), ("erfc", 0.3, 0.0),
                                        ("coulomb", 0.0, 2.5), ("erfc", 0.106, np.pi / 0.106 ** 2)])
def test_planewave_closed_form(kind, mu, g0):
    n, L = 8, 6.0
    g = O.Grid.cubic(n, L, kind, mu, g0)
    occ, allm = _pw_set(5, 9, n)
    phi = synth.planewave_orbitals(n, L, occ)
    psi = synth.planewave_orbitals(n, L, allm)
    W = O.build_W(phi, psi, g)
    lam = O.planewave_exchange_eigs(occ, allm, g)
    ref = lam[:, None, None, None] * psi
    assert np.linalg.norm(W - ref) <= 1e-13 * np.linalg.norm(ref)


def test_planewave_folding_near_nyquist():
    # differences k_j - k_i beyond the Nyquist range must fold back onto the grid
    n, L = 6, 4.0
    g = O.Grid.cubic(n, L)
    occ = [(2, 2, -3), (-3, 1, 2)]
    allm = occ + [(-3, -3, -3), (2, -3, 1)]
    phi = synth.planewave_orbitals(n, L, occ)
    psi = synth.planewave_orbitals(n, L, allm)
    W = O.build_W(phi, psi, g)
    lam = O.planewave_exchange_eigs(occ, allm, g)
    np.testing.assert_allclose(W, lam[:, None, None, None] * psi, atol=1e-13)


def test_rotated_planewaves_closed_form():
    # Phi = PW U, Psi = PW U': V_X[Phi] = V_X[PW] and W = PW diag(lam) U'
    n, L = 8, 5.0
    g = O.Grid.cubic(n, L)
    occ, allm = _pw_set(4, 7, n, seed=4)
    pw_occ = synth.planewave_orbitals(n, L, occ)
    pw_all = synth.planewave_orbitals(n, L, allm)
    U = synth.random_unitary(4, 1)
    Up = synth.random_unitary(7, 2)
    phi = np.einsum("ab,a...->b...", U, pw_occ)
    psi = np.einsum("ab,a...->b...", Up, pw_all)
    W = O.build_W(phi, psi, g)
    lam = O.planewave_exchange_eigs(occ, allm, g)
    ref = np.einsum("ab,a...->b...", Up, lam[:, None, None, None] * pw_all)
    assert np.linalg.norm(W - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind,mu,g0", [("coulomb", 0.0, 0.0), ("erfc", 0.7, 0.4)])
def test_fft_form_equals_dense_form(kind, mu, g0):
    n, L = (6, 4, 5), (5.0, 4.0, 6.0)
    g = O.Grid(n, L, kind, mu, g0)
    rng = np.random.default_rng(7)
    shape = (3,) + n
    phi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    psi = rng.standard_normal((4,) + n) + 1j * rng.standard_normal((4,) + n)
    W = O.build_W(phi, psi, g)
    Wd = O.build_W_dense(phi, psi, g)
    assert np.linalg.norm(W - Wd) <= 1e-13 * np.linalg.norm(Wd)


def test_exchange_operator_negative_semidefinite_and_rank_full():
    g = O.Grid.cubic(4, 3.0)
    phi = synth.smooth_orbitals(4, 3.0, 3, seed=1, ecut=40.0)
    VX = O.exchange_matrix_dense(phi, g)
    np.testing.assert_allclose(VX, VX.conj().T, atol=1e-14)
    ev = np.linalg.eigvalsh(VX)
    assert ev.max() <= 1e-12 * abs(ev.min())
    # full rank well beyond N_occ (Hadamard product with the kernel, Section 2)
    assert np.sum(np.abs(ev) > 1e-10 * abs(ev.min())) > 10 * phi.shape[0]


def test_unitary_mixing_of_phi_leaves_W_unchanged():
    g = O.Grid.cubic(8, 5.0)
    phi = synth.smooth_orbitals(8, 5.0, 5, seed=2)
    psi = synth.smooth_orbitals(8, 5.0, 6, seed=3)
    U = synth.random_unitary(5, 9)
    W1 = O.build_W(phi, psi, g)
    W2 = O.build_W(np.einsum("ab,a...->b...", U, phi), psi, g)
    assert np.linalg.norm(W1 - W2) <= 1e-13 * np.linalg.norm(W1)


def test_pair_symmetry_projected_matrix_hermitian():
    # u_ji = conj(u_ij) when psi = phi, so <phi_k, W_l> is Hermitian before any symmetrisation
    g = O.Grid.cubic(10, 6.0, "erfc", 0.5)
    phi = synth.smooth_orbitals(10, 6.0, 6, seed=5)
    W = O.build_W(phi, phi, g)
    M = g.dV * phi.reshape(6, -1).conj() @ W.reshape(6, -1).T
    assert np.linalg.norm(M - M.conj().T) <= 1e-14 * np.linalg.norm(M)
    u_ij = O.pair_potential(phi[1], phi[4], g)
    u_ji = O.pair_potential(phi[4], phi[1], g)
    np.testing.assert_allclose(u_ji, np.conj(u_ij), atol=1e-15 * np.abs(u_ij).max() * 100)


def test_scale_and_linearity_in_psi():
    g = O.Grid.cubic(8, 5.0)
    phi = synth.smooth_orbitals(8, 5.0, 3, seed=2)
    psi = synth.smooth_orbitals(8, 5.0, 4, seed=3)
    A = (np.arange(16).reshape(4, 4) + 1j) / 7.0
    W = O.build_W(phi, psi, g)
    W2 = O.build_W(phi, np.einsum("ab,a...->b...", A, psi), g, scale=0.25)
    np.testing.assert_allclose(W2, 0.25 * np.einsum("ab,a...->b...", A, W), atol=1e-14)


def test_real_orbitals_give_real_operator_and_packed_solve():
    # Gamma-point setting: for real phi, psi the exact operator keeps W real
    # (K(G) real and even), and two real pair charges solved as one complex
    # field rho_a + i rho_b come back as u_a + i u_b -- the identity the
    # real-orbital build relies on
    n, L = 12, 5.5
    g = O.Grid.cubic(n, L, "erfc", 0.4, 0.3)
    psi = synth.real_orbitals(n, L, 5, seed=14)
    W = O.build_W(psi[:3], psi, g)
    assert np.abs(W.imag).max() <= 1e-13 * np.abs(W).max()
    ua = O.pair_potential(psi[0], psi[3], g)
    ub = O.pair_potential(psi[1], psi[3], g)
    K = O.kernel_g(g)
    rho = psi[0] * psi[3] + 1j * psi[1] * psi[3]
    u = np.fft.ifftn(K * np.fft.fftn(rho))
    assert np.abs(ua.imag).max() <= 1e-13 * np.abs(ua).max()
    assert np.abs(u.real - ua.real).max() <= 1e-13 * np.abs(ua).max()
    assert np.abs(u.imag - ub.real).max() <= 1e-13 * np.abs(ub).max()

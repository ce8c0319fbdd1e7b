"""Pins of the oracle's interaction kernel against facts fixed outside it.

* the screened kernel's Fourier transform, by numerical quadrature of the
  real-space erfc(mu r)/r (Section 2, Eq. EXSR)
* the Coulomb Poisson problem, by a real-space finite-difference Laplacian
  (Section 2: applying V_X is a set of Poisson problems, Eq. applyVX)
* limits of the screened kernel (mu -> inf, mu -> 0)
"""
import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
from paper_1601_07159_amd import synth


def _radial_ft_erfc(G, mu):
    # 3-D Fourier transform of a radial f(r) = erfc(mu r)/r:
    #   (4 pi / G) int_0^inf r f(r) sin(G r) dr = (4 pi / G) int_0^inf erfc(mu r) sin(G r) dr
    R = 12.0 / mu                     # erfc(12) ~ 1e-64: the tail is nothing
    val, err = integrate.quad(lambda r: special.erfc(mu * r), 0.0, R, weight="sin",
                              wvar=G, limit=400)
    return 4.0 * np.pi / G * val


@pytest.mark.parametrize("mu", [0.106, 0.5, 1.3])
def test_erfc_kernel_equals_fourier_integral(mu):
    g = O.Grid.cubic(8, 9.0, "erfc", mu)
    K = O.kernel_g(g)
    gaxis = 2 * np.pi * (np.fft.fftfreq(8) * 8) / 9.0
    for idx in [(1, 0, 0), (0, 2, 1), (3, 3, 4), (7, 5, 1)]:
        G = np.sqrt(sum(gaxis[i] ** 2 for i in idx))
        ref = _radial_ft_erfc(G, mu)
        assert abs(K[idx] - ref) <= 1e-9 * abs(ref), (idx, K[idx], ref)


def test_coulomb_kernel_solves_poisson_equation():
    # u = ifftn(K fftn(rho)) must solve -lap u = 4 pi rho for zero-mean rho.
    # Check with a second-order finite-difference Laplacian in real space on a
    # smooth charge: the residual must fall like h^2 as the grid is refined.
    errs = []
    for n in (16, 32, 64):
        L = 7.0
        g = O.Grid.cubic(n, L)
        x = np.arange(n) * L / n
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        rho = (np.cos(2 * np.pi * X / L) * np.sin(4 * np.pi * Y / L)
               + 0.5 * np.cos(2 * np.pi * (Z + X) / L)).astype(complex)
        one = np.ones_like(rho)  # conj(phi_i) = 1, so the pair charge is rho itself
        u = O.pair_potential(one, rho, g)
        h = L / n
        lap = sum(np.roll(u, 1, a) + np.roll(u, -1, a) - 2 * u for a in range(3)) / h ** 2
        errs.append(np.max(np.abs(-lap - 4 * np.pi * rho)) / np.max(np.abs(4 * np.pi * rho)))
    assert errs[-1] < 5e-3
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5  # second order


def test_erfc_limits():
    coul = O.kernel_g(O.Grid.cubic(6, 5.0))
    big = O.kernel_g(O.Grid.cubic(6, 5.0, "erfc", 1e4, g0=0.7))
    small = O.kernel_g(O.Grid.cubic(6, 5.0, "erfc", 1e-4))
    nz = np.ones(coul.shape, bool)
    nz[0, 0, 0] = False
    assert np.max(np.abs(big[nz])) < 1e-6 * np.max(coul)
    assert big[0, 0, 0] == 0.7
    np.testing.assert_allclose(small[nz], coul[nz], rtol=1e-12)


def test_kernel_g0_and_nyquist_symmetry():
    g = O.Grid((6, 8, 4), (4.0, 5.0, 3.0), g0=1.25)
    K = O.kernel_g(g)
    assert K[0, 0, 0] == 1.25
    # K depends on |G| only, so K(G) = K(-G) on the grid (index -m mod n)
    Kneg = K[np.ix_((-np.arange(6)) % 6, (-np.arange(8)) % 8, (-np.arange(4)) % 4)]
    np.testing.assert_array_equal(K, Kneg)


def test_generator_orthonormal_and_smooth():
    g = O.Grid.cubic(12, 6.0)
    psi = synth.smooth_orbitals(12, 6.0, 10, seed=3)
    S = g.dV * psi.reshape(10, -1).conj() @ psi.reshape(10, -1).T
    np.testing.assert_allclose(S, np.eye(10), atol=1e-13)

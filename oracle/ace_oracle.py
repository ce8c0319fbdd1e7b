"""Plain FP64 oracle of the ACE build (test infrastructure only; see package
docstring).  Arrays of orbitals are complex128 with shape (N, n0, n1, n2): N
orbitals, each a field on the periodic real-space grid.

Discretisation (the paper works in the continuum, Section 2): a cell of edges
L0, L1, L2 bohr, N_g = n0 n1 n2 points, volume element dV = Omega / N_g, inner
product <f, g> = dV * sum_r conj(f(r)) g(r).  The paper takes real orbitals;
for complex ones the pair charge in Eq. (applyVX2) is conj(phi_i) psi, the
outer factor is phi_i, and transposes become conjugate transposes.  For real
inputs every formula below reduces to the printed one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

__all__ = [
    "Grid", "kernel_g", "pair_potential", "build_W", "build_W_dense",
    "exchange_matrix_dense", "compress", "ace_apply", "ace_dense",
    "exchange_energy_direct", "exchange_energy_trace", "exchange_energy_ace",
    "exchange_energy_grad", "orthonormalize", "planewave_exchange_eigs",
]


@dataclass(frozen=True)
class Grid:
    """Periodic orthorhombic cell and its real-space grid.

    kind  'coulomb' : kernel 1/|r - r'|                    (Eq. VXkernel)
          'erfc'    : screened kernel erfc(mu |r-r'|)/|r-r'| (Eq. EXSR)
    g0    value used for the G = 0 Fourier component (the Coulomb term
          diverges there; the paper is silent, 0 is the default reading).
    """
    n: tuple
    L: tuple
    kind: str = "coulomb"
    mu: float = 0.0
    g0: float = 0.0

    @staticmethod
    def cubic(n: int, L: float, kind: str = "coulomb", mu: float = 0.0, g0: float = 0.0):
        return Grid((n, n, n), (float(L),) * 3, kind, mu, g0)

    @property
    def ng(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def omega(self) -> float:
        return float(self.L[0] * self.L[1] * self.L[2])

    @property
    def dV(self) -> float:
        return self.omega / self.ng


def _g_axis(n: int, L: float) -> np.ndarray:
    # integer frequency m in FFT order, G = 2 pi m / L
    m = np.fft.fftfreq(n) * n
    return 2.0 * np.pi * m / L


def kernel_g(grid: Grid) -> np.ndarray:
    """Fourier components K(G) of the interaction on the grid, shape n.

    Coulomb 1/r -> 4 pi / |G|^2.  erfc(mu r)/r -> (4 pi/|G|^2)(1 - exp(-|G|^2/(4 mu^2))),
    the only change the paper makes for the short-range hybrid (Section 2,
    after Eq. EXSR).  K(0) = grid.g0.
    """
    gx, gy, gz = (_g_axis(grid.n[a], grid.L[a]) for a in range(3))
    g2 = gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2
    K = np.empty_like(g2)
    nz = g2 > 0.0
    K[nz] = 4.0 * np.pi / g2[nz]
    if grid.kind == "erfc":
        K[nz] *= -np.expm1(-g2[nz] / (4.0 * grid.mu ** 2))
    elif grid.kind != "coulomb":
        raise ValueError(grid.kind)
    K[~nz] = grid.g0
    return K


def pair_potential(phi_i: np.ndarray, psi_j: np.ndarray, grid: Grid, K=None) -> np.ndarray:
    """Solution of one Poisson-type problem of Eq. (applyVX2):
    u(r) = int v(r - r') conj(phi_i(r')) psi_j(r') dr'.

    On the periodic grid the convolution with v is diagonal in Fourier space:
    dV sum_r' v(r - r') f(r') = ifftn(K * fftn(f)) with NumPy's conventions
    (the 1/N_g sits in ifftn; v(r) = Omega^-1 sum_G K(G) exp(iG.r))."""
    if K is None:
        K = kernel_g(grid)
    rho = np.conj(phi_i) * psi_j
    return np.fft.ifftn(K * np.fft.fftn(rho, axes=(-3, -2, -1)), axes=(-3, -2, -1))


def build_W(phi: np.ndarray, psi: np.ndarray, grid: Grid, scale: float = 1.0,
            columns=None) -> np.ndarray:
    """W_j = scale * (V_X[phi] psi_j) = -scale * sum_i phi_i * u_ij  (Eqs. applyVX2, W).

    phi: (N_occ, n0, n1, n2) orbitals defining V_X; psi: (N_band, ...) vectors it
    is applied to (psi = phi gives Eq. W; N_band > N_occ is the oversampled
    case at the end of Section 3).  ``columns`` restricts the output to a
    subset of j (used to time a bounded sample)."""
    K = kernel_g(grid)
    cols = range(psi.shape[0]) if columns is None else columns
    W = np.zeros((len(cols),) + psi.shape[1:], dtype=np.complex128)
    for out, j in enumerate(cols):
        u = pair_potential(phi, psi[j][None], grid, K)   # all i at once
        W[out] = -scale * np.sum(phi * u, axis=0)
    return W


def exchange_matrix_dense(phi: np.ndarray, grid: Grid) -> np.ndarray:
    """Dense N_g x N_g matrix of V_X[phi] (tiny grids only), with no FFT.

    The discrete kernel C[r, r'] = N_g^-1 sum_G K(G) exp(i G.(r - r')) is built
    from explicit exponential sums; then V_X = -(Phi Phi^H) o C, the Hadamard
    product of the density matrix with the kernel (Eq. VXkernel)."""
    K = kernel_g(grid)
    ng = grid.ng
    # fractional coordinates x in [0,1) and integer frequencies m, flattened in C order
    idx = np.indices(grid.n).reshape(3, -1)
    x = idx / np.asarray(grid.n, dtype=float)[:, None]
    m = np.stack([(np.fft.fftfreq(grid.n[a]) * grid.n[a])[idx[a]] for a in range(3)])
    phase = 2.0 * np.pi * (x.T @ m)            # [r, G] = G . r
    E = np.exp(1j * phase)                      # e^{i G.r}
    C = (E * K.reshape(-1)[None, :]) @ E.conj().T / ng
    P = phi.reshape(phi.shape[0], ng).T         # N_g x N_occ
    return -(P @ P.conj().T) * C


def build_W_dense(phi: np.ndarray, psi: np.ndarray, grid: Grid) -> np.ndarray:
    VX = exchange_matrix_dense(phi, grid)
    Y = VX @ psi.reshape(psi.shape[0], grid.ng).T
    return Y.T.reshape(psi.shape)


def compress(psi: np.ndarray, W: np.ndarray, grid: Grid):
    """ACE compression (Section 3, Eqs. ACEconstruct2, Wtilde, ACE).

    1. M_kl = <psi_k, W_l>                       (projected exchange matrix)
    2. M <- (M + M^H)/2                          (exact only in exact arithmetic)
    3. -M = L L^H, L lower with positive real diagonal
    4. xi = W L^{-H}, i.e. xi_k = sum_i W_i (L^{-H})_ik
    Returns (M, L, xi) with xi shaped like W."""
    nb = psi.shape[0]
    P = psi.reshape(nb, -1)
    Wm = W.reshape(nb, -1)
    M = grid.dV * (P.conj() @ Wm.T)
    M = 0.5 * (M + M.conj().T)
    L = np.linalg.cholesky(-M)
    # xi (as N_g x nb columns) satisfies xi L^H = W  <=>  conj(L) xi^T = W^T
    xi_rows = scipy.linalg.solve_triangular(L.conj(), Wm, lower=True)
    return M, L, xi_rows.reshape(W.shape)


def ace_apply(xi: np.ndarray, X: np.ndarray, grid: Grid) -> np.ndarray:
    """V_ACE X = -xi (xi^H X), inner products carrying dV (Eq. ACE)."""
    nb = xi.shape[0]
    Xi = xi.reshape(nb, -1)
    Xm = X.reshape(X.shape[0], -1)
    C = grid.dV * (Xi.conj() @ Xm.T)            # nb x nx
    return -(C.T @ Xi).reshape(X.shape)


def ace_dense(xi: np.ndarray, grid: Grid) -> np.ndarray:
    """Dense matrix of V_ACE acting on grid vectors (tiny grids only)."""
    Xi = xi.reshape(xi.shape[0], -1).T           # N_g x nb
    return -grid.dV * (Xi @ Xi.conj().T)


def exchange_energy_direct(phi: np.ndarray, grid: Grid) -> float:
    """E_X of Eq. (EX) with no compression:
    -1/2 sum_ij <rho_ji, v * rho_ji>,  rho_ji = conj(phi_j) phi_i, evaluated by
    Parseval as -1/2 (dV/N_g) sum_ij sum_G K(G) |fftn(rho_ji)(G)|^2."""
    K = kernel_g(grid)
    e = 0.0
    for j in range(phi.shape[0]):
        rhat = np.fft.fftn(np.conj(phi[j])[None] * phi, axes=(1, 2, 3))
        e += float(np.sum(K[None] * np.abs(rhat) ** 2))
    return -0.5 * grid.dV / grid.ng * e


def exchange_energy_trace(M: np.ndarray, nocc: int) -> float:
    """E_X = 1/2 sum_{i<N_occ} <phi_i, V_X phi_i> = 1/2 Re tr M[:N_occ, :N_occ]."""
    return 0.5 * float(np.real(np.trace(M[:nocc, :nocc])))


def exchange_energy_ace(phi: np.ndarray, xi: np.ndarray, grid: Grid) -> float:
    """E_X from the projection vectors with no Poisson solve (Eq. EX_ACE):
    -1/2 sum_{i,k} |<xi_k, phi_i>|^2."""
    A = grid.dV * (xi.reshape(xi.shape[0], -1).conj() @ phi.reshape(phi.shape[0], -1).T)
    return -0.5 * float(np.sum(np.abs(A) ** 2))


def exchange_energy_grad(phi: np.ndarray, grid: Grid) -> np.ndarray:
    """Wirtinger derivative dE_X/dphi* of E_X(phi) = 1/2 sum_i <phi_i, V_X[phi] phi_i>.

    E_X is quartic in phi; each of its two conj(phi) factors contributes one
    half, so dE_X/dphi_i* = dV * (V_X[phi] phi_i) = dV * W_i with psi = phi.
    (Not in the paper; derived from Eq. EX.)"""
    return grid.dV * build_W(phi, phi, grid)


def orthonormalize(X: np.ndarray, grid: Grid) -> np.ndarray:
    """Orthonormal basis Q of span(X) with <Q_a, Q_b> = delta_ab and X = Q R,
    R upper triangular with positive real diagonal (the constraint of Eq. HF;
    the paper does not fix a method, this factorisation is unique)."""
    nb = X.shape[0]
    A = np.sqrt(grid.dV) * X.reshape(nb, -1).T
    q, r = np.linalg.qr(A)
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    return (q.T / np.sqrt(grid.dV)).reshape(X.shape)


def planewave_exchange_eigs(mvecs_occ, mvecs_all, grid: Grid) -> np.ndarray:
    """Closed form for plane-wave orbitals phi_i = exp(i k_i.r)/sqrt(Omega):
    V_X psi_j = lambda_j psi_j with lambda_j = -(1/Omega) sum_i K(k_j - k_i),
    the difference folded back onto the grid's frequency range.  Computed from
    the kernel formula directly (no FFT, no grid fields)."""
    lam = np.zeros(len(mvecs_all))
    for j, mj in enumerate(mvecs_all):
        s = 0.0
        for mi in mvecs_occ:
            g2 = 0.0
            for a in range(3):
                d = (mj[a] - mi[a]) % grid.n[a]
                if d > grid.n[a] // 2:      # fold onto the FFT frequency range
                    d -= grid.n[a]
                g2 += (2.0 * np.pi * d / grid.L[a]) ** 2
            if g2 == 0.0:
                k = grid.g0
            else:
                k = 4.0 * np.pi / g2
                if grid.kind == "erfc":
                    k *= -np.expm1(-g2 / (4.0 * grid.mu ** 2))
            s += k
        lam[j] = -s / grid.omega
    return lam

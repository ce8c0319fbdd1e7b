"""Plain FP64 oracle of the self-consistent loops that use the exchange
operator (test infrastructure only; it shares no code with the GPU path).

The loops of Section 2 (Alg. 1: the exchange operator applied directly as
V_X[phi] by Poisson solves) and Section 3 (Alg. 2: the operator replaced by
its adaptive compression V_ACE, rebuilt once per outer iteration), for the
Hamiltonian of the linear eigenvalue problem Eq. HFlineig,
    H = -1/2 Laplacian + V_loc + alpha V_X[phi],
with a fixed local potential V_loc standing for V_ion + V_H (the paper's inner
loop also updates the density; with a fixed local potential that loop is the
linear eigensolve alone) and alpha the exchange fraction (1 for Fock exchange,
1/4 for HSE/PBE0).

Inner eigensolver (the paper names Davidson or LOBPCG; any iterative scheme
for Eq. HFlineig serves): Chebyshev-filtered subspace iteration on N_band +
n_extra vectors: a degree-m Chebyshev filter that damps [a, b] and amplifies
below a, with a the largest Ritz value, a0 the smallest and b an upper bound of
the spectrum; then orthonormalisation and a Rayleigh-Ritz step.  The n_extra
buffer vectors only let the top of the wanted N_band converge (the filter
cannot separate the vector at a from those just above it); the exchange
operator uses the lowest N_band (Psi) and N_occ (phi) Ritz vectors only.

The outer loop updates phi <- the lowest N_occ Ritz vectors and monitors the
exchange energy of Eq. EX (times alpha) of those orbitals.
"""
from __future__ import annotations

import numpy as np

from . import ace_oracle as A


def _g2(grid):
    gx, gy, gz = (2.0 * np.pi * (np.fft.fftfreq(grid.n[a]) * grid.n[a]) / grid.L[a]
                  for a in range(3))
    return gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2


def kinetic(X: np.ndarray, grid) -> np.ndarray:
    """-1/2 Laplacian on the periodic grid (spectral): ifftn(|G|^2/2 fftn(x))."""
    return np.fft.ifftn(0.5 * _g2(grid) * np.fft.fftn(X, axes=(-3, -2, -1)), axes=(-3, -2, -1))


def spectrum_upper_bound(grid, vloc) -> float:
    """max |G|^2/2 on the grid plus max V_loc: an upper bound of H's spectrum
    (the exchange operator is negative semidefinite)."""
    return float(0.5 * np.max(_g2(grid)) + np.max(vloc))


def apply_h(X, grid, vloc, exchange=None):
    """H X for a block X (N, n0, n1, n2).  exchange: None, ("vx", phi, alpha)
    for alpha V_X[phi] (Eq. applyVX2), or ("ace", xi) for V_ACE (Eq. ACE)."""
    Y = kinetic(X, grid) + vloc[None] * X
    if exchange is not None:
        if exchange[0] == "vx":
            _, phi, alpha = exchange
            Y = Y + A.build_W(phi, X, grid, scale=alpha)
        elif exchange[0] == "ace":
            Y = Y + A.ace_apply(exchange[1], X, grid)
        else:
            raise ValueError(exchange[0])
    return Y


def chebyshev_filter(X, apply, m: int, a: float, b: float, a0: float):
    """Scaled degree-m Chebyshev filter p_m(H) X (Zhou and Saad): with
    e = (b - a)/2, c = (b + a)/2, p_m(t) = T_m((t - c)/e) / T_m((a0 - c)/e),
    so p_m(a0) = 1 and |p_m| <= 1/|T_m((a0 - c)/e)| on [a, b].  The three-term
    recurrence of T_m is carried with the scaling ratios sigma_k."""
    e = 0.5 * (b - a)
    c = 0.5 * (b + a)
    sigma = e / (a0 - c)
    tau = 2.0 / sigma
    Y = (apply(X) - c * X) * (sigma / e)
    Xp = X
    for _ in range(2, m + 1):
        sigma_new = 1.0 / (tau - sigma)
        Yn = (apply(Y) - c * Y) * (2.0 * sigma_new / e) - (sigma * sigma_new) * Xp
        Xp, Y, sigma = Y, Yn, sigma_new
    return Y


def rayleigh_ritz(X, HX, grid):
    """Ritz pairs of H on span(X), X orthonormal: S = dV X^H (HX), S = Q diag(e) Q^H
    (LAPACK, ascending), returns X Q, (HX) Q, e."""
    nb = X.shape[0]
    Xm = X.reshape(nb, -1)
    Hm = HX.reshape(nb, -1)
    S = grid.dV * (Xm.conj() @ Hm.T)
    e, Q = np.linalg.eigh(0.5 * (S + S.conj().T))
    return (Q.T @ Xm).reshape(X.shape), (Q.T @ Hm).reshape(X.shape), e


def scf(grid, vloc, X0, n_occ: int, alpha: float, mode: str, degree: int, n_inner: int,
        n_outer: int, n_band: int | None = None):
    """Outer loop of Alg. 1 (mode "vx"), Alg. 2 (mode "ace") or no exchange
    (mode "none"), each outer iteration: fix the exchange operator from the
    current occupied orbitals (Alg. 2 also builds W = alpha V_X[phi] Psi and the
    compression from the N_band lowest vectors Psi, Eqs. W, ACEconstruct2,
    Wtilde), a Rayleigh-Ritz step, then n_inner filtered subspace iterations on
    all of X0's vectors (N_band plus buffers; n_band None: all are Psi).
    Returns a dict with the exchange energy alpha E_X[phi] (Eq. EX) of the
    occupied Ritz vectors after every outer iteration, the Ritz values after
    every outer iteration and the last vectors."""
    b_up = spectrum_upper_bound(grid, vloc)
    X = A.orthonormalize(np.asarray(X0, dtype=np.complex128), grid)
    nb = X.shape[0] if n_band is None else n_band
    e_hist, ritz_hist = [], []
    e = None
    for _ in range(n_outer):
        phi = X[:n_occ].copy()
        if mode == "ace":
            psi = X[:nb]
            W = A.build_W(phi, psi, grid, scale=alpha)
            _, _, xi = A.compress(psi, W, grid)
            ex = ("ace", xi)
        elif mode == "vx":
            ex = ("vx", phi, alpha)
        elif mode == "none":
            ex = None
        else:
            raise ValueError(mode)

        def apply(Z):
            return apply_h(Z, grid, vloc, ex)

        X, HX, e = rayleigh_ritz(X, apply(X), grid)
        for _ in range(n_inner):
            Y = chebyshev_filter(X, apply, degree, float(e[-1]), b_up, float(e[0]))
            X = A.orthonormalize(Y, grid)
            X, HX, e = rayleigh_ritz(X, apply(X), grid)
        e_hist.append(alpha * A.exchange_energy_direct(X[:n_occ], grid))
        ritz_hist.append(e.copy())
    return {"E_X": e_hist, "ritz": ritz_hist, "X": X}

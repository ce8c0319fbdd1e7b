"""The self-consistent loops of the paper on the GPU: Alg. 1 (the exchange
operator applied directly, V_X[phi] by pair Poisson solves in every
Hamiltonian application) and Alg. 2 (V_ACE built once per outer iteration and
reused by every application), for H = -1/2 Laplacian + V_loc + alpha V_X
(Section 2, Eq. HFlineig, with a fixed local potential standing for
V_ion + V_H, so the inner loop is the linear eigensolve alone).

Sequencing only: every vector operation is a libace call (ace_apply_h,
ace_combine, ace_orthonormalize, ace_rayleigh_ritz, ace_build_W, ace_compress,
ace_exchange_energy); the host reads the Ritz values (the filter bounds) and
the exchange energies.

Inner eigensolver: Chebyshev-filtered subspace iteration on N_band + n_extra
vectors (degree-m filter damping [a, b] with a the largest Ritz value, a0 the
smallest, b the upper bound max |G|^2/2 + max V_loc of the spectrum; then
orthonormalisation and a Rayleigh-Ritz step).  The buffer vectors let the top
of the wanted block converge; V_ACE is built from the lowest N_band Ritz
vectors (Psi, the oversampling ratio r = N_band / N_occ of Section 3) and V_X
from the lowest N_occ (phi).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import ace


def spectrum_upper_bound(grid: ace.Grid, vloc_max: float) -> float:
    """max over the grid of |G|^2 / 2 (the Nyquist corner, |m_a| = n / 2 per
    axis) plus max V_loc; the exchange operator is negative semidefinite."""
    return 0.5 * sum((math.pi * grid.n / L) ** 2 for L in grid.L) + float(vloc_max)


class ScfLoop:
    """One outer/inner loop configuration on one context."""

    def __init__(self, ctx: ace.Context, grid: ace.Grid, prec: str, vloc: np.ndarray,
                 n_occ: int, n_band: int, alpha: float, mode: str, degree: int = 8):
        if mode not in ("ace", "vx", "none"):
            raise ValueError(mode)
        self.ctx, self.grid, self.prec = ctx, grid, prec
        self.n_occ, self.n_band, self.alpha, self.mode, self.degree = (
            n_occ, n_band, float(alpha), mode, int(degree))
        vt = torch.float64 if prec == "fp64" else torch.float32
        self.vloc = torch.from_numpy(np.ascontiguousarray(vloc, dtype=np.float64)).to(
            ctx.device, vt).reshape(-1)
        self.b_up = spectrum_upper_bound(grid, float(np.max(vloc)))
        self.times = {"inner": [], "ace_build": [], "apply_h": []}

    # -- pieces --------------------------------------------------------------
    def _h(self, Z, out, ex):
        kind, ops = ex
        if kind == "ace":
            return self.ctx.apply_h(Z, self.grid, self.prec, vloc=self.vloc, xi=ops, out=out)
        if kind == "vx":
            return self.ctx.apply_h(Z, self.grid, self.prec, vloc=self.vloc, phi=ops,
                                    scale_x=self.alpha, out=out)
        return self.ctx.apply_h(Z, self.grid, self.prec, vloc=self.vloc, out=out)

    def _filter(self, X, HX, ex, a, a0, work):
        """Scaled degree-m Chebyshev filter p_m(H) X (Zhou and Saad), damping
        [a, b] and normalised to 1 at a0; HX = H X is given (the Rayleigh-Ritz
        step's (HX) Q).  Returns the work buffer holding the result."""
        g, p, c_ = self.grid, self.prec, self.ctx
        b = self.b_up
        e = 0.5 * (b - a)
        c = 0.5 * (b + a)
        sigma = e / (a0 - c)
        tau = 2.0 / sigma
        HY, B0, B1 = work
        Y = c_.combine(g, p, sigma / e, HX, -c * sigma / e, X, out=B0)
        Xp, free = X, B1
        for _ in range(2, self.degree + 1):
            s_new = 1.0 / (tau - sigma)
            self._h(Y, HY, ex)
            # the new iterate overwrites Xp's buffer once Xp is not the caller's X
            dst = free if Xp is X else Xp
            Yn = c_.combine(g, p, 2.0 * s_new / e, HY, -2.0 * s_new * c / e, Y,
                            -sigma * s_new, Xp, out=dst)
            Xp, Y, sigma = Y, Yn, s_new
        return Y

    def run(self, X0: torch.Tensor, n_inner: int, n_outer: int, timing: bool = False):
        """Outer iterations of Alg. 1 / Alg. 2 from the orbitals X0 (N_band +
        buffers, rows of N_g values).  Returns the exchange energy alpha E_X
        (Eq. EX) of the occupied Ritz vectors after every outer iteration, the
        Ritz values after every outer iteration, and the final vectors."""
        c_, g, p = self.ctx, self.grid, self.prec
        nb_all = X0.shape[0]
        Xa = c_.orthonormalize(X0, g, p)
        Xb, Ha, Hb = torch.empty_like(Xa), torch.empty_like(Xa), torch.empty_like(Xa)
        work = (torch.empty_like(Xa), torch.empty_like(Xa), torch.empty_like(Xa))
        phi = torch.empty_like(Xa[:self.n_occ])
        ev = torch.empty(nb_all, dtype=torch.float64, device=Xa.device)
        e_hist, ritz_hist, marks = [], [], []

        def tick():
            if not timing:
                return None
            t = torch.cuda.Event(enable_timing=True)
            t.record()
            return t

        def rr(Xin, Hin):
            Xout = Xa if Xin is Xb else Xb
            Hout = Ha if Hin is Hb else Hb
            return c_.rayleigh_ritz(Xin, Hin, g, p, out_X=Xout, out_HX=Hout, evals=ev)

        X = Xa
        for _ in range(n_outer):
            phi.copy_(X[:self.n_occ])
            t0 = tick()
            if self.mode == "ace":
                psi = X[:self.n_band]
                W = c_.build_W(phi, psi, g, p, scale=self.alpha)
                xi = c_.compress(psi, W, g, p)
                ex = ("ace", xi)
            elif self.mode == "vx":
                ex = ("vx", phi)
            else:
                ex = ("none", None)
            if timing:
                marks.append(("ace_build", t0, tick()))
            Hin = Ha if X is Xa else Hb
            self._h(X, Hin, ex)
            X, HX, _ = rr(X, Hin)
            for _ in range(n_inner):
                t0 = tick()
                e_host = ev.cpu().numpy()
                Y = self._filter(X, HX, ex, float(e_host[-1]), float(e_host[0]), work)
                Xo = c_.orthonormalize(Y, g, p, out=Xa if X is Xb else Xb)
                Ho = Ha if Xo is Xa else Hb
                self._h(Xo, Ho, ex)
                X, HX, _ = rr(Xo, Ho)
                if timing:
                    marks.append(("inner", t0, tick()))
            e = c_.exchange_energy(X[:self.n_occ], g, p)
            e_hist.append(self.alpha * float(e.item()))
            ritz_hist.append(ev.cpu().numpy().copy())
        if timing:
            torch.cuda.synchronize()
            for kind, a, b in marks:
                self.times[kind].append(a.elapsed_time(b))
        return {"E_X": e_hist, "ritz": ritz_hist, "X": X}

"""GPU parity of the eigensolver pieces and of the self-consistent loops
(Alg. 1 with V_X applied by pair solves, Alg. 2 with V_ACE; Section 2 Eq.
HFlineig with a fixed local potential) against the FP64 oracle: the
Hamiltonian application element by element, the Rayleigh-Ritz step, and the
whole loops (exchange energy after every outer iteration, final Ritz values)."""
import numpy as np
import pytest

import oracle as O
from oracle import scf_oracle as S
from paper_1601_07159_amd import synth
from tests._helpers import ggrid, ogrid, rel, to_gpu, to_np, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ace():
    from paper_1601_07159_amd import ace as A
    return A


def _vloc_gpu(v, prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(v)).to("cuda", dt).reshape(-1)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["none", "vx", "ace"])
@pytest.mark.parametrize("n,L", [(12, 7.0), (24, 10.0)])
def test_apply_h_matches_oracle(ace, prec, mode, n, L):
    print(f"apply_h prec={prec} mode={mode} n={n}", flush=True)
    g, gg = ogrid(n, L, "erfc", 0.3), ggrid(n, L, "erfc", 0.3)
    vloc = synth.local_potential(n, L, 7, depth=1.2)
    psi = synth.smooth_orbitals(n, L, 9, seed=31)
    phi = psi[:4]
    X = synth.smooth_orbitals(n, L, 5, seed=32)
    alpha = 0.25
    ctx = ace.Context()
    if mode == "none":
        ex, kw = None, {}
    elif mode == "vx":
        ex, kw = ("vx", phi, alpha), dict(phi=to_gpu(phi, prec), scale_x=alpha)
    else:
        W = O.build_W(phi, psi, g, scale=alpha)
        _, _, xi = O.compress(psi, W, g)
        ex, kw = ("ace", xi), dict(xi=to_gpu(xi, prec))
    ref = S.apply_h(X, g, vloc, ex)
    Y = ctx.apply_h(to_gpu(X, prec), gg, prec, vloc=_vloc_gpu(vloc, prec), **kw)
    assert rel(to_np(Y), ref) <= tol(prec)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nb", [6, 40, 90, 130])
def test_rayleigh_ritz_matches_oracle(ace, prec, nb):
    """The Jacobi eigensolver in LDS (n <= 88) and in global memory (above):
    eigenvalues against LAPACK's, the rotated vectors span the same Ritz
    vectors (up to a phase per vector), and H X_out = (HX)_out."""
    import torch
    n, L = 16, 9.0
    print(f"rayleigh_ritz prec={prec} nb={nb}", flush=True)
    g, gg = ogrid(n, L), ggrid(n, L)
    vloc = synth.local_potential(n, L, 9, depth=1.0)
    X = O.orthonormalize(synth.smooth_orbitals(n, L, nb, seed=nb), g)
    HX = S.apply_h(X, g, vloc)
    Xr, Hr, e = S.rayleigh_ritz(X, HX, g)
    ctx = ace.Context()
    Xg, Hg, eg = ctx.rayleigh_ritz(to_gpu(X, prec), to_gpu(HX, prec), gg, prec)
    torch.cuda.synchronize()
    eg = eg.cpu().numpy()
    assert np.max(np.abs(eg - e)) <= (1e-11 if prec == "fp64" else 1e-5) * np.max(np.abs(e))
    Xg, Hg = to_np(Xg), to_np(Hg)
    # phases: <xr_k, xg_k> has modulus 1 for simple Ritz values
    ov = g.dV * np.sum(Xr.reshape(nb, -1).conj() * Xg.reshape(nb, -1), axis=1)
    gap = np.minimum(np.abs(np.diff(e, prepend=-1e9)), np.abs(np.diff(e, append=1e9)))
    simple = gap > 1e-3
    assert np.max(np.abs(np.abs(ov[simple]) - 1.0)) <= (1e-9 if prec == "fp64" else 1e-4)
    assert rel(Hg, S.apply_h(Xg, g, vloc)) <= tol(prec) * 10
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["vx", "ace"])
def test_scf_loop_matches_oracle(ace, prec, mode):
    """The whole outer/inner loop from the same start: exchange energy after
    every outer iteration and the final Ritz values of the N_band states."""
    from paper_1601_07159_amd.scf import ScfLoop
    n, L, nocc, nband, nall, alpha = 12, 7.0, 4, 6, 8, 0.25
    print(f"scf loop prec={prec} mode={mode}", flush=True)
    g, gg = ogrid(n, L, "erfc", 0.3), ggrid(n, L, "erfc", 0.3)
    vloc = synth.local_potential(n, L, 5, depth=1.5)
    X0 = synth.smooth_orbitals(n, L, nall, seed=2)
    ref = S.scf(g, vloc, X0, nocc, alpha, mode, 8, 4, 6, n_band=nband)
    ctx = ace.Context()
    loop = ScfLoop(ctx, gg, prec, vloc, nocc, nband, alpha, mode, degree=8)
    out = loop.run(to_gpu(X0, prec).reshape(nall, -1), n_inner=4, n_outer=6)
    t = 1e-9 if prec == "fp64" else 1e-5
    assert rel(out["E_X"], ref["E_X"]) <= t
    assert np.max(np.abs(out["ritz"][-1][:nband] - ref["ritz"][-1][:nband])) <= t * 10
    ctx.close()


def test_scf_constant_potential_levels(ace):
    """No exchange, constant potential: the GPU loop finds the plane-wave
    levels 1/2 |k|^2 + V_0."""
    from paper_1601_07159_amd.scf import ScfLoop
    n, L, v0 = 12, 7.0, -0.4
    gg = ggrid(n, L)
    X0 = synth.smooth_orbitals(n, L, 10, seed=1)
    ctx = ace.Context()
    loop = ScfLoop(ctx, gg, "fp64", np.full((n, n, n), v0), 7, 7, 0.0, "none", degree=8)
    out = loop.run(to_gpu(X0, "fp64").reshape(10, -1), n_inner=12, n_outer=1)
    k2 = (2.0 * np.pi / L) ** 2
    exact = np.array([v0] + [v0 + 0.5 * k2] * 6)
    assert np.max(np.abs(out["ritz"][-1][:7] - exact)) <= 1e-8
    ctx.close()

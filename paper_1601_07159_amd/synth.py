"""Seeded synthetic inputs for the ACE build.

This module only manufactures inputs (orbitals, and a local potential for the
eigensolver loops); it performs none of the exchange arithmetic (no pair
densities, no Coulomb kernel, no compression).  Both the
FP64 oracle tests and the GPU path draw their inputs from here, so that the
two sides consume byte-identical arrays.

Orbitals stand in for the occupied / oversampled orbitals of the paper's
silicon and water systems (Section 4): smooth fields made of random plane-wave
coefficients inside a kinetic-energy sphere |G|^2/2 <= Ecut with Gaussian
amplitudes exp(-|G|^2/8), orthonormalised in coefficient space and brought to
the real-space grid.  Normalisation is the physical one, dV * sum |phi|^2 = 1
with dV = Omega / N_g.

Layout of every returned array: complex, shape (N, n0, n1, n2), C order, i.e.
orbital-major with each orbital's N_g grid values contiguous.
"""
from __future__ import annotations

import numpy as np


def _axis_g(n: int, L: float) -> np.ndarray:
    """Reciprocal-lattice components 2*pi*m/L for the FFT ordering of m."""
    m = np.fft.fftfreq(n) * n
    return 2.0 * np.pi * m / L


def _g2_grid(n3, L3) -> np.ndarray:
    gx, gy, gz = (_axis_g(int(n3[a]), float(L3[a])) for a in range(3))
    return gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2


def _as3(v, cast):
    if np.ndim(v) == 0:
        return (cast(v),) * 3
    return tuple(cast(x) for x in v)


def smooth_orbitals(n, L, nband: int, seed: int, ecut: float = 10.0,
                    orthonormal: bool = True, draw: str = "grid") -> np.ndarray:
    """Random smooth orbitals on an n0 x n1 x n2 periodic grid of an
    orthorhombic cell with edges L (bohr), complex128, shape (nband, n0, n1, n2).

    Recipe: coefficients c_b(G) = (a + i b)/sqrt(2) * exp(-|G|^2/8) on the
    sphere |G|^2/2 <= ecut (a, b standard normal from default_rng(seed));
    when ``orthonormal`` the coefficient vectors are orthonormalised by a QR
    factorisation with positive diagonal; each orbital is then
    psi_b(r) = (1/sqrt(Omega)) sum_G c_b(G) exp(i G.r).
    draw="grid" takes normals for every grid point (those outside the sphere
    are then zeroed); draw="sphere" takes them for the sphere's points only,
    in C order (a cheaper stream for large batches; different orbitals).
    """
    n3 = _as3(n, int)
    L3 = _as3(L, float)
    ng = n3[0] * n3[1] * n3[2]
    omega = L3[0] * L3[1] * L3[2]
    g2 = _g2_grid(n3, L3)
    mask = (0.5 * g2 <= ecut)
    amp = np.exp(-g2 / 8.0) * mask
    rng = np.random.default_rng(seed)
    if draw == "grid":
        re = rng.standard_normal((nband,) + n3)
        im = rng.standard_normal((nband,) + n3)
        c = (re + 1j * im) / np.sqrt(2.0) * amp
    elif draw == "sphere":
        sel = mask.reshape(-1)
        k = int(sel.sum())
        re = rng.standard_normal((nband, k))
        im = rng.standard_normal((nband, k))
        c = np.zeros((nband, sel.size), dtype=np.complex128)
        c[:, sel] = (re + 1j * im) / np.sqrt(2.0) * amp.reshape(-1)[sel]
        c = c.reshape((nband,) + n3)
    else:
        raise ValueError(draw)
    if orthonormal:
        sel = mask.reshape(-1)
        if nband > int(sel.sum()):
            raise ValueError("more orbitals than plane waves inside the cutoff sphere")
        # coefficients outside the sphere are zero: factor only the rows inside
        q, r = np.linalg.qr(c.reshape(nband, -1)[:, sel].T)
        d = np.diag(r)
        q = q * (d / np.abs(d))[None, :]
        full = np.zeros((nband, sel.size), dtype=np.complex128)
        full[:, sel] = q.T
        c = full.reshape((nband,) + n3)
    else:
        # Keep roughly unit norm so that non-orthonormal inputs stay well scaled.
        c = c / np.sqrt(np.sum(np.abs(c) ** 2, axis=(1, 2, 3), keepdims=True))
    import scipy.fft
    psi = scipy.fft.ifftn(c, axes=(1, 2, 3), workers=-1) * (ng / np.sqrt(omega))
    return np.ascontiguousarray(psi)


def real_orbitals(n, L, nband: int, seed: int, ecut: float = 10.0) -> np.ndarray:
    """Real smooth orbitals (the Gamma-point case), float64, shape (nband, n0,
    n1, n2): the real parts of ``smooth_orbitals(n, L, nband, seed, ecut,
    orthonormal=False)``, orthonormalised on the grid (QR with positive
    diagonal of the N_g x nband matrix, then scaled so dV sum psi^2 = 1)."""
    n3 = _as3(n, int)
    L3 = _as3(L, float)
    ng = n3[0] * n3[1] * n3[2]
    dv = L3[0] * L3[1] * L3[2] / ng
    x = np.real(smooth_orbitals(n, L, nband, seed, ecut, orthonormal=False))
    q, r = np.linalg.qr(x.reshape(nband, ng).T)
    q = q * np.sign(np.diag(r))[None, :]
    return np.ascontiguousarray((q.T / np.sqrt(dv)).reshape((nband,) + n3))


def planewave_orbitals(n, L, mvecs) -> np.ndarray:
    """Plane waves exp(i k.r)/sqrt(Omega), k = 2*pi*m/L, one per integer
    triple in ``mvecs``; complex128, shape (len(mvecs), n0, n1, n2)."""
    n3 = _as3(n, int)
    L3 = _as3(L, float)
    omega = L3[0] * L3[1] * L3[2]
    x = [np.arange(n3[a]) / n3[a] for a in range(3)]  # fractional coordinates
    out = np.empty((len(mvecs),) + n3, dtype=np.complex128)
    for b, m in enumerate(mvecs):
        ph = (2.0 * np.pi * m[0] * x[0][:, None, None]
              + 2.0 * np.pi * m[1] * x[1][None, :, None]
              + 2.0 * np.pi * m[2] * x[2][None, None, :])
        out[b] = np.exp(1j * ph) / np.sqrt(omega)
    return out


def random_unitary(k: int, seed: int) -> np.ndarray:
    """Haar-like random k x k unitary (QR of a complex Gaussian, phases fixed)."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def random_directions(shape, count: int, seed: int, norm: float) -> np.ndarray:
    """``count`` complex Gaussian directions of the given orbital-block shape,
    orthonormalised in the flattened space and scaled to Frobenius norm ``norm``."""
    rng = np.random.default_rng(seed)
    size = int(np.prod(shape))
    z = (rng.standard_normal((size, count)) + 1j * rng.standard_normal((size, count)))
    q, _ = np.linalg.qr(z)
    return (q.T * norm).reshape((count,) + tuple(shape))


def batched_instances(count: int = 48, seed: int = 1000, orbital_seed: int = 2000,
                      grids=(32, 40, 48, 64), nocc_range=(16, 128), extra: int = 16,
                      spacing: float = 0.43):
    """Draw the sizes of a batch of independent instances: grid n uniform over
    ``grids``, N_occ uniform over the inclusive ``nocc_range``, N_band = N_occ +
    ``extra``, cubic cell L = spacing * n.  Returns a list of dicts (orbitals are
    produced lazily by :func:`instance_orbitals`)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.choice(grids))
        nocc = int(rng.integers(nocc_range[0], nocc_range[1] + 1))
        out.append(dict(n=n, L=spacing * n, nocc=nocc, nband=nocc + extra,
                        seed=orbital_seed + b))
    return out


def instance_orbitals(inst) -> np.ndarray:
    return smooth_orbitals(inst["n"], inst["L"], inst["nband"], inst["seed"], draw="sphere")


def local_potential(n, L, seed: int, depth: float = 1.0, gmax2: float = 3.0) -> np.ndarray:
    """A smooth random real local potential (stands for V_ion + V_H in the
    linear eigenvalue problem), float64, shape (n0, n1, n2): Fourier
    coefficients (a + i b) exp(-|G|^2/2) on |G|^2 <= gmax2 (a, b ~ N(0, 1) from
    default_rng(seed)), made Hermitian (c(-G) = conj c(G)) so the field is real,
    G = 0 removed, then scaled so that min V = -depth."""
    n3 = _as3(n, int)
    L3 = _as3(L, float)
    g2 = _g2_grid(n3, L3)
    rng = np.random.default_rng(seed)
    c = (rng.standard_normal(n3) + 1j * rng.standard_normal(n3)) * np.exp(-g2 / 2.0)
    c = c * ((g2 <= gmax2) & (g2 > 0))
    # Hermitian part: the coefficient at -G (index -k mod n per axis) conjugated
    cm = np.conj(c[(-np.arange(n3[0])) % n3[0]][:, (-np.arange(n3[1])) % n3[1]]
                 [:, :, (-np.arange(n3[2])) % n3[2]])
    v = np.real(np.fft.ifftn(0.5 * (c + cm)))
    return np.ascontiguousarray(depth * v / (-np.min(v)))

"""Shared helpers for the GPU parity tests (inputs, tolerances, conversions)."""
import numpy as np

# Tolerances on relative Frobenius error against the FP64 oracle.
TOL_FP64 = 1e-10
TOL_FP32 = 1e-5


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def to_gpu(x, prec):
    import torch
    dt = {"fp64": torch.complex128, "real64": torch.float64,
          "real32": torch.float32}.get(prec, torch.complex64)
    if prec.startswith("real"):
        x = np.real(x)
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dt)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def ogrid(n, L, kind="coulomb", mu=0.0, g0=0.0):
    import oracle as O
    return O.Grid.cubic(n, L, kind, mu, g0)


def ggrid(n, L, kind="coulomb", mu=0.0, g0=0.0):
    from paper_1601_07159_amd.ace import Grid
    return Grid.cubic(n, L, kind, mu, g0)


def tol(prec):
    return TOL_FP64 if prec in ("fp64", "real64") else TOL_FP32

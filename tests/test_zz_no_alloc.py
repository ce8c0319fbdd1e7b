"""ace_apply_noalloc (the allocation-free variant of ace_apply, scratch in a
static device array of the library) through the C ABI: its output equals
ace_apply's on the same inputs, on two calls in a row (the second smaller, so
stale scratch from the first would show), it records into a graph on a context
that never allocated a workspace, and sizes beyond its scratch are refused."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1601_07159_amd import synth
from tests._helpers import ggrid, ogrid, rel, to_gpu, to_np, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ace():
    from paper_1601_07159_amd import ace as A
    return A


def _noalloc(ctx, grid, prec, xi, X, Y):
    from paper_1601_07159_amd import _lib
    from paper_1601_07159_amd.ace import _prec
    lib = _lib.load()
    g = grid.as_c()
    ctx._bind_stream()
    return lib.ace_apply_noalloc(ctx._h, ctypes.byref(g), _prec(prec),
                                 ctypes.c_void_p(xi.data_ptr()), xi.shape[0], xi.stride(0),
                                 ctypes.c_void_p(X.data_ptr()), X.shape[0], X.stride(0),
                                 ctypes.c_void_p(Y.data_ptr()), Y.stride(0))


def _case(n, L, nb, nx, prec, seed):
    xi = synth.smooth_orbitals(n, L, nb, seed=seed) * 0.3
    X = synth.smooth_orbitals(n, L, nx, seed=seed + 1)
    return xi, X, to_gpu(xi, prec).reshape(nb, -1), to_gpu(X, prec).reshape(nx, -1)


def test_noalloc_apply_matches_apply_twice(ace):
    """Two calls in a row, the second with fewer orbitals on a smaller grid;
    each equals ace_apply bit for bit and the oracle to the precision's
    tolerance."""
    import torch
    ctx = ace.Context(0)
    for (n, L, nb, nx, prec, seed) in [(24, 10.0, 40, 33, "fp32", 5), (16, 7.0, 9, 5, "fp64", 9)]:
        print(f"noalloc apply n={n} nb={nb} nx={nx} prec={prec}", flush=True)
        xi, X, xg, Xg = _case(n, L, nb, nx, prec, seed)
        g = ggrid(n, L)
        Y = torch.full_like(Xg, float("nan"))
        assert _noalloc(ctx, g, prec, xg, Xg, Y) == 0
        Yref = ctx.apply(xg, Xg, g, prec)
        torch.cuda.synchronize()
        assert torch.equal(Y, Yref)
        ref = O.ace_apply(xi, X, ogrid(n, L)).reshape(nx, -1)
        assert rel(to_np(Y), ref) <= tol(prec)
    ctx.close()


def test_noalloc_apply_under_capture_without_workspace(ace):
    """A fresh context has no workspace: ace_apply under capture is refused
    (ACE_E_CAPTURE), the allocation-free apply records and replays, and every
    replay equals the eager result on the new data."""
    import torch
    n, L, nb, nx, prec = 16, 7.0, 12, 7, "fp32"
    xi, X, xg, Xg = _case(n, L, nb, nx, prec, 21)
    g = ggrid(n, L)
    ctx = ace.Context(0)
    Y = torch.zeros_like(Xg)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    refused = None
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            try:
                ctx.apply(xg, Xg, g, prec, out=Y)
            except ace.AceError as e:
                refused = e.status
            st = _noalloc(ctx, g, prec, xg, Xg, Y)
    torch.cuda.current_stream().wait_stream(side)
    assert refused == 6 and st == 0
    ref_ctx = ace.Context(0)
    for rep in range(3):
        new = to_gpu(synth.smooth_orbitals(n, L, nx, seed=40 + rep), prec).reshape(nx, -1)
        Xg.copy_(new)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        Yref = ref_ctx.apply(xg, new, g, prec)
        torch.cuda.synchronize()
        assert torch.equal(Y, Yref), rep
    ctx.close()
    ref_ctx.close()


def test_noalloc_apply_refuses_sizes_beyond_its_scratch(ace):
    import torch
    n, nb = 8, 1800          # the 1800 x 1800 complex128 matrix alone exceeds 48 MiB
    xg = torch.zeros((nb, n ** 3), dtype=torch.complex128, device="cuda")
    Xg = torch.zeros_like(xg)
    Y = torch.zeros_like(xg)
    ctx = ace.Context(0)
    assert _noalloc(ctx, ggrid(n, 4.0), "fp64", xg, Xg, Y) == 5   # ACE_E_UNSUPPORTED
    msg = ctx._lib.ace_last_error(ctx._h).decode()
    assert "allocation-free" in msg and "scratch" in msg
    torch.cuda.synchronize()
    assert torch.all(Y == 0)
    ctx.close()

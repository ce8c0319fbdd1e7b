"""Behaviour of the C ABI around its calls: graph capture without a reserved
workspace (ACE_E_CAPTURE, capture left intact), ordering of calls made on
different streams through one context, xi computed in place of W, the tuning
cache named at ace_create, and the failing-pivot report of the n > 88
factorisations (Section 3, the Cholesky after Eq. ACEconstruct2)."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1601_07159_amd import synth
from tests._helpers import ggrid, ogrid, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ace():
    from paper_1601_07159_amd import ace as A
    return A


def test_capture_without_reserve_is_refused_cleanly(ace):
    """A call that would grow the workspace inside a capture returns
    ACE_E_CAPTURE before it enqueues anything; the capture ends normally, the
    empty graph replays, and the context still works afterwards."""
    import torch
    n, L, nocc, nband = 16, 6.5, 4, 6
    g = ggrid(n, L)
    psi = to_gpu(synth.smooth_orbitals(n, L, nband, seed=41), "fp32").reshape(nband, -1)
    W = torch.empty_like(psi)
    ctx = ace.Context(0)                      # fresh: no workspace yet
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    status = None
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            try:
                ctx.build_W(psi[:nocc], psi, g, "fp32", out=W)
            except ace.AceError as e:
                status = e.status
    torch.cuda.current_stream().wait_stream(side)
    assert status == 6                        # ACE_E_CAPTURE
    graph.replay()
    torch.cuda.synchronize()
    # the same call outside the capture works and matches a second context
    W1 = ctx.build_W(psi[:nocc], psi, g, "fp32")
    W2 = ace.Context(0).build_W(psi[:nocc], psi, g, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(W1, W2)
    ctx.close()


def test_capture_with_synchronising_info_is_refused(ace):
    """compress / orthonormalise with info_dev == NULL synchronise, so under
    capture they are refused with ACE_E_CAPTURE even after ace_reserve."""
    import torch
    n, L, nb = 16, 6.5, 6
    g = ggrid(n, L)
    psi = to_gpu(synth.smooth_orbitals(n, L, nb, seed=42), "fp64").reshape(nb, -1)
    ctx = ace.Context(0)
    ctx.reserve(g, "fp64", nb, nb, nb)
    W = ctx.build_W(psi, psi, g, "fp64")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    got = []
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for call in (lambda: ctx.compress(psi, W, g, "fp64"),
                         lambda: ctx.orthonormalize(psi, g, "fp64")):
                try:
                    call()
                except ace.AceError as e:
                    got.append(e.status)
    torch.cuda.current_stream().wait_stream(side)
    assert got == [6, 6]
    graph.replay()
    torch.cuda.synchronize()
    ctx.close()


def test_calls_on_two_streams_are_ordered(ace):
    """One context used from two streams with no host synchronisation between
    the calls: the second stream waits for the first one's work on the shared
    workspace, so the results equal those of a single-stream run bit for bit."""
    import torch
    n, L, nocc, nband = 24, 10.0, 8, 12
    g = ggrid(n, L)
    pa = to_gpu(synth.smooth_orbitals(n, L, nband, seed=51), "fp32").reshape(nband, -1)
    pb = to_gpu(synth.smooth_orbitals(n, L, nband, seed=52), "fp32").reshape(nband, -1)
    ref = ace.Context(0)
    Wa_ref = ref.build_W(pa[:nocc], pa, g, "fp32")
    xa_ref = ref.compress(pa, Wa_ref, g, "mixed")
    Wb_ref = ref.build_W(pb[:nocc], pb, g, "fp32")
    xb_ref = ref.compress(pb, Wb_ref, g, "mixed")
    torch.cuda.synchronize()
    ctx = ace.Context(0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    for rep in range(3):
        with torch.cuda.stream(s1):
            Wa = ctx.build_W(pa[:nocc], pa, g, "fp32")
            xa = ctx.compress(pa, Wa, g, "mixed", info=info[0:1])
        with torch.cuda.stream(s2):
            Wb = ctx.build_W(pb[:nocc], pb, g, "fp32")
            xb = ctx.compress(pb, Wb, g, "mixed", info=info[1:2])
        torch.cuda.synchronize()
        assert torch.equal(Wa, Wa_ref) and torch.equal(xa, xa_ref), rep
        assert torch.equal(Wb, Wb_ref) and torch.equal(xb, xb_ref), rep
    assert info.tolist() == [0, 0]
    ctx.close()
    ref.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_xi_may_overwrite_W(ace, prec):
    """ace_compress with xi == W (same pointer and ld) gives the same xi as
    with a separate output."""
    import torch
    n, L, nocc, nband = 16, 7.0, 5, 90        # 90 bands: the n > 88 factorisation
    g = ggrid(n, L)
    psi = to_gpu(synth.smooth_orbitals(n, L, nband, seed=61), prec).reshape(nband, -1)
    ctx = ace.Context(0)
    W = ctx.build_W(psi[:nocc], psi, g, prec)
    xi_sep = ctx.compress(psi, W, g, prec)
    W2 = W.clone()
    out = ctx.compress(psi, W2, g, prec, out=W2)
    torch.cuda.synchronize()
    assert out.data_ptr() == W2.data_ptr()
    assert torch.equal(W2, xi_sep)
    ctx.close()


def test_tune_cache_named_at_create(ace, tmp_path):
    """ace_create loads the settings of its tune_cache (a missing file is not
    an error) and ace_autotune without a path appends to that cache."""
    import torch
    n, L, nocc, nband = 16, 6.5, 5, 8
    g = ggrid(n, L)
    psi = to_gpu(synth.smooth_orbitals(n, L, nband, seed=71), "fp32").reshape(nband, -1)
    missing = str(tmp_path / "none.txt")
    ace.Context(0, tune_cache=missing).close()
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{n} 8 0 0 8\n")        # octet line shape for n = 16, complex64
    c_cache = ace.Context(0, tune_cache=str(cache))
    c_knob = ace.Context(0)
    c_knob.set_tuning("fft_shape", 8)
    c_def = ace.Context(0)
    Wc = c_cache.build_W(psi[:nocc], psi, g, "fp32")
    Wk = c_knob.build_W(psi[:nocc], psi, g, "fp32")
    Wd = c_def.build_W(psi[:nocc], psi, g, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(Wc, Wk)
    assert not torch.equal(Wc, Wd)            # the octet lines round differently
    before = cache.read_text().count("\n")
    c_cache.autotune(g, "fp32", nocc, nband)
    assert cache.read_text().count("\n") == before + 1
    for c in (c_cache, c_knob, c_def):
        c.close()


@pytest.mark.parametrize("nband,zero", [(100, 95), (520, 515)])
def test_not_positive_definite_pivot_large(ace, nband, zero):
    """A zero orbital makes the pivot of its row of -M exactly 0: the blocked
    factorisations (LDS panels for n <= 512, global memory beyond) report that
    1-based pivot in info and ACE_E_NOT_PD without info."""
    import torch
    n, L, nocc = 16, 10.0, 8
    print(f"not-PD pivot nband={nband} zero={zero}", flush=True)
    psi = synth.smooth_orbitals(n, L, nband, seed=81)
    psi[zero] = 0.0
    W = O.build_W(psi[:nocc], psi, ogrid(n, L))
    gg = ggrid(n, L)
    p, w = to_gpu(psi, "fp64"), to_gpu(W, "fp64")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ace.compress(p, w, gg, "fp64", info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == zero + 1
    with pytest.raises(ace.AceError) as e:
        ace.compress(p, w, gg, "fp64")
    assert e.value.status == 2
    # the same matrix without the zero orbital factors (pins that the earlier
    # pivots are positive, so the reported one is the first)
    keep = [k for k in range(nband) if k != zero]
    info.zero_()
    ace.compress(to_gpu(psi[keep], "fp64"), to_gpu(W[keep], "fp64"), gg, "fp64", info=info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0

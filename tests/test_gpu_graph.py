"""The single-instance entry points under HIP graph capture (the calls are
stream-ordered and, after ace_reserve, allocate nothing): a captured build ->
compress -> apply -> energy sequence is replayed several times on new data,
with eager work and synchronisations in between, and every replay is checked
against the eager calls on the same data."""
import pytest

from paper_1601_07159_amd import synth
from tests._helpers import ggrid, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ace():
    from paper_1601_07159_amd import ace as A
    return A


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_captured_path_replays_follow_new_data(ace, prec):
    import torch
    n, L, nocc, nband = 16, 6.5, 6, 9
    g = ggrid(n, L)
    dev = torch.device("cuda", 0)
    psi0 = to_gpu(synth.smooth_orbitals(n, L, nband, seed=900), prec).reshape(nband, -1)
    ctx = ace.Context(0)
    ctx.reserve(g, prec, nocc, nband, nband)
    # static buffers of the graph
    psi = psi0.clone()
    W = torch.empty_like(psi)
    xi = torch.empty_like(psi)
    Y = torch.empty_like(psi)
    e = torch.zeros((), dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)

    def path():
        ctx.build_W(psi[:nocc], psi, g, prec, out=W)
        ctx.compress(psi, W, g, prec, info=info, out=xi)
        ctx.apply(xi, psi, g, prec, out=Y)
        ctx.exchange_energy(psi[:nocc], g, prec, xi=xi, out=e)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        path()                              # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        path()
    torch.cuda.synchronize()

    ctx_ref = ace.Context(0)
    for rep in range(3):
        new = to_gpu(synth.smooth_orbitals(n, L, nband, seed=910 + rep), prec).reshape(nband, -1)
        psi.copy_(new)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        # eager reference on the same data, separate context and buffers
        Wr = ctx_ref.build_W(new[:nocc], new, g, prec)
        xir = ctx_ref.compress(new, Wr, g, prec)
        Yr = ctx_ref.apply(xir, new, g, prec)
        er = ctx_ref.exchange_energy(new[:nocc], g, prec, xi=xir)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        assert torch.equal(W, Wr), f"replay {rep}: W"
        assert torch.equal(xi, xir), f"replay {rep}: xi"
        assert torch.equal(Y, Yr), f"replay {rep}: V_ACE psi"
        assert float(e) == float(er), f"replay {rep}: E_X"
    ctx.close()
    ctx_ref.close()

"""GPU checks of the build autotuner (ace_autotune, ace_tune_load), which picks
the pair-batch width, the band block and the line shape of the FFT passes: the
choice is one of the candidates, it is written to and read back from the cache
file, and builds that use it match the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1601_07159_amd import synth
from tests._helpers import ggrid, ogrid, rel, to_gpu, to_np, tol

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_autotune_choice_persists_and_builds_match_oracle(tmp_path, prec):
    from paper_1601_07159_amd import ace
    n, L, nocc, nband = 24, 10.0, 6, 9
    print(f"autotune prec={prec} n={n}", flush=True)
    psi = synth.smooth_orbitals(n, L, nband, seed=41)
    g, gg = ogrid(n, L), ggrid(n, L)
    ref = O.build_W(psi[:nocc], psi, g)
    cache = str(tmp_path / "tune.txt")
    ctx = ace.Context()
    r = ctx.autotune(gg, prec, nocc, nband, cache_path=cache)
    assert r["fft_shape"] in (0, 1, 4, 8, 16)
    assert r["accum_shape"] in (0, 1, 16)
    assert r["pair_budget"] > 0 and r["jblock"] >= 0 and r["ms"] > 0
    fields = open(cache).read().split()
    assert len(fields) == 6 and int(fields[0]) == n and int(fields[4]) == r["fft_shape"]
    assert int(fields[5]) == r["accum_shape"]
    x = to_gpu(psi, prec)
    W = to_np(ctx.build_W(x[:nocc], x, gg, prec))
    ctx.close()
    assert rel(W.reshape(ref.shape), ref) <= tol(prec)
    ctx2 = ace.Context()
    ctx2.tune_load(cache)
    W2 = to_np(ctx2.build_W(x[:nocc], x, gg, prec))
    ctx2.close()
    assert rel(W2.reshape(ref.shape), ref) <= tol(prec)
    assert np.array_equal(W, W2)  # the same settings, the same bits


def test_tune_load_reads_lines_without_shape(tmp_path):
    from paper_1601_07159_amd import ace
    n, L, nocc, nband = 16, 6.0, 3, 5
    psi = synth.smooth_orbitals(n, L, nband, seed=43)
    ref = O.build_W(psi[:nocc], psi, ogrid(n, L))
    cache = tmp_path / "old.txt"
    cache.write_text(f"{n} 8 268435456 0\n")  # four fields: shape 0 (the defaults)
    ctx = ace.Context()
    ctx.tune_load(str(cache))
    x = to_gpu(psi, "fp32")
    W = to_np(ctx.build_W(x[:nocc], x, ggrid(n, L), "fp32"))
    ctx.close()
    assert rel(W.reshape(ref.shape), ref) <= tol("fp32")


def test_environment_tune_on_first_build(tmp_path, monkeypatch):
    """ACE_TUNE=1: the first build of a grid size runs the tuner once and
    appends its choice to the ACE_TUNE_CACHE file; ACE_LOG records it; the
    builds match the oracle."""
    from paper_1601_07159_amd import ace
    n, L, nocc, nband = 16, 7.0, 4, 7
    print(f"env tune n={n}", flush=True)
    cache, log = tmp_path / "tune.txt", tmp_path / "ace.log"
    monkeypatch.setenv("ACE_TUNE", "1")
    monkeypatch.setenv("ACE_TUNE_CACHE", str(cache))
    monkeypatch.setenv("ACE_LOG", str(log))
    psi = synth.smooth_orbitals(n, L, nband, seed=45)
    ref = O.build_W(psi[:nocc], psi, ogrid(n, L))
    x = to_gpu(psi, "fp32")
    ctx = ace.Context()
    W1 = to_np(ctx.build_W(x[:nocc], x, ggrid(n, L), "fp32"))
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[:2] == [str(n), "8"]
    W2 = to_np(ctx.build_W(x[:nocc], x, ggrid(n, L), "fp32"))
    assert len(cache.read_text().splitlines()) == 1      # tuned once
    with pytest.raises(ace.AceError):
        ctx.build_W(x[:nocc], x, ggrid(n, L), "fp32", scale=float("nan"))
    ctx.close()
    text = log.read_text()
    assert f"tuned n={n} elem_bytes=8" in text
    assert "scale must be finite" in text
    assert np.array_equal(W1, W2)
    assert rel(W1.reshape(ref.shape), ref) <= tol("fp32")


def test_environment_tune_off_uses_defaults(tmp_path, monkeypatch):
    """ACE_TUNE=0: a loaded setting (here the octet line shape, which rounds
    differently from the default shape) is not used."""
    import torch
    from paper_1601_07159_amd import ace
    n, L, nocc, nband = 16, 6.5, 5, 8
    psi = to_gpu(synth.smooth_orbitals(n, L, nband, seed=71), "fp32").reshape(nband, -1)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{n} 8 0 0 8\n")
    g = ggrid(n, L)
    c_def = ace.Context()
    c_on = ace.Context(0, tune_cache=str(cache))
    monkeypatch.setenv("ACE_TUNE", "0")
    c_off = ace.Context(0, tune_cache=str(cache))
    Wd, Won, Woff = (c.build_W(psi[:nocc], psi, g, "fp32") for c in (c_def, c_on, c_off))
    torch.cuda.synchronize()
    assert torch.equal(Woff, Wd)
    assert not torch.equal(Won, Wd)
    for c in (c_def, c_on, c_off):
        c.close()

"""GPU parity of ace_build_W_batched (many independent ACE builds in one HIP
graph) against the FP64 oracle and against the single-instance entry points."""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle as O
from paper_1601_07159_amd import synth
from tests._helpers import ggrid, ogrid, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ace():
    from paper_1601_07159_amd import ace as A
    return A


SMALL = [  # n, L, nocc, extra, kind, mu
    (16, 6.0, 5, 3, "coulomb", 0.0),
    (24, 10.0, 9, 4, "erfc", 0.2),
    (32, 13.0, 4, 2, "coulomb", 0.0),
    (16, 7.0, 7, 0, "erfc", 0.5),
    (24, 9.0, 3, 5, "coulomb", 0.0),
    (32, 14.0, 6, 1, "erfc", 0.106),
]


def _make(ace, prec, specs, seed0):
    import torch
    insts, host = [], []
    for k, (n, L, nocc, extra, kind, mu) in enumerate(specs):
        psi = synth.smooth_orbitals(n, L, nocc + extra, seed=seed0 + k)
        x = to_gpu(psi, prec)
        d = dict(grid=ggrid(n, L, kind, mu), phi=x[:nocc], psi=x, W=torch.empty_like(x),
                 xi=torch.empty_like(x), info=torch.full((1,), -1, dtype=torch.int32,
                                                         device="cuda"))
        insts.append(d)
        host.append((psi, ogrid(n, L, kind, mu), nocc))
    return insts, host


def test_batched_fp64_matches_oracle_and_single_calls(ace):
    import torch
    insts, host = _make(ace, "fp64", SMALL, 40)
    ctx = ace.Context()
    ctx.build_batched(insts, "fp64", n_branches=3)
    torch.cuda.synchronize()
    for d, (psi, og, nocc) in zip(insts, host):
        W = O.build_W(psi[:nocc], psi, og)
        _, _, xi = O.compress(psi, W, og)
        assert int(d["info"].item()) == 0
        assert rel(to_np(d["W"]), W) <= 1e-10
        assert rel(to_np(d["xi"]), xi) <= 1e-10
        # single-instance path: same kernels and blocking, so bitwise equal
        W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], "fp64")
        xi1 = ctx.compress(d["psi"], W1, d["grid"], "fp64")
        assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
    ctx.close()


def test_batched_mixed_precisions_in_one_batch(ace):
    # each instance names its own precision; FP64 and FP32 instances share one
    # graph and each equals its single call in that precision, bit for bit
    import torch
    insts, host = [], []
    for k, prec in enumerate(["fp64", "fp32", "fp64", "fp32"]):
        i, h = _make(ace, prec, [SMALL[k]], 90 + k)
        i[0]["prec"] = prec
        insts += i
        host += h
    ctx = ace.Context()
    ctx.build_batched(insts, "fp32", n_branches=2)
    torch.cuda.synchronize()
    for d, (psi, og, nocc) in zip(insts, host):
        assert int(d["info"].item()) == 0
        assert d["W"].dtype == (torch.complex128 if d["prec"] == "fp64" else torch.complex64)
        W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], d["prec"])
        xi1 = ctx.compress(d["psi"], W1, d["grid"], d["prec"])
        torch.cuda.synchronize()
        assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
        ref = O.build_W(psi[:nocc], psi, og)
        assert rel(to_np(d["W"]), ref) <= (1e-10 if d["prec"] == "fp64" else 1e-5)
    ctx.close()


def test_batched_branch_knob(ace):
    # the branch count is a tuning knob (1..16, 0 = default); the result does
    # not depend on it
    import torch
    insts, _ = _make(ace, "fp32", SMALL[:5], 120)
    ctx = ace.Context()
    outs = []
    for nbr in (1, 5, 16):
        ctx.set_tuning("branches", nbr)
        assert ctx.get_tuning("branches") == nbr
        ctx.build_batched(insts, "fp32")
        torch.cuda.synchronize()
        outs.append([d["W"].clone() for d in insts])
    for a, b in zip(outs[0], outs[2]):
        assert torch.equal(a, b)
    with pytest.raises(ace.AceError):
        ctx.set_tuning("branches", 17)
    ctx.close()


def test_batched_graph_replay_follows_new_data(ace):
    # the second and later calls replay the captured graph; the data behind the
    # same pointers changes in between and every replay must follow it
    import torch
    insts, host = _make(ace, "fp32", SMALL[:4], 60)
    ctx = ace.Context()
    ctx.build_batched(insts, "fp32", n_branches=2)
    torch.cuda.synchronize()
    for rep in range(3):
        for k, d in enumerate(insts):
            n, L, nocc, extra = SMALL[k][:4]
            new = synth.smooth_orbitals(n, L, nocc + extra, seed=500 + 10 * rep + k)
            d["psi"].copy_(to_gpu(new, "fp32"))
        torch.cuda.synchronize()
        ctx.build_batched(insts, "fp32", n_branches=2)      # replay
        torch.cuda.synchronize()
        for d in insts:
            W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], "fp32")
            xi1 = ctx.compress(d["psi"], W1, d["grid"], "fp32")
            torch.cuda.synchronize()
            assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
    ctx.close()


def test_config4_48_instances(ace):
    """48 instances, n uniform in {32, 40, 48, 64}, N_occ uniform in [16, 128],
    N_band = N_occ + 16, L = 0.43 n, FP32: every instance equals its single
    call bitwise; sampled W columns of two instances against the oracle."""
    import torch
    specs = synth.batched_instances()
    with cf.ThreadPoolExecutor(8) as ex:
        orbs = list(ex.map(synth.instance_orbitals, specs))
    insts = []
    for s, psi in zip(specs, orbs):
        x = to_gpu(psi, "fp32")
        insts.append(dict(grid=ggrid(s["n"], s["L"]), phi=x[:s["nocc"]], psi=x,
                          W=torch.empty_like(x), xi=torch.empty_like(x),
                          info=torch.full((1,), -1, dtype=torch.int32, device="cuda")))
    ctx = ace.Context()
    ctx.build_batched(insts, "fp32", n_branches=4)
    torch.cuda.synchronize()
    for d in insts:
        assert int(d["info"].item()) == 0
        W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], "fp32")
        xi1 = ctx.compress(d["psi"], W1, d["grid"], "fp32")
        torch.cuda.synchronize()
        assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
    for k in (int(np.argmin([s["n"] for s in specs])), int(np.argmax([s["n"] for s in specs]))):
        s, psi = specs[k], orbs[k]
        cols = [0, s["nband"] - 1]
        ref = O.build_W(psi[:s["nocc"]], psi, ogrid(s["n"], s["L"]), columns=cols)
        Wn = to_np(insts[k]["W"])
        for c, j in enumerate(cols):
            assert rel(Wn[j], ref[c]) <= 1e-5
    ctx.close()


def test_batched_recaptures_after_tuning(ace, tmp_path):
    # a new autotuned setting (here a line shape and a pair budget read from a
    # cache file) changes the build's launches; the cached graph must be
    # captured again, so the batch still equals the single calls under the new
    # setting, bit for bit
    import torch
    insts, host = _make(ace, "fp32", SMALL[:3], 80)
    ctx = ace.Context()
    ctx.build_batched(insts, "fp32", n_branches=2)          # capture
    torch.cuda.synchronize()
    before = [d["W"].clone() for d in insts]
    cache = tmp_path / "tune.txt"
    cache.write_text("".join(f"{n} 8 {1 << 20} 0 4\n" for n in (16, 24, 32)))
    ctx.tune_load(str(cache))                                # quad lines, 1 MiB budget
    ctx.build_batched(insts, "fp32", n_branches=2)          # must not replay the old graph
    torch.cuda.synchronize()
    changed = 0
    for d, (psi, og, nocc), old in zip(insts, host, before):
        W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], "fp32")
        assert torch.equal(W1, d["W"])
        changed += int(not torch.equal(old, d["W"]))
        ref = O.build_W(psi[:nocc], psi, og)
        assert rel(to_np(d["W"]), ref) <= 1e-5
        assert rel(to_np(old), ref) <= 1e-5
    assert changed > 0  # the new setting rounds differently, so a stale graph would show
    ctx.close()


# ---------------------------------------------------------------------------
# Persistent form (ACE_TUNE_BATCH_FORM = 2): one persistent kernel per grid
# size runs every instance's passes from a task queue.  Its slab and plane
# passes are the one-thread-per-line forms, so single calls with line shape 1
# have the same arithmetic and must agree bit for bit.

def _persistent_ctx(ace, budget=0):
    ctx = ace.Context()
    ctx.set_tuning("batch_form", 2)
    ctx.set_tuning("fft_shape", 1)
    if budget:
        ctx.set_tuning("pair_budget", budget)
    return ctx


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_persistent_equals_single_calls(ace, prec):
    import torch
    print(f"persistent batch prec={prec}", flush=True)
    insts, host = _make(ace, prec, SMALL, 200)
    ctx = _persistent_ctx(ace)
    ctx.build_batched(insts, prec)
    torch.cuda.synchronize()
    t = 1e-10 if prec == "fp64" else 1e-5
    for d, (psi, og, nocc) in zip(insts, host):
        assert int(d["info"].item()) == 0
        W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], prec)
        xi1 = ctx.compress(d["psi"], W1, d["grid"], prec)
        torch.cuda.synchronize()
        assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
        assert rel(to_np(d["W"]), O.build_W(psi[:nocc], psi, og)) <= t
    ctx.close()


def test_persistent_chunked_builds_and_mixed_sizes(ace):
    # a small pair budget splits every build into chunks (triangle blocks,
    # rectangles, several accumulations into the same bands), so the tasks of
    # one instance form a long dependency chain; instances of one size share
    # one persistent kernel, FP64 and FP32 instances of a size run in two
    import torch
    specs = SMALL + [(24, 8.0, 12, 6, "coulomb", 0.0), (16, 6.5, 10, 2, "erfc", 0.3)]
    insts, host = [], []
    for k, sp in enumerate(specs):
        prec = "fp64" if k % 3 == 0 else "fp32"
        i, h = _make(ace, prec, [sp], 300 + k)
        i[0]["prec"] = prec
        insts += i
        host += h
    budget = 6 * 32 ** 3 * 16  # a few pairs per chunk at every size
    ctx = _persistent_ctx(ace, budget)
    ctx.build_batched(insts, "fp32")
    torch.cuda.synchronize()
    for d, (psi, og, nocc) in zip(insts, host):
        assert int(d["info"].item()) == 0
        W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], d["prec"])
        xi1 = ctx.compress(d["psi"], W1, d["grid"], d["prec"])
        torch.cuda.synchronize()
        assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
        ref = O.build_W(psi[:nocc], psi, og)
        assert rel(to_np(d["W"]), ref) <= (1e-10 if d["prec"] == "fp64" else 1e-5)
    ctx.close()


def test_persistent_replay_follows_new_data(ace):
    import torch
    insts, _ = _make(ace, "fp32", SMALL[:4], 400)
    ctx = _persistent_ctx(ace, 4 * 24 ** 3 * 8)
    ctx.build_batched(insts, "fp32")
    torch.cuda.synchronize()
    for rep in range(3):
        for k, d in enumerate(insts):
            n, L, nocc, extra = SMALL[k][:4]
            new = synth.smooth_orbitals(n, L, nocc + extra, seed=450 + 10 * rep + k)
            d["psi"].copy_(to_gpu(new, "fp32"))
        torch.cuda.synchronize()
        ctx.build_batched(insts, "fp32")  # replay
        torch.cuda.synchronize()
        for d in insts:
            W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], "fp32")
            xi1 = ctx.compress(d["psi"], W1, d["grid"], "fp32")
            torch.cuda.synchronize()
            assert torch.equal(W1, d["W"]) and torch.equal(xi1, d["xi"])
    ctx.close()


def test_persistent_accumulate_forms(ace):
    # both accumulate forms (one thread per pencil with LDS accumulators, split
    # lines with register accumulators) inside the persistent kernel
    import torch
    for accum in (1, 16):
        insts, _ = _make(ace, "fp32", SMALL[:3], 500 + accum)
        ctx = _persistent_ctx(ace)
        ctx.set_tuning("accum_shape", accum)
        ctx.build_batched(insts, "fp32")
        torch.cuda.synchronize()
        for d in insts:
            W1 = ctx.build_W(d["phi"], d["psi"], d["grid"], "fp32")
            torch.cuda.synchronize()
            assert torch.equal(W1, d["W"])
        ctx.close()

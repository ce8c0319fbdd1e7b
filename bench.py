"""Benchmark of the ACE build on one MI355X.

One step = the whole hot path on one batch of orbitals:
  orthonormalise psi (FP64 CholQR2) -> W = V_X[phi] psi (n_occ x n_band pair
  Poisson solves) -> compress (M = <psi, W>, Cholesky, xi = W L^{-H}) ->
  V_ACE psi (low-rank apply; 20 times at the 72^3 workload, whose definition
  repeats the application per build) -> E_X from xi.
Default workload: 48^3 grid, cubic L = 20.5 bohr, N_occ = 64, N_band = 80,
mixed precision (FP32 FFTs and apply, BF16-split M, FP64 Cholesky/TRSM).

Prints ONE JSON line; metric value = pair Poisson solves per second of whole
steps (N_occ * N_band pairs per step).  Inputs are synthetic smooth orthonormal
orbitals (seeded), resident in HBM before timing starts.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "cfg1": dict(n=24, L=10.0, nocc=8, nband=8, nx=8, kind="coulomb", mu=0.0, prec="fp64",
                 desc="24^3 grid, L=10 bohr, N_occ=N_band=8, complex128, Coulomb"),
    "cfg2": dict(n=48, L=20.5, nocc=64, nband=80, nx=80, kind="coulomb", mu=0.0, prec="mixed",
                 desc="48^3 grid, L=20.5 bohr, N_occ=64, N_band=80, complex64 FFTs, "
                      "BF16-split M, FP64 Cholesky/TRSM, Coulomb"),
    "cfg3": dict(n=72, L=30.8, nocc=216, nband=256, nx=256, kind="erfc", mu=0.106, prec="fp32",
                 applies=20, x_seeds=list(range(100, 120)),
                 golden="tests/golden/smooth72_erfc_seed0.json",
                 desc="72^3 grid, L=30.8 bohr, N_occ=216, N_band=256, FP32 FFTs, FP64 "
                      "compression, erfc mu=0.106, 20 applications of V_ACE per build on "
                      "X_t = generator(seed 100 + t)"),
    "cfg2r": dict(n=48, L=20.5, nocc=64, nband=80, nx=80, kind="coulomb", mu=0.0, prec="real32",
                  desc="48^3 grid, L=20.5 bohr, N_occ=64, N_band=80, real orbitals (Gamma "
                       "point): two pair charges per complex64 FFT, BF16-split M, FP64 "
                       "Cholesky/TRSM, Coulomb"),
    "cfg4": dict(n=48, L=20.64, nocc=0, nband=0, nx=0, kind="coulomb", mu=0.0, prec="fp32",
                 desc="48 independent instances (n in {32,40,48,64}, N_occ in [16,128], "
                      "N_band = N_occ + 16, L = 0.43 n), one HIP-graph launch per step: "
                      "build W and compress, FP32 FFTs"),
    "cfg5": dict(n=64, L=27.0, nocc=128, nband=128, nx=0, kind="coulomb", mu=0.0, prec="fp32",
                 desc="autograd E_X(phi) forward + hand-written backward, 64^3 grid, "
                      "L=27 bohr, N_occ=128, complex64"),
    "scf": dict(n=48, L=20.5, nocc=64, nband=80, nx=0, kind="erfc", mu=0.106, prec="fp32",
                alpha=0.25, extra=8, degree=8, inner=10, outer=12, depth=2.0,
                desc="Alg. 1 / Alg. 2 loops: H = -1/2 Laplacian + V_loc + 0.25 V_X (erfc, "
                     "mu=0.106), 48^3 grid, L=20.5 bohr, N_occ=64, Chebyshev-filtered "
                     "subspace iteration (degree 8, 8 buffer vectors), 10 inner "
                     "iterations per outer iteration, complex64"),
}

HBM_PEAK_GBS = 8000.0
FFT_SOURCES = ["paper_1601_07159_amd/csrc/fft_passes.hip", "paper_1601_07159_amd/csrc/fft_core.h",
               "paper_1601_07159_amd/csrc/pass_bodies.h"]


def fft_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in FFT_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, pairs_per_launch):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/hbm_traffic_<workload>.json, written from two rocprofv3 --pmc runs),
    or None when it is missing or the FFT sources changed since it was taken."""
    import json as _json
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = _json.load(f)
    if d.get("source_hash") != fft_source_hash() or kernel not in d.get("kernels", {}):
        return None
    k = d["kernels"][kernel]
    return k["bytes_per_pair"] * pairs_per_launch


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_inputs(cfg):
    import oracle as O
    from paper_1601_07159_amd import synth
    if cfg.get("prec", "").startswith("real"):
        psi = synth.real_orbitals(cfg["n"], cfg["L"], cfg["nband"], seed=0)
    else:
        psi = synth.smooth_orbitals(cfg["n"], cfg["L"], cfg["nband"], seed=0)
    return psi, O.Grid.cubic(cfg["n"], cfg["L"], cfg["kind"], cfg["mu"])


def _oracle_columns(args):
    """Worker of the all-core oracle timing (a fresh interpreter: spawned, so
    nothing of the parent's GPU runtime is inherited): regenerates the seeded
    inputs, waits at the barrier until every worker is ready, then computes its
    columns of W with the oracle and returns its own wall time."""
    cfg, cols, barrier = args
    import oracle as O
    psi, g = _oracle_inputs(cfg)
    phi = psi[:cfg["nocc"]]
    O.build_W(phi, psi, g, columns=[cols[0]])          # warm (plans, pages)
    barrier.wait()
    t0 = time.perf_counter()
    O.build_W(phi, psi, g, columns=cols)
    return time.perf_counter() - t0


def host_cores():
    """Cores this process may run on, capped at the 16 a one-GPU machine grants."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(cfg, seconds=10.0, all_cores=True):
    """Time the FP64 oracle's pair solves on a bounded sample of the workload,
    in the two modes of the paper's setting and a parallel host:
      single core  whole columns j of W (each column = N_occ pair solves), as
                   many as fit in about `seconds` of one thread's work;
      all cores    the oracle's columns spread over one process per host core
                   (multiprocessing over j), each process taking as many
                   columns as fit in about `seconds`; rate = all pairs / the
                   slowest process's time.
    Returns the all-core figure as the baseline (cores = processes used) with
    the single-core one beside it."""
    import multiprocessing as mp

    import oracle as O
    psi, g = _oracle_inputs(cfg)
    phi = psi[:cfg["nocc"]]
    t0 = time.perf_counter()
    O.build_W(phi, psi, g, columns=[0])
    per_col = max(time.perf_counter() - t0, 1e-6)
    ncols = int(max(1, min(cfg["nband"] - 1, seconds / per_col)))
    t0 = time.perf_counter()
    O.build_W(phi, psi, g, columns=list(range(1, 1 + ncols)))
    dt = time.perf_counter() - t0
    pairs = ncols * cfg["nocc"]
    single = {"value": pairs / dt, "unit": "pair solves/s", "cores": 1, "kind": "oracle",
              "sample": f"oracle build_W columns j=1..{ncols} ({pairs} pair solves, FP64 "
                        f"NumPy pocketfft, one thread), {dt:.1f} s"}
    cores = host_cores()
    if not all_cores or cores < 2:
        return dict(single, host_cores=cores)
    del psi, phi
    per_proc = int(max(1, seconds / per_col))
    ctx = mp.get_context("spawn")
    with ctx.Manager() as mgr:
        barrier = mgr.Barrier(cores)
        jobs = [(cfg, [(k * per_proc + q) % cfg["nband"] for q in range(per_proc)], barrier)
                for k in range(cores)]
        with ctx.Pool(cores) as pool:
            times = pool.map(_oracle_columns, jobs, chunksize=1)
    pairs_all = cores * per_proc * cfg["nocc"]
    t_all = max(times)
    return {"value": pairs_all / t_all, "unit": "pair solves/s", "cores": cores,
            "kind": "oracle",
            "sample": f"oracle build_W, {cores} processes x {per_proc} columns of W "
                      f"({pairs_all} pair solves, FP64 NumPy pocketfft, one thread each), "
                      f"slowest process {t_all:.1f} s",
            "host_cores": cores, "single_core": single}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "mixed", "real64", "real32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--pair-budget", type=int, default=0,
                    help="bytes of pair spectra in flight (0 = library default)")
    ap.add_argument("--fft-shape", type=int, default=0, choices=[0, 1, 4, 8, 16],
                    help="line shape of the slab and plane passes (0 = library default)")
    ap.add_argument("--accum-shape", type=int, default=0, choices=[0, 1, 16],
                    help="form of the accumulate pass (0 = library default)")
    ap.add_argument("--batch-form", type=int, default=0, choices=[0, 1, 2],
                    help="cfg4: W stage of the batched build (1 launches, 2 persistent)")
    ap.add_argument("--branches", type=int, default=4,
                    help="cfg4: concurrent branch streams of the launches form (1..16)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="cfg4: skip the autotuner (library defaults)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain copy of known size (for counter scaling)")
    ap.add_argument("--no-others", action="store_true",
                    help="the default cfg2 run with its CPU baseline also times cfg1, cfg2r, "
                         "cfg3, cfg4 and cfg5 for a few steps each (child processes, after the timed "
                         "region) and reports them under extra.other_workloads; this skips them")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the ACE path runs on one GPU; --gpus above 1 is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1601_07159_amd import ace, synth

    cfg = dict(WORKLOADS[args.workload])
    if args.prec:
        cfg["prec"] = args.prec
    if args.workload == "cfg4":
        return run_batched(args, cfg)
    if args.workload == "cfg5":
        return run_autograd(args, cfg)
    if args.workload == "scf":
        return run_scf(args, cfg)
    prec = cfg["prec"]
    n, L, nocc, nband, nx = cfg["n"], cfg["L"], cfg["nocc"], cfg["nband"], cfg["nx"]
    applies = cfg.get("applies", 1)
    grid = ace.Grid.cubic(n, L, cfg["kind"], cfg["mu"])
    ng = grid.ng
    real = prec.startswith("real")
    dtypes = {"fp64": torch.complex128, "real64": torch.float64, "real32": torch.float32}
    cdt = dtypes.get(prec, torch.complex64)
    ref_prec = "real64" if real else "fp64"
    # bytes of one complex FFT element (real orbitals are transformed in pairs)
    sbytes = 16 if prec in ("fp64", "real64") else 8

    log(f"bench: workload {args.workload} prec={prec}: generating inputs")
    psi_np = (synth.real_orbitals(n, L, nband, seed=0) if real
              else synth.smooth_orbitals(n, L, nband, seed=0))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    psi_in = torch.from_numpy(psi_np).to(dev, cdt)

    ctx = ace.Context(0)
    if args.pair_budget:
        ctx.set_pair_budget(args.pair_budget)
    if args.fft_shape:
        ctx.set_tuning("fft_shape", args.fft_shape)
    if args.accum_shape:
        ctx.set_tuning("accum_shape", args.accum_shape)
    ctx.reserve(grid, prec, nocc, nband, nx)

    def make_bufs(dt):
        return dict(Q=torch.empty((nband, ng), dtype=dt, device=dev),
                    W=torch.empty((nband, ng), dtype=dt, device=dev),
                    xi=torch.empty((nband, ng), dtype=dt, device=dev),
                    Y=torch.empty((nx, ng), dtype=dt, device=dev),
                    e=torch.empty((), dtype=torch.float64, device=dev),
                    info=torch.zeros(1, dtype=torch.int32, device=dev))

    bufs = make_bufs(cdt)
    # Orbitals V_ACE is applied to: the screened 72^3 workload applies it to
    # X_t = generator(seed 100 + t), t < 20 (new orbitals each call, as in an
    # eigensolver's inner iterations); the others to the first n_x orbitals
    # of psi (V_ACE psi = W on span(psi) then checks the compression).
    X_seeds = cfg.get("x_seeds")
    X_host = {}
    if X_seeds:
        import concurrent.futures as cf
        log(f"bench: generating {len(X_seeds)} apply inputs X_t")
        with cf.ThreadPoolExecutor(4) as ex:
            for sd, x in zip(X_seeds, ex.map(
                    lambda sd: synth.smooth_orbitals(n, L, nx, seed=sd), X_seeds)):
                X_host[sd] = torch.from_numpy(x).reshape(nx, ng).to(dev, torch.complex128)
        Xs = [X_host[sd].to(cdt) for sd in X_seeds]
    else:
        Xs = None

    stage_ev = []

    def step(p, b, src, timed=False):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(6)] if timed else None
        if timed:
            evs[0].record()
        ctx.orthonormalize(src.reshape(nband, ng), grid, p, info=b["info"], out=b["Q"])
        if timed:
            evs[1].record()
        ctx.build_W(b["Q"][:nocc], b["Q"], grid, p, out=b["W"])
        if timed:
            evs[2].record()
        ctx.compress(b["Q"], b["W"], grid, p, info=b["info"], out=b["xi"])
        if timed:
            evs[3].record()
        if b.get("X") is not None:
            for X in b["X"]:
                ctx.apply(b["xi"], X, grid, p, out=b["Y"])
        else:
            for _ in range(applies):
                ctx.apply(b["xi"], b["Q"][:nx], grid, p, out=b["Y"])
        if timed:
            evs[4].record()
        ctx.exchange_energy(b["Q"][:nocc], grid, p, xi=b["xi"], out=b["e"])
        if timed:
            evs[5].record()
            stage_ev.append(evs)

    bufs["X"] = Xs
    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        step(prec, bufs, psi_in)
    torch.cuda.synchronize()

    # 1) the timed steps: nothing but the step itself
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(prec, bufs, psi_in)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # 2) the same number of steps again with the library's per-kernel HIP
    #    events and per-stage events (they add a few microseconds of gaps per
    #    launch, so they stay out of the first region)
    ctx.profile(True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step(prec, bufs, psi_in, timed=True)
    torch.cuda.synchronize()
    wall_prof = time.perf_counter() - t1
    prof = ctx.profile_report()
    ctx.profile(False)
    stages = ["orthonormalize", "build_W", "compress", "apply", "energy"]
    st_ms = {s: float(np.mean([ev[k].elapsed_time(ev[k + 1]) for ev in stage_ev]))
             for k, s in enumerate(stages)}
    pairs = nocc * nband
    value = pairs * args.steps / wall
    log(f"bench: {ms_step:.3f} ms/step ({wall_prof * 1e3 / args.steps:.3f} with per-kernel "
        f"events), stages {st_ms}")

    # dominant FFT-pass kernel and its roofline
    # algorithmic HBM bytes per pair, in units of N_g * s:
    #   pair_fwd_slab: write the slab spectra (inputs amortised over the pair block)
    #   plane_kernel:  read + write
    #   pencil_accum:  read (phi and W amortised over the pair block)
    fft_units = {"pair_fwd_slab": 1, "plane_kernel": 2, "pencil_accum": 1, "pair_fwd_real": 1,
                 "pencil_accum_real": 1}
    # pairs each pass handles per step: with the i <-> j symmetry (psi starts
    # with phi) the forward and plane passes transform the occupied triangle
    # plus the rectangle of extra bands; the accumulate pass reads every pair
    sym = ctx.get_tuning("symmetry") == 1
    if real:
        # real orbitals: units of two pairs.  With the i <-> j symmetry and an
        # even n_occ (one chunk) the occupied triangle is packed by column
        # (column c holds floor(c / 2) + 1 units), then (orbital pair, extra
        # band) units; the accumulate pass serves band pairs (2g, 2g + 1) of the
        # occupied block from one read of each unit of later columns.  Without
        # it: (orbital pair, band) units for every band.
        half = (nocc + 1) // 2
        if sym and nocc % 2 == 0:
            transformed = sum(c // 2 + 1 for c in range(nocc)) + (nband - nocc) * half
            accum_reads = (nocc // 2) * nocc + (nband - nocc) * half
        else:
            transformed = accum_reads = half * nband
        per_step = {"pair_fwd_real": transformed, "plane_kernel": transformed,
                    "pencil_accum_real": accum_reads}
    else:
        transformed = (nocc * (nocc + 1) // 2 + nocc * (nband - nocc)) if sym else pairs
        per_step = {"pair_fwd_slab": transformed, "plane_kernel": transformed,
                    "pencil_accum": pairs}
    dom = max(fft_units, key=lambda k: prof.get(k, {"ms": 0})["ms"])
    d = prof[dom]
    avg_ms = d["ms"] / d["launches"]
    pairs_per_launch = per_step[dom] * args.steps / d["launches"]
    bytes_per_pair = fft_units[dom] * ng * sbytes
    achieved = bytes_per_pair * pairs_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, dom, pairs_per_launch)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "algorithmic_bytes_per_launch": round(bytes_per_pair * pairs_per_launch),
                "avg_launch_ms": round(avg_ms, 4), "pairs_per_launch": pairs_per_launch}
    build_ms = st_ms["build_W"]
    build_bytes = (3 * transformed + per_step.get("pencil_accum", per_step.get(
        "pencil_accum_real", transformed))) * ng * sbytes
    extra = {
        "profiled_ms_per_step": round(wall_prof * 1e3 / args.steps, 4),
        "stage_ms": {k: round(v, 4) for k, v in st_ms.items()},
        "build_pairs_per_s": pairs / (build_ms * 1e-3),
        "build_fft_algorithmic_GBs": build_bytes / (build_ms * 1e-3) / 1e9,
        "build_transformed_pairs": transformed,
        "build_roofline_ms": build_bytes / (HBM_PEAK_GBS * 1e9) * 1e3,
        "applies_per_step": applies,
        "apply_tflops": 16.0 * ng * nband * nx * applies / (st_ms["apply"] * 1e-3) / 1e12,
        "per_kernel": {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 5)}
                       for k, v in prof.items()},
    }

    # errors vs an FP64 run on the same seed (outside the timed region)
    if not args.no_fp64 and prec not in ("fp64", "real64"):
        log("bench: FP64 comparison run")
        dt64 = dtypes[ref_prec]
        b64 = make_bufs(dt64)
        b64["X"] = [X_host[sd] for sd in X_seeds] if X_seeds else None
        psi64 = torch.from_numpy(psi_np).to(dev, dt64)
        step(ref_prec, b64, psi64)
        torch.cuda.synchronize()
        t = []
        for _ in range(max(2, min(args.steps, 5))):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            step(ref_prec, b64, psi64)
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        extra["fp64_ms_per_step"] = float(np.median(t))
        stage_ev.clear()
        step(ref_prec, b64, psi64, timed=True)
        torch.cuda.synchronize()
        ev = stage_ev[-1]
        extra["fp64_stage_ms"] = {s: round(ev[k].elapsed_time(ev[k + 1]), 4)
                                  for k, s in enumerate(stages)}
        extra["apply_tflops_fp64"] = 16.0 * ng * nband * nx * applies / (
            extra["fp64_stage_ms"]["apply"] * 1e-3) / 1e12

        def relerr(a, b):
            a = a.to(b.dtype)
            return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
        extra["errors_vs_fp64"] = {
            "W": relerr(bufs["W"], b64["W"]),
            "xi": relerr(bufs["xi"], b64["xi"]),
            ("V_ACE_X%d" % (len(X_seeds) - 1) if X_seeds else "V_ACE_psi"):
                relerr(bufs["Y"], b64["Y"]),
            "E_X": abs(float(bufs["e"]) - float(b64["e"])) / abs(float(b64["e"])),
            "E_X_fp64": float(b64["e"]),
        }
        del b64, psi64

    if cfg.get("golden"):
        log("bench: errors against the oracle's stored full-size values")
        extra["errors_vs_oracle"] = golden_errors(ctx, cfg, grid, prec, bufs, Xs, nocc)

    if args.copy_probe:
        # a plain copy kernel of known size (256 MiB read, 256 MiB written) for
        # the HBM counter scaling; torch's copy_ may go through a DMA engine,
        # which the counters do not see, so the copy is an elementwise kernel
        src = torch.zeros(256 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        extra["copy_probe_bytes"] = 2 * src.numel() * 8

    out = {
        "metric": "pair Poisson solves/s (whole ACE build step)",
        "value": round(value, 1),
        "unit": "pair solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "mixed": "f32+bf16split", "real64": "f64",
                  "real32": "f32+bf16split"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['desc']}", "precision": prec,
                   "grid": n, "L_bohr": L, "n_occ": nocc, "n_band": nband, "n_x": nx,
                   "pairs_per_step": pairs, "parallelism": "single GPU"},
        "roofline": roofline,
        "extra": extra,
    }
    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = with_ratios(cpu_baseline(cfg), value)
    if args.workload == "cfg2" and not args.no_cpu and not args.no_others:
        extra["other_workloads"] = other_workloads(args)
    print(json.dumps(out), flush=True)
    ctx.close()


def other_workloads(args):
    """The other configurations, a few timed steps each, as child processes of
    this run (so that one bench invocation times every workload): the summary
    of each one's JSON line."""
    import subprocess
    res = {}
    steps, warmup = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    for w in ("cfg1", "cfg2r", "cfg3", "cfg4", "cfg5"):
        log(f"bench: other workload {w} ({steps} steps)")
        cmd = [sys.executable, os.path.abspath(__file__), "--workload", w, "--steps", str(steps),
               "--warmup", str(warmup), "--no-cpu", "--no-others"]
        try:
            r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
            line = [x for x in r.stdout.strip().splitlines() if x.startswith("{")]
            if r.returncode != 0 or not line:
                res[w] = {"error": f"exit {r.returncode}: {r.stderr.strip()[-300:]}"}
                continue
            d = json.loads(line[-1])
        except (subprocess.TimeoutExpired, json.JSONDecodeError) as e:
            res[w] = {"error": repr(e)[:300]}
            continue
        e = d.get("extra", {})
        rf = d.get("roofline") or {}
        res[w] = {k: v for k, v in {
            "config": d["config"].get("workload"), "metric": d["metric"], "value": d["value"],
            "unit": d["unit"], "ms_per_step": d["ms_per_step"], "steps": d["steps"],
            "dtype": d["dtype"],
            "roofline": {k2: rf.get(k2) for k2 in ("kernel", "bound", "achieved", "peak", "unit",
                                                   "frac", "traffic")},
            "errors_vs_fp64": e.get("errors_vs_fp64"), "errors_vs_oracle": e.get("errors_vs_oracle"),
            "forms": e.get("forms"), "stage_ms": e.get("stage_ms"),
        }.items() if v is not None}
    return res


def with_ratios(cpu, gpu_value):
    """GPU rate over the oracle's rate for each oracle mode timed."""
    r = {"all_cores" if cpu["cores"] > 1 else "single_core": gpu_value / cpu["value"]}
    if "single_core" in cpu:
        r["single_core"] = gpu_value / cpu["single_core"]["value"]
    cpu["ratio_gpu_over_oracle"] = r
    return cpu


def golden_errors(ctx, cfg, grid, prec, bufs, Xs, nocc):
    """Relative errors of the run's outputs against values the FP64 oracle
    computed for this workload (tests/golden, written by make_golden.py):
    E_X and eig(-M) for g0 = 0 and g0 = pi/mu^2, and sampled entries of
    V_ACE X_0 and V_ACE X_19."""
    import math

    import numpy as np
    import torch

    from paper_1601_07159_amd import ace
    with open(os.path.join(ROOT, cfg["golden"])) as f:
        gold = json.load(f)
    out = {}

    def rel(a, b):
        a, b = np.asarray(a), np.asarray(b)
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def samples(Y, d):
        Yc = Y.reshape(Y.shape[0], -1)
        idx_b = torch.tensor(d["band"], device=Y.device)
        idx_r = torch.tensor(d["point"], device=Y.device)
        v = Yc[idx_b, idx_r].cpu().numpy().astype(np.complex128)
        return rel(v, np.asarray(d["re"]) + 1j * np.asarray(d["im"]))

    Q = bufs["Q"]
    for tag, g0 in (("g0_0", 0.0), ("g0_pi_over_mu2", math.pi / cfg["mu"] ** 2)):
        gr = ace.Grid.cubic(grid.n, grid.L[0], grid.kind, grid.mu, g0)
        W = ctx.build_W(Q[:nocc], Q, gr, prec)
        xi, Lm = ctx.compress(Q, W, gr, prec, want_L=True)
        e = float(ctx.exchange_energy(Q[:nocc], gr, prec, xi=xi).item())
        eig = torch.linalg.eigvalsh((Lm @ Lm.conj().T).cpu()).numpy()
        ref_e = gold[f"E_X_trace_{tag}"]
        out[f"E_X_{tag}"] = abs(e - ref_e) / abs(ref_e)
        out[f"eig_minus_M_{tag}"] = rel(eig, gold[f"eig_minus_M_{tag}"])
        out[f"E_X_{tag}_value"] = e
        if tag == "g0_0" and Xs:
            out["V_ACE_X0_samples"] = samples(ctx.apply(xi, Xs[0], gr, prec), gold["apply_X0"])
            out["V_ACE_X19_samples"] = samples(ctx.apply(xi, Xs[-1], gr, prec),
                                               gold["apply_X19"])
        del W, xi
    torch.cuda.synchronize()
    return out


def _timed_loop(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _base_record(args, cfg, metric, value, unit, ms, dtype, config, roofline, extra):
    return {"metric": metric, "value": round(value, 1), "unit": unit, "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config, "roofline": roofline, "extra": extra}


def run_batched(args, cfg):
    """48 independent instances; one step = ace_build_W_batched (W and xi of
    every instance) replayed from its HIP graph.  Beside it (extra.forms), the
    same 48 builds as plain single calls on one stream, FP32 and FP64 (unless
    --no-fp64)."""
    import concurrent.futures as cf

    import torch

    from paper_1601_07159_amd import ace, synth
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    specs = synth.batched_instances()
    log("bench: cfg4: generating 48 instances")
    with cf.ThreadPoolExecutor(8) as ex:
        orbs = list(ex.map(synth.instance_orbitals, specs))
    insts, pairs, transformed, fft_bytes = [], 0, 0, 0
    for sp, psi in zip(specs, orbs):
        x = torch.from_numpy(psi).to(dev, torch.complex64).reshape(sp["nband"], -1)
        g = ace.Grid.cubic(sp["n"], sp["L"])
        insts.append(dict(grid=g, phi=x[:sp["nocc"]], psi=x, W=torch.empty_like(x),
                          xi=torch.empty_like(x),
                          info=torch.zeros(1, dtype=torch.int32, device=dev)))
        p = sp["nocc"] * sp["nband"]
        tr = sp["nocc"] * (sp["nocc"] + 1) // 2 + sp["nocc"] * (sp["nband"] - sp["nocc"])
        pairs += p
        transformed += tr
        fft_bytes += (3 * tr + p) * g.ng * 8
    del orbs
    ctx = ace.Context(0)
    nbr = args.branches
    tuned = {}
    if not args.no_autotune:
        # pair-batch width, band block and FFT line shape per grid size, tuned
        # on that size's median instance (outside the timed region)
        for n in sorted({sp["n"] for sp in specs}):
            same = sorted((sp for sp in specs if sp["n"] == n), key=lambda sp: sp["nocc"])
            med = same[len(same) // 2]
            r = ctx.autotune(ace.Grid.cubic(n, med["L"]), "fp32", med["nocc"], med["nband"])
            tuned[n] = {k: r[k] for k in ("pair_budget", "jblock", "fft_shape", "accum_shape")}
            log(f"bench: cfg4: autotuned n={n}: {tuned[n]} ({r['ms']:.2f} ms per build)")
    ctx.set_tuning("branches", nbr)
    forms = {}
    if args.batch_form == 0:
        # both forms of the W stage, the library default timed last
        ctx.set_tuning("batch_form", 2)
        forms["batched_persistent_fp32_ms"] = round(
            _timed_loop(lambda: ctx.build_batched(insts, "fp32"), args.steps, args.warmup) * 1e3, 3)
        log(f"bench: cfg4: persistent form {forms['batched_persistent_fp32_ms']:.2f} ms per step")
        ctx.set_tuning("batch_form", 1)
        forms["batched_launches_fp32_ms"] = round(
            _timed_loop(lambda: ctx.build_batched(insts, "fp32"), args.steps, args.warmup) * 1e3, 3)
        log(f"bench: cfg4: launches form {forms['batched_launches_fp32_ms']:.2f} ms per step")
        ctx.set_tuning("batch_form", 0)
    else:
        ctx.set_tuning("batch_form", args.batch_form)
    ms = _timed_loop(lambda: ctx.build_batched(insts, "fp32"), args.steps, args.warmup) * 1e3
    bad = [k for k, d in enumerate(insts) if int(d["info"].item()) != 0]
    log(f"bench: cfg4: batched graph {ms:.2f} ms per step")

    def singles(ds, prec):
        for d in ds:
            ctx.build_W(d["phi"], d["psi"], d["grid"], prec, out=d["W"])
            ctx.compress(d["psi"], d["W"], d["grid"], prec, out=d["xi"], info=d["info"])

    forms["batched_graph_fp32_ms"] = round(ms, 3)
    steps_f = max(1, min(args.steps, 3))
    forms["single_calls_fp32_ms"] = round(
        _timed_loop(lambda: singles(insts, "fp32"), steps_f, 1) * 1e3, 3)
    log(f"bench: cfg4: single calls fp32 {forms['single_calls_fp32_ms']:.2f} ms per step")
    if not args.no_fp64:
        d64 = []
        for d in insts:
            x = d["psi"].to(torch.complex128)
            d64.append(dict(grid=d["grid"], phi=x[:d["phi"].shape[0]], psi=x,
                            W=torch.empty_like(x), xi=torch.empty_like(x), info=d["info"]))
        forms["single_calls_fp64_ms"] = round(
            _timed_loop(lambda: singles(d64, "fp64"), steps_f, 1) * 1e3, 3)
        log(f"bench: cfg4: single calls fp64 {forms['single_calls_fp64_ms']:.2f} ms per step")
        del d64
        torch.cuda.empty_cache()
    achieved = fft_bytes / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "all FFT passes of the batch (graph replay)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes_per_launch": fft_bytes, "avg_launch_ms": round(ms, 4)}
    extra = {"instances": len(insts), "branches": nbr, "autotuned": tuned, "forms": forms,
             "pairs_per_step": pairs,
             "transformed_pairs_per_step": transformed, "failed_cholesky": bad,
             "fft_roofline_ms": fft_bytes / (HBM_PEAK_GBS * 1e9) * 1e3}
    config = {"workload": f"cfg4: {cfg['desc']}", "precision": "fp32",
              "instances": len(insts), "pairs_per_step": pairs, "parallelism": "single GPU"}
    out = _base_record(args, cfg, "pair Poisson solves/s (batched ACE build, 48 instances)",
                       pairs / (ms * 1e-3), "pair solves/s", ms, "f32", config, roofline, extra)
    if not args.no_cpu:
        sp = specs[0]
        out["cpu_baseline"] = with_ratios(
            cpu_baseline(dict(n=sp["n"], L=sp["L"], nocc=sp["nocc"], nband=sp["nband"],
                              kind="coulomb", mu=0.0)), out["value"])
    print(json.dumps(out), flush=True)
    ctx.close()


def run_autograd(args, cfg):
    """One step = E_X(phi) forward (pair spectra i <= j, Parseval sum) plus the
    hand-written backward dE/dphi* (W = V_X[phi] phi recomputed)."""
    import torch

    from paper_1601_07159_amd import ace, synth
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, L, nocc = cfg["n"], cfg["L"], cfg["nocc"]
    grid = ace.Grid.cubic(n, L)
    log("bench: cfg5: generating orbitals")
    phi0 = torch.from_numpy(synth.smooth_orbitals(n, L, nocc, seed=0)).to(
        dev, torch.complex64).reshape(nocc, -1)
    phi = phi0.clone().requires_grad_(True)
    ctx = ace.context(0)
    if args.fft_shape:
        ctx.set_tuning("fft_shape", args.fft_shape)

    def step():
        phi.grad = None
        e = ace.ExchangeEnergy.apply(phi, grid, "fp32")
        e.backward()

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ms = _timed_loop(step, args.steps, 0) * 1e3
    # per-kernel HIP events in a second region of the same length
    ctx.profile(True)
    ctx.profile_reset()
    ms_prof = _timed_loop(step, args.steps, 0) * 1e3
    prof = ctx.profile_report()
    ctx.profile(False)
    fwd_pairs = nocc * (nocc + 1) // 2
    bwd_pairs = nocc * nocc
    solves = fwd_pairs + bwd_pairs
    ng = grid.ng
    # per-kernel pairs per step: forward energy = slab + energy pencil pass on
    # the triangle; backward = build with the i <-> j symmetry (triangle only)
    units = {"pair_fwd_slab": 1, "plane_kernel": 2, "pencil_accum": 1, "pencil_energy": 1}
    per_step = {"pair_fwd_slab": 2 * fwd_pairs, "plane_kernel": fwd_pairs,
                "pencil_accum": bwd_pairs, "pencil_energy": fwd_pairs}
    dom = max(units, key=lambda k: prof.get(k, {"ms": 0})["ms"])
    d = prof[dom]
    avg_ms = d["ms"] / d["launches"]
    ppl = per_step[dom] * args.steps / d["launches"]
    achieved = units[dom] * ng * 8 * ppl / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "algorithmic_bytes_per_launch": round(units[dom] * ng * 8 * ppl),
                "avg_launch_ms": round(avg_ms, 4), "pairs_per_launch": ppl}
    roofline["traffic"] = measured_traffic(args.workload, dom, ppl)
    extra = {"forward_pairs": fwd_pairs, "backward_pairs": bwd_pairs,
             "profiled_ms_per_step": round(ms_prof, 4),
             "per_kernel": {k: {"launches": v["launches"], "avg_ms": round(v["ms"] / v["launches"], 5)}
                            for k, v in prof.items()}}
    if args.copy_probe:
        # a plain copy of known size, for the scaling of the HBM counters
        src = torch.zeros(256 * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        extra["copy_probe_bytes"] = 2 * src.numel() * 8
    config = {"workload": f"cfg5: {cfg['desc']}", "precision": "fp32", "grid": n, "L_bohr": L,
              "n_occ": nocc, "solves_per_step": solves, "parallelism": "single GPU"}
    out = _base_record(args, cfg, "pair Poisson solves/s (E_X forward + backward)",
                       solves / (ms * 1e-3), "pair solves/s", ms, "f32", config, roofline, extra)
    if not args.no_cpu:
        out["cpu_baseline"] = with_ratios(cpu_baseline(dict(cfg, nband=nocc)), out["value"])
    print(json.dumps(out), flush=True)


def run_scf(args, cfg):
    """The loops of Alg. 1 (V_X applied by pair solves in every Hamiltonian
    application) and Alg. 2 (V_ACE), and the loop without exchange, on the
    same input: time per inner (eigensolver) iteration and per ACE
    construction (the ratio the paper's timing figure reports), then the
    exchange-energy differences per outer iteration for the oversampling
    ratios r = N_band / N_occ = 1, 1.25, 1.5, 2 and for Alg. 1 (the
    oversampling study).  All loops start from the orbitals of the loop
    without exchange, converged first (as hybrid calculations start from a
    semilocal one)."""
    import numpy as np
    import torch

    from paper_1601_07159_amd import ace, synth
    from paper_1601_07159_amd.scf import ScfLoop
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n, L, nocc, prec = cfg["n"], cfg["L"], cfg["nocc"], cfg["prec"]
    grid = ace.Grid.cubic(n, L, cfg["kind"], cfg["mu"])
    ctx = ace.Context(0)
    vloc = synth.local_potential(n, L, seed=11, depth=cfg["depth"])
    ratios = [1.0, 1.25, 1.5, 2.0]
    nb_max = int(round(nocc * max(ratios))) + cfg["extra"]
    log(f"bench: scf: start orbitals ({nb_max}) and the loop without exchange")
    X0 = torch.from_numpy(synth.smooth_orbitals(n, L, nb_max, seed=0)).to(
        dev, torch.complex64).reshape(nb_max, -1)
    base = ScfLoop(ctx, grid, prec, vloc, nocc, nb_max - cfg["extra"], 0.0, "none",
                   cfg["degree"]).run(X0, n_inner=30, n_outer=1)
    Xs = base["X"].clone()
    nband = cfg["nband"]
    nb = nband + cfg["extra"]
    timing = {}
    for mode in ("none", "vx", "ace"):
        log(f"bench: scf: timing mode {mode}")
        lp = ScfLoop(ctx, grid, prec, vloc, nocc, nband, cfg["alpha"], mode, cfg["degree"])
        lp.run(Xs[:nb].clone(), n_inner=2, n_outer=1)           # warm-up
        lp.times = {"inner": [], "ace_build": [], "apply_h": []}
        lp.run(Xs[:nb].clone(), n_inner=cfg["inner"], n_outer=args.steps, timing=True)
        timing[mode] = {"inner_ms": float(np.median(lp.times["inner"])),
                        "ace_build_ms": float(np.median(lp.times["ace_build"]))}
    per_outer = {m: timing[m]["inner_ms"] * cfg["inner"] + timing[m]["ace_build_ms"]
                 for m in timing}
    conv = {}
    for r in ratios:
        nbr = int(round(nocc * r))
        log(f"bench: scf: convergence r = {r} (N_band = {nbr})")
        lp = ScfLoop(ctx, grid, prec, vloc, nocc, nbr, cfg["alpha"], "ace", cfg["degree"])
        out = lp.run(Xs[:nbr + cfg["extra"]].clone(), n_inner=cfg["inner"],
                     n_outer=cfg["outer"])
        conv[f"ace_r{r}"] = out["E_X"]
    log("bench: scf: convergence without ACE (Alg. 1)")
    lp = ScfLoop(ctx, grid, prec, vloc, nocc, nband, cfg["alpha"], "vx", cfg["degree"])
    out = lp.run(Xs[:nb].clone(), n_inner=cfg["inner"], n_outer=cfg["outer"])
    conv["vx"] = out["E_X"]
    diffs = {k: [abs(v[i] - v[i - 1]) for i in range(1, len(v))] for k, v in conv.items()}
    ratio = per_outer["vx"] / per_outer["ace"]
    roofline = {"bound": "hbm", "kernel": "n/a (loop timing)", "achieved": None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}
    extra = {"time_per_inner_iteration_ms": {m: round(timing[m]["inner_ms"], 3) for m in timing},
             "ace_construction_ms": round(timing["ace"]["ace_build_ms"], 3),
             "time_per_outer_iteration_ms": {m: round(v, 2) for m, v in per_outer.items()},
             "outer_time_ratio_vx_over_ace": ratio,
             "outer_time_ratio_vx_over_none": per_outer["vx"] / per_outer["none"],
             "outer_time_ratio_ace_over_none": per_outer["ace"] / per_outer["none"],
             "E_X_per_outer": conv, "E_X_difference_per_outer": diffs,
             "n_band_timing": nband, "buffer_vectors": cfg["extra"]}
    config = {"workload": f"scf: {cfg['desc']}", "precision": prec, "grid": n, "L_bohr": L,
              "n_occ": nocc, "parallelism": "single GPU"}
    out = _base_record(args, cfg, "outer-iteration time ratio, Alg. 1 (V_X) / Alg. 2 (ACE)",
                       ratio, "x", per_outer["ace"], "f32", config, roofline, extra)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

"""bench.py's command-line contract, on the CPU: more than one GPU is refused
with a message and exit status 2 before anything touches a device, and the
documented options exist."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--workload", "--no-cpu", "--no-fp64", "--no-others",
                "--fft-shape", "--accum-shape", "--batch-form", "--branches", "--copy-probe"):
        assert opt in r.stdout, opt
    for w in ("cfg1", "cfg2", "cfg2r", "cfg3", "cfg4", "cfg5", "scf"):
        assert w in r.stdout, w

"""The C-ABI checks of tests/native/host_checks.cpp, linked with libace's
host code built under AddressSanitizer and UndefinedBehaviorSanitizer (the
device code as usual; paper_1601_07159_amd/build.py builds both): a
host-side out-of-bounds access, use after free, leak or undefined operation
in argument validation, workspace management, the batched build's host logic,
the tuning-cache reader or the environment handling ends the program with a
sanitizer report.  Without a GPU only the checks that need no context run."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "native", "ace_host_checks")
SUPP = os.path.join(ROOT, "tests", "native", "lsan.supp")


def _run(args, tmp_path):
    if not os.path.exists(EXE):
        pytest.skip("sanitized host checks not built (paper_1601_07159_amd/build.py)")
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:detect_stack_use_after_return=1",
               LSAN_OPTIONS=f"suppressions={SUPP}:print_suppressions=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               TMPDIR=str(tmp_path))
    for k in ("ACE_LOG", "ACE_TUNE", "ACE_TUNE_CACHE"):
        env.pop(k, None)
    print(f"host checks {' '.join(args)}", flush=True)
    r = subprocess.run([EXE, *args], env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout[-4000:])
    print(r.stderr[-8000:])
    return r


def test_host_checks_without_context(tmp_path):
    r = _run(["--no-device"], tmp_path)
    assert r.returncode == 0
    assert ", 0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.gpu
def test_host_checks_on_gpu(tmp_path):
    r = _run([], tmp_path)
    assert r.returncode == 0
    assert ", 0 failures" in r.stdout and "skipped" not in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr

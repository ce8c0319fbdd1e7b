"""The C-ABI library loads and exports every function include/ace.h declares;
host-side argument handling needs no GPU."""
import ctypes
import os
import re

import pytest

from paper_1601_07159_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(ace_[A-Za-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libace.so not built")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 17
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.EXPORTED) <= declared


def test_status_strings_and_supported_sizes(lib):
    assert lib.ace_status_string(0) == b"ok"
    assert lib.ace_status_string(2) == b"matrix not positive definite"
    assert lib.ace_status_string(6) == b"not allowed while the stream is being captured"
    assert _lib.ACE_E_CAPTURE == 6
    buf = (ctypes.c_int * 32)()
    k = lib.ace_supported_n(buf, 32)
    sizes = [buf[i] for i in range(k)]
    for n in (24, 32, 40, 48, 64, 72):
        assert n in sizes


def test_null_context_is_an_argument_error(lib):
    g = _lib.AceGrid()
    assert lib.ace_build_W(None, ctypes.byref(g), 0, None, 1, 1, None, 1, 1, None, 1, 1.0) == 1
    assert lib.ace_compress(None, ctypes.byref(g), 0, None, 1, None, 1, 1, None, 1, None,
                            None) == 1
    assert lib.ace_apply(None, ctypes.byref(g), 0, None, 1, 1, None, 1, 1, None, 1) == 1
    assert lib.ace_destroy(None) == 1
    assert lib.ace_create(None, None, None) == 1


def test_environment_read_at_create(tmp_path):
    """ace_create reads ACE_LOG and ACE_TUNE_CACHE before it looks for a
    device: the log names the cache and the settings it held.  Without a GPU the
    call then fails with ACE_E_HIP; with one it succeeds."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    cache.write_text("16 8 0 0 8\n24 16 268435456 0 4 1\nnot a setting\n")
    log = tmp_path / "ace.log"
    code = (
        "import ctypes\n"
        "from paper_1601_07159_amd import _lib\n"
        "lib = _lib.load()\n"
        "c = ctypes.c_void_p()\n"
        "st = lib.ace_create(ctypes.byref(c), None, None)\n"
        "assert st in (0, 4), st\n"
        "if st == 0:\n"
        "    lib.ace_destroy(c)\n"
    )
    env = dict(os.environ, ACE_LOG=str(log), ACE_TUNE_CACHE=str(cache), ACE_TUNE="0",
               PYTHONPATH=ROOT)
    subprocess.run([sys.executable, "-c", code], env=env, check=True, cwd=ROOT, timeout=120)
    text = log.read_text()
    assert f"tuning cache {cache}: read, 2 settings" in text
    env["ACE_TUNE_CACHE"] = str(tmp_path / "absent.txt")
    subprocess.run([sys.executable, "-c", code], env=env, check=True, cwd=ROOT, timeout=120)
    assert "absent.txt: not found, 0 settings" in log.read_text()

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

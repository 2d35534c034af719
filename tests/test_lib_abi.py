"""CPU-side checks of the C ABI library: it loads, exports every symbol that
include/mlcr.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "mlcr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-zA-Z_][a-zA-Z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_symbols_exported():
    from paper_1308_5299_amd import _lib
    lib = _lib.load()
    names = _header_functions()
    assert "apply_A" in names and "sht_synth" in names and "wcycle_solve" in names
    for n in names:
        assert hasattr(lib, n), n
    # the binding covers every declared function
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def test_argument_errors_without_gpu():
    from paper_1308_5299_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.mlcr_geom_create(0, 10, ctypes.byref(h)) == -1
    assert b"nside" in lib.mlcr_last_error()
    assert lib.mlcr_geom_create(4, -1, ctypes.byref(h)) == -1
    assert lib.mlcr_geom_create(4, 8, None) == -1
    assert lib.sht_synth(None, 4, 1, None, None, 0, None) == -1
    assert lib.apply_A(None, 0, 1, None, None, 0, None) == -1
    assert lib.mlcr_version().startswith(b"mlcr")

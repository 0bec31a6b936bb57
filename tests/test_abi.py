"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/frobinv.h declares (no device work)."""
import ctypes
import os
import re

import pytest

from paper_2208_01239_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "frobinv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(frob_[a-z0-9_]+)\s*\(", text)))


def test_header_names_match_binding():
    names = header_functions()
    assert names, "no declarations found"
    assert set(names) == set(_lib.SIGNATURES), (set(names) ^ set(_lib.SIGNATURES))


def test_library_exports_every_symbol():
    lib = _lib.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_defaults_without_device():
    lib = _lib.load()
    assert lib.frob_status_string(0) == b"FROB_OK"
    assert lib.frob_status_string(1) == b"FROB_SINGULAR"
    assert lib.frob_status_string(-1) == b"FROB_E_ARG"
    o = _lib.frob_opts_t()
    lib.frob_default_opts(ctypes.byref(o))
    assert o.shift == _lib.FROB_SHIFT_AUTO and o.refine == 0 and o.mu == 0.0


def test_argument_validation_without_device():
    lib = _lib.load()
    # null handle and bad sizes are rejected before any device call
    assert lib.frob_inv_general(None, 4, None, 4, None, 4, None, None, 4, None, None) == _lib.FROB_E_ARG
    assert lib.frob_destroy(None) == _lib.FROB_E_ARG
    h = ctypes.c_void_p()
    assert lib.frob_create(None, 0) == _lib.FROB_E_ARG

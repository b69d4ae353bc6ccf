"""The C ABI: the built library loads and exports every function include/gf2.h
declares; the Python binding uses the same names.  No GPU needed."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gf2.h")
LIB = os.path.join(ROOT, "paper_1405_3273_amd", "libgf2.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gf2_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls_of_the_method():
    names = declared_functions()
    for fn in ("gf2_sigma_tau", "gf2_fourier", "gf2_dyson", "gf2_density_fock", "gf2_iterate"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libgf2.so is not built (python -m paper_1405_3273_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1405_3273_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()
    for n in _lib.EXPORTED:
        assert callable(getattr(_lib, n))


def test_struct_layouts_match_header_sizes():
    """ctypes mirrors of the structs have the C sizes (ints and doubles, natural alignment)."""
    from paper_1405_3273_amd import _lib
    assert ctypes.sizeof(_lib.gf2_dims) == 4 * 4 + 8
    assert ctypes.sizeof(_lib.gf2_params) == 4 * 8 + 2 * 4 + 8 + 8 + 4 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(_lib.gf2_state) == 8 + 4 * 8 + 4 + 4 + 8
    assert ctypes.sizeof(_lib.gf2_report) == 6 * 8 + 2 * 4 + 4 * 8


def test_last_error_is_callable_without_a_gpu():
    if not os.path.exists(LIB):
        pytest.fail("libgf2.so is not built")
    lib = ctypes.CDLL(LIB)
    lib.gf2_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.gf2_last_error(), bytes)

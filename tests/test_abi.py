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


def _c_layout():
    """sizeof and field offsets of the ABI structs as the C compiler lays them out."""
    import subprocess
    import tempfile
    fields = {"gf2_dims": ["n", "nelec", "ntau", "niw", "beta"],
              "gf2_params": [f for f, _ in _params_fields()],
              "gf2_state": ["mu", "F", "P", "G_tau", "Sigma_tau", "iteration", "has_P", "energy"],
              "gf2_report": ["energy", "e1b", "e2b", "dE", "dP", "mu", "n_inner", "n_eval",
                             "ms_sigma", "ms_fourier", "ms_inner", "ms_total"]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gf2.h"', "int main(void) {"]
    for st, fl in fields.items():
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(src, "w") as fh:
            fh.write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    res = {}
    for line in out.splitlines():
        st, key, val = line.split()
        res[(st, key)] = int(val)
    return res


def _params_fields():
    from paper_1405_3273_amd import _lib
    return _lib.gf2_params._fields_


def test_struct_layouts_match_header():
    """ctypes mirrors of the structs have the C compiler's sizes and field offsets."""
    from paper_1405_3273_amd import _lib
    lay = _c_layout()
    for st in ("gf2_dims", "gf2_params", "gf2_state", "gf2_report"):
        cls = getattr(_lib, st)
        assert ctypes.sizeof(cls) == lay[(st, "size")], st
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == lay[(st, f)], (st, f)


def test_last_error_is_callable_without_a_gpu():
    if not os.path.exists(LIB):
        pytest.fail("libgf2.so is not built")
    lib = ctypes.CDLL(LIB)
    lib.gf2_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.gf2_last_error(), bytes)

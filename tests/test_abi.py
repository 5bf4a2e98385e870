"""CPU checks of the C-ABI library: it loads and exports every entry point pp.h declares."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pp_[a-z_]+)\s*\(", text)) - {"pp_alloc_fn", "pp_release_fn"})


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["pp_create_observable", "pp_apply_layer", "pp_truncate", "pp_expectation"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2606_20441_amd import pp
    if not os.path.exists(pp.LIB_PATH):
        from paper_2606_20441_amd import build
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", pp.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(pp_[a-z_]+)\b", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    assert set(pp.EXPORTED) <= exported


def test_library_loads_without_gpu():
    import ctypes
    from paper_2606_20441_amd import pp
    lib = ctypes.CDLL(pp.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    lib.pp_last_error.restype = ctypes.c_char_p
    assert lib.pp_last_error() == b""


def test_c_header_compiles_as_c():
    src = os.path.join(ROOT, "include", "pp.h")
    r = subprocess.run(["gcc", "-fsyntax-only", "-x", "c", "-std=c99", "-Wall", "-Werror", src],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

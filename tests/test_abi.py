"""The C-ABI library loads and exports every entry point include/rfa.h
declares (no compute calls: this runs without a GPU)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_1907_05709_amd import rfa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(rfa_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for must in ("rfa_create_grid", "rfa_set_tissue", "rfa_set_needle", "rfa_step",
                 "rfa_damage"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(rfa.LIB_PATH):
        pytest.fail("librfa.so not built (python -m paper_1907_05709_amd.build)")
    L = ctypes.CDLL(rfa.LIB_PATH)
    missing = [n for n in declared_entry_points() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_entry_points()) <= set(rfa.exported_symbols())


def test_status_strings_without_gpu():
    # pure host functions: no device work
    assert rfa.rfa_status_string(rfa.RFA_OK) == "ok"
    assert "stability" in rfa.rfa_status_string(rfa.RFA_ERR_UNSTABLE)
    o = rfa.rfa_default_options()
    assert o.t_death == 60.0 and o.A == 7.39e39 and o.R == 8.314 and o.omega_cap == 1e30


@pytest.mark.parametrize("lang,std", [("c", "-std=c99"), ("c++", "-std=c++11")])
def test_header_compiles_as_plain_c_and_cpp(lang, std, tmp_path):
    """The boundary is usable from C: the header needs no C++ or HIP types."""
    import shutil
    import subprocess
    cc = shutil.which("gcc" if lang == "c" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    src = tmp_path / ("use.c" if lang == "c" else "use.cpp")
    src.write_text('#include "rfa.h"\nint main(void) { rfa_options o; '
                   'return rfa_default_options(&o) == RFA_OK ? 0 : 1; }\n')
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

"""CPU-side checks of the C ABI: the library loads and exports every symbol
that include/*.h declares, and the binding knows each signature. No compute
call is made (there is no GPU here)."""
import os
import re
import subprocess

import pytest

import paper_2609_07204_amd as mc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(mc_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_headers_declare_entry_points():
    names = declared_symbols()
    assert {"mc_ctx_create", "mc_mincut", "mc_workspace_size", "mc_last_error"} <= names
    assert {"mc_step_contract", "mc_step_capforest", "mc_step_pr12", "mc_step_components"} <= names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmincut.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", mc.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = declared_symbols() - exported
    assert not missing, missing


def test_binding_covers_every_symbol():
    assert declared_symbols() == set(mc.SIGNATURES)
    if os.path.exists(mc.LIB_PATH):
        L = mc.lib()
        for name in mc.SIGNATURES:
            assert getattr(L, name) is not None


def test_default_options_and_errors_without_gpu():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmincut.so not built")
    o = mc.default_options()
    assert o.seed == 1 and o.heuristic_min_n == 10000 and o.lp_iters == 2
    import ctypes
    b = ctypes.c_size_t()
    # invalid arguments are rejected before any device call
    assert mc.lib().mc_workspace_size(None, 10, 10, ctypes.byref(b)) == -1
    assert mc.lib().mc_mincut(None, None, None, 0, None, None, None) == -1
    assert b"NULL" in mc.lib().mc_last_error()
    assert mc.lib().mc_step_ws_size(0, 0, 1, ctypes.byref(b)) == -1
    assert mc.lib().mc_step_ws_size(100, 1000, 4, ctypes.byref(b)) == 0 and b.value > 0

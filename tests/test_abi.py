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


def _need_lib():
    if not os.path.exists(mc.LIB_PATH):
        pytest.skip("libmincut.so not built")


def test_check_graph_statuses():
    # the host checks that mc_mincut, mc_mincut_batch and mc_server_submit
    # run before any device work (no GPU needed)
    _need_lib()
    import numpy as np
    import gen
    g = gen.random_small(9, 0.6, 5, 1, 9)
    assert mc.check_graph(g) == 0 and mc.check_graph(g, symmetric=True) == 0
    one = gen.Graph(1, np.zeros(2, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64))
    assert mc.check_graph(one) == -1                                      # n < 2
    bad = gen.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    bad.row_ptr[2], bad.row_ptr[3] = bad.row_ptr[3], bad.row_ptr[2] + 1  # decreasing
    if bad.row_ptr[2] > bad.row_ptr[3]:
        assert mc.check_graph(bad) == -2
    bad = gen.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    bad.col[0] = g.n                                                       # target out of range
    assert mc.check_graph(bad) == -2
    bad = gen.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    bad.w[0] = -3                                                          # negative weight
    assert mc.check_graph(bad) == -2
    asym = gen.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    asym.w[0] += 1                                                         # one direction heavier
    assert mc.check_graph(asym) == 0 and mc.check_graph(asym, symmetric=True) == -2
    big = gen.from_edges(2, [0], [1], [1 << 61])
    assert mc.check_graph(big) == -3                                       # 2 * 2^61 = 2^62
    ok = gen.from_edges(2, [0], [1], [(1 << 61) - 1])
    assert mc.check_graph(ok) == 0


def test_option_values_rejected_before_device_work():
    _need_lib()
    import ctypes
    h = ctypes.c_void_p()
    for field, value in [("pr_tri_deg_cap", 65), ("pr_tri_deg_cap", -1), ("batch_pass_threads", 100),
                         ("batch_lp", 3), ("capforest_mode", 3), ("deterministic", 2), ("lp_iters", -1),
                         ("finish_max_n", 1025), ("queue", 3), ("contract_mode", 2), ("contract_mode", -1)]:
        o = mc.default_options(**{field: value})
        assert mc.lib().mc_ctx_create(0, None, ctypes.byref(o), ctypes.byref(h)) == -1, field
        assert field in mc.lib().mc_last_error().decode()
    assert mc.lib().mc_ctx_set_options(None, None) == -1


def test_outputs_untouched_on_argument_errors():
    _need_lib()
    import ctypes
    import numpy as np
    lam = ctypes.c_int64(-77)
    side = np.full(4, 9, np.uint8)
    assert mc.lib().mc_mincut(None, None, None, 0, ctypes.byref(lam), side.ctypes.data, None) == -1
    assert lam.value == -77 and (side == 9).all()
    lams = np.full(3, -5, np.int64)
    st = np.full(3, 99, np.int32)
    assert mc.lib().mc_mincut_batch(None, 3, None, None, 0, lams.ctypes.data, None, st.ctypes.data) == -1
    assert (lams == -5).all() and (st == 99).all()

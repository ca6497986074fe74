"""CPU oracle for the exact minimum-cut solver -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its binding) never
links, imports or calls it, and the two share no code.

Thin ctypes wrappers over oracle.c; see that file for what each routine
computes and which passage of the paper it follows.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile oracle.c into liboracle.so with the host C compiler."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        for name in ("orc_brute", "orc_stoer_wagner"):
            getattr(lib, name).argtypes = [i32, P, P, P, P]
            getattr(lib, name).restype = i64
        lib.orc_noi.argtypes = [i32, P, P, P, P, P]
        lib.orc_noi.restype = i64
        lib.orc_brute_st.argtypes = [i32, P, P, P, i32, i32]
        lib.orc_brute_st.restype = i64
        lib.orc_cut_value.argtypes = [i32, P, P, P, P]
        lib.orc_cut_value.restype = i64
        lib.orc_degrees.argtypes = [i32, P, P, P, P]
        lib.orc_degrees.restype = None
        lib.orc_components.argtypes = [i32, i64, P, P, P]
        lib.orc_components.restype = i32
        lib.orc_contract.argtypes = [i32, P, P, P, P, i32, P, P, P]
        lib.orc_contract.restype = i64
        lib.orc_pr12.argtypes = [i32, P, P, P, i64, P, P]
        lib.orc_pr12.restype = None
        lib.orc_pr34.argtypes = [i32, P, P, P, i64, i32, P, P, P, P]
        lib.orc_pr34.restype = None
        lib.orc_lp.argtypes = [i32, P, P, P, P, P]
        lib.orc_lp.restype = None
        lib.orc_capforest_pass.argtypes = [i32, P, P, P, P, i32, i32, P, P, P, P, P]
        lib.orc_capforest_pass.restype = i64
        _lib = lib
    return _lib


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, np.int32)
    col = np.ascontiguousarray(g.col, np.int32)
    w = np.ascontiguousarray(g.w, np.int64)
    return rp, col, w


def _ptr(a):
    return a.ctypes.data if a.size else None


def _solve(fn, g):
    rp, col, w = _csr(g)
    side = np.zeros(max(g.n, 1), np.uint8)
    lam = fn(g.n, _ptr(rp), _ptr(col), _ptr(w), side.ctypes.data)
    if lam < 0:
        raise ValueError("oracle failed with code %d" % lam)
    return int(lam), side[:g.n]


def brute(g):
    """Minimum cut by enumerating every cut (n <= 24). Returns (lambda, side)."""
    if g.n > 24:
        raise ValueError("brute force is limited to n <= 24")
    return _solve(_L().orc_brute, g)


def stoer_wagner(g):
    """Stoer-Wagner minimum cut. Returns (lambda, side) with side[0] == 0."""
    return _solve(_L().orc_stoer_wagner, g)


def noi(g, return_rounds=False):
    """Repeated full CAPFOREST + contraction. Returns (lambda, side)."""
    rp, col, w = _csr(g)
    side = np.zeros(max(g.n, 1), np.uint8)
    rounds = np.zeros(1, np.int32)
    lam = _L().orc_noi(g.n, _ptr(rp), _ptr(col), _ptr(w), side.ctypes.data, rounds.ctypes.data)
    if lam < 0:
        raise ValueError("oracle failed with code %d" % lam)
    if return_rounds:
        return int(lam), side[:g.n], int(rounds[0])
    return int(lam), side[:g.n]


def mincut(g):
    """lambda and a side, by the cheapest oracle that applies to the size."""
    if g.n <= 16:
        return brute(g)
    if g.n <= 3000:
        return stoer_wagner(g)
    return noi(g)


def brute_st(g, s, t):
    """Minimum s-t cut by enumeration (n <= 24)."""
    rp, col, w = _csr(g)
    return int(_L().orc_brute_st(g.n, _ptr(rp), _ptr(col), _ptr(w), s, t))


def cut_value(g, side):
    rp, col, w = _csr(g)
    side = np.ascontiguousarray(side, np.uint8)
    return int(_L().orc_cut_value(g.n, _ptr(rp), _ptr(col), _ptr(w), side.ctypes.data))


def degrees(g):
    rp, col, w = _csr(g)
    out = np.zeros(max(g.n, 1), np.int64)
    _L().orc_degrees(g.n, _ptr(rp), _ptr(col), _ptr(w), out.ctypes.data)
    return out[:g.n]


def components(n, a, b):
    """Canonical component labels of the pairs (a[i], b[i]) on [0,n):
    components numbered by their smallest vertex. Returns (labels, count)."""
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    lab = np.zeros(max(n, 1), np.int32)
    nc = _L().orc_components(n, a.size, _ptr(a), _ptr(b), lab.ctypes.data)
    return lab[:n], int(nc)


def contract(g, labels, n2):
    """Canonical contraction of g by labels in [0, n2): rows sorted by target,
    loops dropped, parallel entries summed. Returns a gen.Graph-like tuple
    (row_ptr, col, w)."""
    rp, col, w = _csr(g)
    labels = np.ascontiguousarray(labels, np.int32)
    orp = np.zeros(n2 + 1, np.int32)
    ocol = np.zeros(max(g.nnz, 1), np.int32)
    ow = np.zeros(max(g.nnz, 1), np.int64)
    m2 = _L().orc_contract(g.n, _ptr(rp), _ptr(col), _ptr(w), labels.ctypes.data, n2,
                           orp.ctypes.data, ocol.ctypes.data, ow.ctypes.data)
    if m2 < 0:
        raise MemoryError("orc_contract")
    return orp, ocol[:m2].copy(), ow[:m2].copy()


def pr12(g, lam):
    """Padberg-Rinaldi test 1 flags per entry and test-2 pointer per vertex."""
    rp, col, w = _csr(g)
    flag = np.zeros(max(g.nnz, 1), np.uint8)
    ptr = np.zeros(max(g.n, 1), np.int32)
    _L().orc_pr12(g.n, _ptr(rp), _ptr(col), _ptr(w), lam, flag.ctypes.data, ptr.ctypes.data)
    return flag[:g.nnz], ptr[:g.n]


def pr34(g, lam, D, ptr2):
    """Padberg-Rinaldi tests 3 and 4 on candidate edges whose rows both have
    at most D entries (see orc_pr34): test-4 flag per entry, smallest test-3
    partner per vertex, accepted test-3 partner per vertex (a matching that
    avoids test-2 pointers)."""
    rp, col, w = _csr(g)
    ptr2 = np.ascontiguousarray(ptr2, np.int32)
    flag = np.zeros(max(g.nnz, 1), np.uint8)
    part = np.zeros(max(g.n, 1), np.int32)
    acc = np.zeros(max(g.n, 1), np.int32)
    _L().orc_pr34(g.n, _ptr(rp), _ptr(col), _ptr(w), lam, D, ptr2.ctypes.data, flag.ctypes.data,
                  part.ctypes.data, acc.ctypes.data)
    return flag[:g.nnz], part[:g.n], acc[:g.n]


def lp_round(g, lab_in):
    rp, col, w = _csr(g)
    lab_in = np.ascontiguousarray(lab_in, np.int32)
    out = np.zeros(max(g.n, 1), np.int32)
    _L().orc_lp(g.n, _ptr(rp), _ptr(col), _ptr(w), lab_in.ctypes.data, out.ctypes.data)
    return out[:g.n]


def capforest_pass(g, lam, start, max_scan=0):
    """One sequential CAPFOREST pass (see oracle.c). Returns a dict with the
    canonical labels of the marked pairs, the scan order, the bound after the
    pass, the smallest valid alpha and the prefix length where it occurs."""
    rp, col, w = _csr(g)
    lam_io = np.array([lam], np.int64)
    lab = np.zeros(max(g.n, 1), np.int32)
    order = np.zeros(max(g.n, 1), np.int32)
    nscan = np.zeros(1, np.int32)
    best_alpha = np.zeros(1, np.int64)
    best_len = np.zeros(1, np.int32)
    marks = _L().orc_capforest_pass(g.n, _ptr(rp), _ptr(col), _ptr(w), lam_io.ctypes.data, start,
                                    max_scan, lab.ctypes.data, order.ctypes.data, nscan.ctypes.data,
                                    best_alpha.ctypes.data, best_len.ctypes.data)
    return {"marks": int(marks), "labels": lab[:g.n], "order": order[:int(nscan[0])],
            "lam": int(lam_io[0]), "best_alpha": int(best_alpha[0]), "best_len": int(best_len[0])}

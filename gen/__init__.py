"""Seeded synthetic graph inputs for the minimum-cut solver and its oracle.

This module only builds inputs: undirected graphs with non-negative integer
weights, returned as symmetric CSR (int32 row pointers and targets, int64
weights, every row sorted by target, no loops, no parallel edges). It holds
none of the solver's arithmetic; both the CPU oracle and the GPU path consume
what it produces.

The random families are generated in C (gen.c) from splitmix64 streams; the
small closed-form families used as pins are built here with numpy.
"""
import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")


def build(force=False):
    """Compile gen.c into libgen.so with the host C compiler."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Edges(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("cap", ctypes.c_int64),
                ("u", ctypes.POINTER(ctypes.c_int32)), ("v", ctypes.POINTER(ctypes.c_int32)),
                ("w", ctypes.POINTER(ctypes.c_int64))]


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        E = ctypes.POINTER(_Edges)
        i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        sig = {
            "gen_regular": [i32, i32, u64, E],
            "gen_planted": [i32, i32, i32, i32, i64, i64, u64, E],
            "gen_er": [i32, dbl, u64, E],
            "gen_chung_lu": [i32, dbl, dbl, dbl, u64, E],
            "gen_rhg": [i32, dbl, dbl, u64, E],
            "gen_weights": [E, i64, i64, u64],
            "gen_kcore": [E, i32],
            "gen_lcc": [E],
            "gen_shuffle": [E, u64],
            "gen_to_csr": [E, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.gen_free.argtypes = [E]
        lib.gen_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR of an undirected weighted graph."""
    n: int
    row_ptr: np.ndarray  # int32, n+1
    col: np.ndarray      # int32, row_ptr[n]
    w: np.ndarray        # int64, row_ptr[n]
    name: str = ""

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    @property
    def m(self):
        return self.nnz // 2

    def edges(self):
        """(u, v, w) arrays of the undirected edges with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        keep = src < self.col
        return src[keep], self.col[keep].astype(np.int64), self.w[keep]


def _finish(e, wlo, whi, seed, name, weights_set=False):
    lib = _L()
    if not weights_set:
        if lib.gen_weights(ctypes.byref(e), wlo, whi, seed) != 0:
            raise MemoryError("gen_weights")
    n, m = int(e.n), int(e.m)
    rp = np.empty(n + 1, np.int32)
    col = np.empty(max(2 * m, 1), np.int32)
    w = np.empty(max(2 * m, 1), np.int64)
    if lib.gen_to_csr(ctypes.byref(e), rp.ctypes.data, col.ctypes.data, w.ctypes.data) != 0:
        raise MemoryError("gen_to_csr")
    lib.gen_free(ctypes.byref(e))
    return Graph(n, rp, col[:2 * m].copy(), w[:2 * m].copy(), name)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


def _post(e, kcore, lcc, shuffle, seed):
    lib = _L()
    if kcore:
        _check(lib.gen_kcore(ctypes.byref(e), kcore), "gen_kcore")
    if lcc:
        _check(lib.gen_lcc(ctypes.byref(e)), "gen_lcc")
    if shuffle:
        _check(lib.gen_shuffle(ctypes.byref(e), seed), "gen_shuffle")


def regular(n, d, seed, wlo=1, whi=1):
    e = _Edges()
    _check(_L().gen_regular(n, d, seed, ctypes.byref(e)), "gen_regular")
    return _finish(e, wlo, whi, seed, "regular(n=%d,d=%d)" % (n, d))


def planted(na, nb, d, bridges, wlo, whi, seed):
    """Two random d-regular blocks with weights in [wlo,whi] joined by
    `bridges` cross edges of weight 1 (minimum cut = bridges w.h.p.)."""
    e = _Edges()
    _check(_L().gen_planted(na, nb, d, bridges, wlo, whi, seed, ctypes.byref(e)), "gen_planted")
    return _finish(e, 0, 0, seed, "planted(%d+%d,d=%d,k=%d)" % (na, nb, d, bridges), weights_set=True)


def erdos_renyi(n, p, seed, wlo=1, whi=1, lcc=True):
    e = _Edges()
    _check(_L().gen_er(n, p, seed, ctypes.byref(e)), "gen_er")
    _post(e, 0, lcc, False, seed)
    return _finish(e, wlo, whi, seed, "er(n=%d,p=%.3g)" % (n, p))


def chung_lu(n, beta, avg_deg, seed, wlo=1, whi=1, kcore=0, lcc=True, shuffle=True, cap=0.0):
    e = _Edges()
    _check(_L().gen_chung_lu(n, beta, avg_deg, cap, seed, ctypes.byref(e)), "gen_chung_lu")
    _post(e, kcore, lcc, shuffle, seed)
    return _finish(e, wlo, whi, seed, "chung_lu(n=%d,beta=%g,d=%g,k=%d)" % (n, beta, avg_deg, kcore))


def rhg(n, avg_deg, gamma, seed, wlo=1, whi=1, kcore=0, lcc=True, shuffle=True):
    e = _Edges()
    _check(_L().gen_rhg(n, avg_deg, gamma, seed, ctypes.byref(e)), "gen_rhg")
    _post(e, kcore, lcc, shuffle, seed)
    return _finish(e, wlo, whi, seed, "rhg(n=%d,d=%g,gamma=%g,k=%d)" % (n, avg_deg, gamma, kcore))


# ----------------------------------------------------------- from edge lists
def from_edges(n, u, v, w, name=""):
    """Build the canonical symmetric CSR from undirected edges. Loops are
    dropped and parallel edges summed, so the result is a simple graph."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    w = np.asarray(w, np.int64)
    keep = u != v
    u, v, w = u[keep], v[keep], w[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    if a.size:
        key = a * n + b
        order = np.argsort(key, kind="stable")
        key, w = key[order], w[order]
        uniq, start = np.unique(key, return_index=True)
        w = np.add.reduceat(w, start)
        a, b = uniq // n, uniq % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return Graph(n, rp, dst.astype(np.int32), ww.astype(np.int64), name)


def raw_csr(n, u, v, w, name=""):
    """Symmetric CSR that keeps loops and parallel edges exactly as given
    (each undirected edge listed in both rows, loops listed once), with rows
    in input order. Used to exercise input normalisation."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    w = np.asarray(w, np.int64)
    loop = u == v
    src = np.concatenate([u, v[~loop]])
    dst = np.concatenate([v, u[~loop]])
    ww = np.concatenate([w, w[~loop]])
    order = np.argsort(src, kind="stable")
    src, dst, ww = src[order], dst[order], ww[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return Graph(n, rp, dst.astype(np.int32), ww.astype(np.int64), name)


# ------------------------------------------------------- splitmix64 in Python
_M64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 stream (Steele, Lea and Flood 2014)."""

    def __init__(self, seed):
        self.s = seed & _M64

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & _M64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def below(self, k):
        return (self.next() * k) >> 64

    def unit(self):
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


# -------------------------------------------------------- closed-form graphs
def complete(n, weight=1):
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, np.full(u.size, weight), "K_%d" % n)


def cycle(weights):
    weights = np.asarray(weights, np.int64)
    n = weights.size
    u = np.arange(n)
    return from_edges(n, u, (u + 1) % n, weights, "cycle(%d)" % n)


def random_tree(n, seed, wlo=1, whi=100):
    r = SplitMix64(seed)
    par = [r.below(i) for i in range(1, n)]
    w = [wlo + r.below(whi - wlo + 1) for _ in range(1, n)]
    return from_edges(n, np.arange(1, n), par, w, "tree(%d)" % n)


def two_cliques(a, b, k, inner_weight=1):
    """K_a on [0,a) and K_b on [a,a+b) joined by k unit bridges whose
    endpoints are all distinct (k <= min(a,b))."""
    ua, va = np.triu_indices(a, 1)
    ub, vb = np.triu_indices(b, 1)
    u = np.concatenate([ua, ub + a, np.arange(k)])
    v = np.concatenate([va, vb + a, a + np.arange(k)])
    w = np.concatenate([np.full(ua.size + ub.size, inner_weight), np.ones(k, np.int64)])
    return from_edges(a + b, u, v, w, "cliques(%d,%d,k=%d)" % (a, b, k))


def wheel(n):
    """Hub 0 and rim 1..n-1 (n >= 4): spokes of weight 2 and rim edges of
    weight n-2, so every vertex has degree 2n-2."""
    rim = np.arange(1, n)
    u = np.concatenate([np.zeros(n - 1, np.int64), rim])
    v = np.concatenate([rim, np.roll(rim, -1)])
    w = np.concatenate([np.full(n - 1, 2), np.full(n - 1, n - 2)])
    return from_edges(n, u, v, w, "wheel(%d)" % n)


def random_small(n, p, seed, wlo=0, whi=9):
    """G(n,p) with weights in [wlo,whi] (may be disconnected or contain
    zero-weight edges): for exhaustive pins on tiny inputs."""
    r = SplitMix64(seed)
    u, v, w = [], [], []
    for i in range(n):
        for j in range(i + 1, n):
            if r.unit() < p:
                u.append(i)
                v.append(j)
                w.append(wlo + r.below(whi - wlo + 1))
    return from_edges(n, u, v, w, "small(n=%d,p=%g,s=%d)" % (n, p, seed))


def permute(g, seed):
    """Relabel the vertices of g by a seeded random permutation."""
    r = SplitMix64(seed)
    perm = list(range(g.n))
    for i in range(g.n - 1, 0, -1):
        j = r.below(i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    perm = np.asarray(perm, np.int64)
    u, v, w = g.edges()
    return from_edges(g.n, perm[u], perm[v], w, g.name + "^perm"), perm


def scale(g, k):
    return Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w * k, "%s*%d" % (g.name, k))


def disjoint_union(g, h):
    u1, v1, w1 = g.edges()
    u2, v2, w2 = h.edges()
    return from_edges(g.n + h.n, np.concatenate([u1, u2 + g.n]), np.concatenate([v1, v2 + g.n]),
                      np.concatenate([w1, w2]), g.name + "+" + h.name)


# ------------------------------------------------------------ the workloads
def config_planted_2x1000(seed=1):
    """Two random 12-regular blocks of 1,000 vertices, weights in [1,10],
    joined by 5 weight-1 cross edges."""
    return planted(1000, 1000, 12, 5, 1, 10, seed)


def config_chung_lu(log2n=22, seed=1):
    """Chung-Lu, n=2^log2n, exponent 2.5, mean degree 20, reduced to the LCC
    of its 10-core, unit weights."""
    return chung_lu(1 << log2n, 2.5, 20.0, seed, 1, 1, kcore=10, lcc=True)


def config_rhg(log2n=23, seed=1):
    """Threshold random hyperbolic graph, n=2^log2n, mean degree 64,
    power-law exponent 5, LCC of the 32-core, weights in [1,100]."""
    return rhg(1 << log2n, 64.0, 5.0, seed, 1, 100, kcore=32, lcc=True)


def batch_params(i, seed0=1000, nmin=64, nmax=65536, dmin=8, dmax=32):
    """Size, mean degree and family of graph i of the batched workload:
    n log-uniform in [nmin,nmax], mean degree uniform in {dmin..dmax},
    family i mod 3 (0 planted, 1 Erdos-Renyi, 2 Chung-Lu)."""
    r = SplitMix64(seed0 + i)
    u = r.unit()
    n = int(math.floor(nmin * (nmax / nmin) ** u))
    n = max(nmin, min(nmax, n))
    d = dmin + r.below(dmax - dmin + 1)
    return n, d, i % 3


def mixed_graph(n, d, fam, seed, wlo, whi):
    """One graph of the mixed planted / Erdos-Renyi / Chung-Lu families."""
    if fam == 0:
        na, nb = n // 2, n - n // 2
        dd = max(2, min(d - (d % 2), na - 1 - ((na - 1) % 2)))
        return planted(na, nb, dd, 5, wlo, whi, seed)
    if fam == 1:
        return erdos_renyi(n, min(1.0, d / max(1, n - 1)), seed, wlo, whi, lcc=True)
    return chung_lu(n, 2.5, float(d), seed, wlo, whi, kcore=0, lcc=True)


def served_params(j, seed0=2000000):
    """Edge count, mean degree and family of pool graph j of the served
    workload: m = floor(10^(3 + 4U)), mean degree uniform in {8..32},
    family j mod 3; n = max(64, 2m / d)."""
    r = SplitMix64(seed0 + j)
    m = int(math.floor(10 ** (3 + 4 * r.unit())))
    d = 8 + r.below(25)
    n = max(64, (2 * m) // d)
    return n, d, j % 3


def config_served_graph(j, seed0=2000000):
    n, d, fam = served_params(j, seed0)
    return mixed_graph(n, d, fam, seed0 + j, 1, 1000)


def config_batch_graph(i, seed0=1000):
    n, d, fam = batch_params(i, seed0)
    return mixed_graph(n, d, fam, seed0 + i, 1, 100)

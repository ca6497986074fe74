"""Checks of the seeded input generators (structure, not the method)."""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import gen


def _well_formed(g):
    rp, col, w = g.row_ptr, g.col, g.w
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size == w.size
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col != src)
    for v in range(min(g.n, 200)):
        assert np.all(np.diff(col[rp[v]:rp[v + 1]]) > 0)
    A = sp.csr_matrix((w, col, rp), shape=(g.n, g.n))
    assert (A != A.T).nnz == 0


def _connected(g):
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    return connected_components(A, directed=False)[0] == 1


def test_regular_and_planted():
    g = gen.regular(200, 6, 3, 1, 1)
    _well_formed(g)
    assert np.all(np.diff(g.row_ptr) == 6)
    p = gen.config_planted_2x1000()
    _well_formed(p)
    deg = np.diff(p.row_ptr)
    assert p.n == 2000 and p.m == 12005
    assert deg.min() == 12 and int(deg.sum()) == 2 * 12005
    cross = [(u, c) for u in range(1000) for c in p.col[p.row_ptr[u]:p.row_ptr[u + 1]] if c >= 1000]
    assert len(cross) == 5
    assert p.w.min() >= 1 and p.w.max() <= 10


def test_seed_reproducible():
    a = gen.config_batch_graph(5)
    b = gen.config_batch_graph(5)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)
    c = gen.config_batch_graph(6)
    assert a.n != c.n or not np.array_equal(a.col, c.col)


def test_chung_lu_core():
    g = gen.config_chung_lu(14)
    _well_formed(g)
    assert np.diff(g.row_ptr).min() >= 10
    assert _connected(g)
    assert np.all(g.w == 1)


def test_rhg_core():
    g = gen.rhg(1 << 12, 32.0, 5.0, 1, 1, 100, kcore=16)
    _well_formed(g)
    assert np.diff(g.row_ptr).min() >= 16
    assert _connected(g)
    assert g.w.min() >= 1 and g.w.max() <= 100
    assert 20 < g.nnz / g.n < 48


def test_er_lcc():
    g = gen.erdos_renyi(3000, 8 / 2999, 4, 1, 100)
    _well_formed(g)
    assert _connected(g)
    assert 6 < g.nnz / g.n < 10


def test_batch_params_ranges():
    ns = []
    for i in range(300):
        n, d, fam = gen.batch_params(i)
        assert 64 <= n <= 65536 and 8 <= d <= 32 and fam == i % 3
        ns.append(n)
    med = np.median(ns)
    assert 800 < med < 5000  # log-uniform over [64, 65536]: median 2048


def test_dense_regular_blocks_by_complement():
    # d close to n - 1: the pairing model gives up and the generator takes
    # the complement of an (n-1-d)-regular graph; the result is still a
    # simple d-regular graph
    for n, d, seed in [(33, 30, 5), (20, 18, 1), (9, 8, 3)]:
        g = gen.regular(n, d, seed)
        deg = np.diff(g.row_ptr)
        assert (deg == d).all(), (n, d, set(deg))
        assert all(len(set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]])) == d for v in range(n))
        assert not any(v in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] for v in range(n))
    g = gen.config_batch_graph(747, 5000)   # halves of 33 vertices, 30-regular
    assert g.n == 66

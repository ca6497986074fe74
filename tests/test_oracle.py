"""Pins for the CPU oracle: every solver and step oracle is checked against
something other than itself -- closed forms, exhaustive enumeration, library
routines, invariants of the definitions (paper, Section 2 and 2.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import gen
import oracle

SOLVERS = [("brute", oracle.brute), ("sw", oracle.stoer_wagner), ("noi", oracle.noi)]


def check_side(g, lam, side):
    assert side.shape == (g.n,)
    assert side[0] == 0
    assert 0 < int(side.sum()) < g.n
    assert oracle.cut_value(g, side) == lam


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("name,fn", SOLVERS)
@pytest.mark.parametrize("n", [2, 3, 4, 7, 11])
def test_complete_graph(name, fn, n):
    lam, side = fn(gen.complete(n, weight=3))
    assert lam == 3 * (n - 1)
    check_side(gen.complete(n, weight=3), lam, side)


@pytest.mark.parametrize("name,fn", SOLVERS)
@pytest.mark.parametrize("seed", range(8))
def test_weighted_cycle(name, fn, seed):
    r = gen.SplitMix64(seed)
    n = 3 + seed % 10
    wts = [1 + r.below(50) for _ in range(n)]
    g = gen.cycle(wts)
    lam, side = fn(g)
    assert lam == sum(sorted(wts)[:2])
    check_side(g, lam, side)


@pytest.mark.parametrize("name,fn", SOLVERS)
@pytest.mark.parametrize("seed", range(8))
def test_tree(name, fn, seed):
    g = gen.random_tree(2 + 2 * seed, seed, 1, 100)
    lam, side = fn(g)
    assert lam == int(g.w.min())
    check_side(g, lam, side)


@pytest.mark.parametrize("name,fn", SOLVERS)
@pytest.mark.parametrize("a,b,k", [(3, 4, 1), (5, 5, 2), (6, 8, 4), (9, 7, 6)])
def test_two_cliques(name, fn, a, b, k):
    g = gen.two_cliques(a, b, k)
    lam, side = fn(g)
    assert lam == k
    check_side(g, lam, side)


@pytest.mark.parametrize("name,fn", SOLVERS)
@pytest.mark.parametrize("n", [4, 5, 9, 13])
def test_wheel(name, fn, n):
    g = gen.wheel(n)
    lam, side = fn(g)
    assert lam == 2 * n - 2
    check_side(g, lam, side)


@pytest.mark.parametrize("name,fn", SOLVERS)
def test_two_vertices(name, fn):
    g = gen.from_edges(2, [0], [1], [17])
    assert fn(g)[0] == 17


@pytest.mark.parametrize("name,fn", SOLVERS)
def test_disconnected(name, fn):
    g = gen.disjoint_union(gen.complete(4), gen.cycle([2, 3, 4]))
    lam, side = fn(g)
    assert lam == 0
    check_side(g, lam, side)


# ----------------------------------------------------- exhaustive agreement
@pytest.mark.parametrize("seed", range(400))
def test_solvers_agree_small(seed):
    n = 2 + seed % 15
    g = gen.random_small(n, [0.2, 0.5, 0.9][seed % 3], seed, 0, 9)
    lam, side = oracle.brute(g)
    check_side(g, lam, side)
    for name, fn in SOLVERS[1:]:
        l2, s2 = fn(g)
        assert l2 == lam, name
        check_side(g, l2, s2)


def test_brute_matches_explicit_enumeration():
    # the Gray-code update against a direct sum over every set S
    for seed in range(20):
        g = gen.random_small(9, 0.6, 100 + seed, 0, 20)
        best = None
        for mask in range(1, 1 << (g.n - 1)):
            side = np.array([0] + [(mask >> (x - 1)) & 1 for x in range(1, g.n)], np.uint8)
            c = oracle.cut_value(g, side)
            best = c if best is None else min(best, c)
        assert oracle.brute(g)[0] == best


# -------------------------------------------------------------- metamorphic
@pytest.mark.parametrize("seed", range(20))
def test_scale_and_permutation(seed):
    g = gen.random_small(10 + seed % 5, 0.5, 7000 + seed, 1, 30)
    lam = oracle.brute(g)[0]
    for name, fn in SOLVERS:
        assert fn(gen.scale(g, 7))[0] == 7 * lam
        gp, _ = gen.permute(g, seed)
        assert fn(gp)[0] == lam


def test_raising_a_weight_never_lowers_lambda():
    for seed in range(20):
        g = gen.random_small(11, 0.5, 900 + seed, 1, 9)
        lam = oracle.brute(g)[0]
        h = gen.Graph(g.n, g.row_ptr.copy(), g.col.copy(), g.w.copy())
        j = seed % h.nnz
        u = int(np.searchsorted(h.row_ptr, j, side="right") - 1)
        v = int(h.col[j])
        h.w[j] += 5
        k = h.row_ptr[v] + int(np.where(h.col[h.row_ptr[v]:h.row_ptr[v + 1]] == u)[0][0])
        h.w[k] += 5
        assert oracle.noi(h)[0] >= lam
        assert oracle.stoer_wagner(h)[0] >= lam


def test_raw_input_folding():
    # loops are ignored and parallel edges add up
    g = gen.raw_csr(4, [0, 0, 1, 2, 2, 3, 1], [1, 1, 2, 3, 2, 0, 1], [2, 3, 4, 5, 100, 6, 50])
    simple = gen.from_edges(4, [0, 1, 2, 3], [1, 2, 3, 0], [5, 4, 5, 6])
    for name, fn in SOLVERS:
        assert fn(g)[0] == oracle.brute(simple)[0] == 9


# ------------------------------------------------- larger closed forms
@pytest.mark.parametrize("name,fn", SOLVERS[1:])
def test_larger_closed_forms(name, fn):
    assert fn(gen.complete(40))[0] == 39
    wts = [5 + (i * 37) % 91 for i in range(700)]
    assert fn(gen.cycle(wts))[0] == sum(sorted(wts)[:2])
    t = gen.random_tree(1500, 3, 2, 500)
    assert fn(t)[0] == int(t.w.min())
    assert fn(gen.two_cliques(25, 30, 7))[0] == 7
    assert fn(gen.wheel(120))[0] == 238


def test_planted_two_blocks():
    g = gen.config_planted_2x1000()
    assert g.n == 2000 and g.m == 12005
    lam_sw, side_sw = oracle.stoer_wagner(g)
    lam_noi, side_noi = oracle.noi(g)
    assert lam_sw == lam_noi == 5
    check_side(g, 5, side_sw)
    check_side(g, 5, side_noi)


# ------------------------------------------------------------ step oracles
def test_degrees():
    g = gen.raw_csr(5, [0, 1, 1, 2, 3], [1, 2, 2, 2, 4], [3, 4, 5, 9, 1])
    assert list(oracle.degrees(g)) == [3, 12, 9, 1, 1]


def _check_contraction(g, lab, n2):
    rp, col, w = oracle.contract(g, lab, n2)
    assert rp[0] == 0 and rp.size == n2 + 1
    loops = sum(int(g.w[j]) for v in range(g.n) for j in range(g.row_ptr[v], g.row_ptr[v + 1])
                if lab[v] == lab[g.col[j]])
    assert int(w.sum()) == int(g.w.sum()) - loops
    for x in range(n2):
        row = col[rp[x]:rp[x + 1]]
        assert np.all(np.diff(row) > 0)
        assert np.all(row != x)
        # the collapsed degree is the capacity of the group's cut
        side = (lab == x).astype(np.uint8)
        assert int(w[rp[x]:rp[x + 1]].sum()) == oracle.cut_value(g, side)
    # entry (x,y) is the total weight between the two groups
    for x in range(n2):
        for j in range(rp[x], rp[x + 1]):
            y = col[j]
            mask = (lab[:, None] == x) & (lab[None, :] == y)
            dense = np.zeros((g.n, g.n), np.int64)
            for v in range(g.n):
                for k in range(g.row_ptr[v], g.row_ptr[v + 1]):
                    dense[v, g.col[k]] += g.w[k]
            assert int(dense[mask].sum()) == int(w[j])


@pytest.mark.parametrize("seed", range(10))
def test_contraction_invariants(seed):
    g = gen.random_small(12, 0.5, 300 + seed, 1, 9)
    r = gen.SplitMix64(seed)
    n2 = 1 + r.below(g.n)
    lab = np.array([r.below(n2) for _ in range(g.n)], np.int32)
    lab[:n2] = np.arange(n2)  # every label used
    _check_contraction(g, lab, n2)


def test_identity_contraction_is_canonical_folding():
    r = gen.SplitMix64(5)
    u = [r.below(30) for _ in range(400)]
    v = [r.below(30) for _ in range(400)]
    w = [r.below(7) for _ in range(400)]
    raw = gen.raw_csr(30, u, v, w)
    rp, col, ww = oracle.contract(raw, np.arange(30, dtype=np.int32), 30)
    ref = gen.from_edges(30, u, v, w)
    keep = ref.w != 0
    src = np.repeat(np.arange(30), np.diff(ref.row_ptr))[keep]
    assert np.array_equal(np.repeat(np.arange(30), np.diff(rp)), src)
    assert np.array_equal(col, ref.col[keep])
    assert np.array_equal(ww, ref.w[keep])


@pytest.mark.parametrize("seed", range(10))
def test_components_match_scipy(seed):
    r = gen.SplitMix64(seed)
    n = 50 + seed
    k = r.below(60)
    a = np.array([r.below(n) for _ in range(k)], np.int32)
    b = np.array([r.below(n) for _ in range(k)], np.int32)
    lab, nc = oracle.components(n, a, b)
    m = sp.coo_matrix((np.ones(k), (a, b)), shape=(n, n))
    nc_ref, lab_ref = connected_components(m, directed=False)
    assert nc == nc_ref
    # same partition
    assert len(set(zip(lab.tolist(), lab_ref.tolist()))) == nc
    # canonical numbering: first occurrences appear as 0, 1, 2, ...
    first = [lab[v] for v in range(n) if lab[v] not in lab[:v]]
    assert first == list(range(nc))


def test_pr12_definitions():
    g = gen.from_edges(5, [0, 0, 1, 2, 3], [1, 2, 2, 3, 4], [6, 1, 2, 7, 7])
    flag, ptr = oracle.pr12(g, 7)
    heavy = [(u, int(c)) for u in range(5) for c, ww in
             zip(g.col[g.row_ptr[u]:g.row_ptr[u + 1]], g.w[g.row_ptr[u]:g.row_ptr[u + 1]]) if ww >= 7]
    got = [(u, int(g.col[j])) for u in range(5) for j in range(g.row_ptr[u], g.row_ptr[u + 1]) if flag[j]]
    assert got == heavy
    # degrees 7, 8, 10, 14, 7; heaviest neighbours 1 (6), 0 (6), 3 (7),
    # 2 and 4 tied at 7 (smaller id wins), 3 (7); all pass 2c >= deg
    assert list(ptr) == [1, 0, 3, 2, 3]
    flag, ptr = oracle.pr12(gen.from_edges(4, [0, 1, 1], [1, 2, 3], [3, 4, 2]), 100)
    # degrees 3, 9, 4, 2: vertex 1's heaviest edge (4) is less than half of 9
    assert list(ptr) == [1, -1, 1, 1] and not flag.any()


def _contract_marks(g, pairs):
    a = np.array([p[0] for p in pairs], np.int32)
    b = np.array([p[1] for p in pairs], np.int32)
    lab, nc = oracle.components(g.n, a, b)
    rp, col, w = oracle.contract(g, lab, nc)
    return gen.Graph(nc, rp, col, w), nc


def test_pr2_counterexample_single_pointer():
    # two 5-cliques of weight 10 and a vertex joined to one vertex of each by
    # weight 3: both edges pass the exchange test, only one may be applied
    X = list(range(5))
    Y = list(range(5, 10))
    a = 10
    u, v, w = [], [], []
    for S in (X, Y):
        for i in S:
            for j in S:
                if i < j:
                    u.append(i); v.append(j); w.append(10)
    u += [a, a]; v += [0, 5]; w += [3, 3]
    g = gen.from_edges(11, u, v, w)
    lam = oracle.brute(g)[0]
    assert lam == 3
    lam_hat = int(oracle.degrees(g).min())
    assert lam_hat == 6
    flag, ptr = oracle.pr12(g, lam_hat)
    assert ptr[a] == 0
    pairs = [(x, int(g.col[j])) for x in range(g.n) for j in range(g.row_ptr[x], g.row_ptr[x + 1]) if flag[j]]
    pairs += [(x, int(ptr[x])) for x in range(g.n) if ptr[x] >= 0]
    h, nc = _contract_marks(g, pairs)
    assert nc == 2 and oracle.brute(h)[0] == 3
    # applying both exchange edges at once would lose the cut
    h2, nc2 = _contract_marks(g, pairs + [(a, 5)])
    assert nc2 == 1


@pytest.mark.parametrize("seed", range(60))
def test_pr12_safe_contraction(seed):
    # contracting every test-1 edge and every test-2 pointer keeps lambda
    # whenever the bound is above it
    g = gen.random_small(6 + seed % 8, 0.6, 5000 + seed, 1, 12)
    lam = oracle.brute(g)[0]
    lam_hat = int(oracle.degrees(g).min())
    if lam_hat <= lam:
        return
    flag, ptr = oracle.pr12(g, lam_hat)
    pairs = [(x, int(g.col[j])) for x in range(g.n) for j in range(g.row_ptr[x], g.row_ptr[x + 1]) if flag[j]]
    pairs += [(x, int(ptr[x])) for x in range(g.n) if ptr[x] >= 0]
    h, nc = _contract_marks(g, pairs)
    assert nc >= 2
    assert oracle.brute(h)[0] == lam


@pytest.mark.parametrize("seed", range(20))
def test_lp_round_rule(seed):
    g = gen.random_small(25, 0.3, 800 + seed, 1, 5)
    r = gen.SplitMix64(seed)
    lab = np.array([r.below(6) for _ in range(g.n)], np.int32)
    out = oracle.lp_round(g, lab)
    for v in range(g.n):
        tot = {}
        for j in range(g.row_ptr[v], g.row_ptr[v + 1]):
            tot[int(lab[g.col[j]])] = tot.get(int(lab[g.col[j]]), 0) + int(g.w[j])
        own = tot.get(int(lab[v]), 0)
        chosen = int(out[v])
        if chosen == lab[v]:
            assert all(t <= own for l, t in tot.items() if l != lab[v])
        else:
            assert tot[chosen] > own
            assert tot[chosen] == max(tot.values())
            assert chosen == min(l for l, t in tot.items() if t == tot[chosen] and l != lab[v])


@pytest.mark.parametrize("seed", range(40))
def test_capforest_marks_are_safe(seed):
    # every pair joined by marks has connectivity >= the final bound, and the
    # recorded alpha is the capacity of the recorded prefix
    g = gen.random_small(5 + seed % 8, 0.6, 6000 + seed, 1, 9)
    if connected_components(sp.csr_matrix((g.w, g.col, g.row_ptr), shape=(g.n, g.n)))[0] > 1:
        return
    lam0 = int(oracle.degrees(g).min())
    res = oracle.capforest_pass(g, lam0, seed % g.n)
    assert res["order"].size == g.n
    lab = res["labels"]
    for x in range(g.n):
        for y in range(x + 1, g.n):
            if lab[x] == lab[y]:
                assert oracle.brute_st(g, x, y) >= res["lam"]
    if res["best_len"] > 0:
        side = np.zeros(g.n, np.uint8)
        side[res["order"][:res["best_len"]]] = 1
        assert oracle.cut_value(g, side) == res["best_alpha"]
        assert res["lam"] == min(lam0, res["best_alpha"])
    if res["lam"] == lam0:
        assert res["marks"] >= 1  # a full pass with a fixed bound marks an edge


def test_capforest_truncated_pass():
    g = gen.complete(8, weight=2)
    res = oracle.capforest_pass(g, 14, 3, max_scan=3)
    assert list(res["order"]) == [3, 0, 1]
    # after two scans every vertex has r = 4; at the third scan r = 6, below 14
    assert res["marks"] == 0


# ------------------------------------------------ Padberg-Rinaldi tests 3, 4
def test_pr34_hand_example():
    # a 4-cycle 0-1-2-3 with chord 0-2 (weights below) and a pendant 4 on 3:
    # edge {0,2} has common neighbours 1 and 3:
    #   s(0,2) = 5 + min(2, 3) + min(4, 1) = 8
    # edge {0,1}: common neighbour 2: s = 2 + min(5, 3) = 5
    g = gen.from_edges(5, [0, 1, 2, 3, 0, 3], [1, 2, 3, 0, 2, 4], [2, 3, 1, 4, 5, 6])
    deg = oracle.degrees(g)
    assert list(deg) == [11, 5, 9, 11, 6]
    flag1, ptr = oracle.pr12(g, 100)
    flag4, part, acc = oracle.pr34(g, 8, 10, np.full(5, -1, np.int32))
    s = {}
    for v in range(5):
        for j in range(g.row_ptr[v], g.row_ptr[v + 1]):
            s[(v, int(g.col[j]))] = bool(flag4[j])
    assert s[(0, 2)] and s[(2, 0)]           # 8 >= 8
    assert not s[(0, 1)] and not s[(3, 4)]   # 5 < 8; no common neighbour
    # test 3 on {0,2} with u = 3: 2 (5 + 4) = 18 >= 11 and 2 (5 + 1) = 12 >= 9
    # on {0,1} with u = 2: 2 (2 + 5) = 14 >= 11 and 2 (2 + 3) = 10 >= 5
    # so vertex 0's smallest partner is 1, vertex 1's is 0 (its only
    # candidate with a common neighbour), vertex 2's is 0
    assert part[0] == 1 and part[1] == 0 and part[2] == 0
    assert acc[0] == 1 and acc[1] == 0 and acc[2] == -1
    # a test-2 pointer on vertex 1 blocks the pair
    flag4, part, acc = oracle.pr34(g, 8, 10, np.array([-1, 2, -1, -1, -1], np.int32))
    assert acc[0] == -1 and acc[1] == -1
    # the degree cap: rows of vertices 0 and 2 have 3 entries
    flag4, part, acc = oracle.pr34(g, 8, 2, np.full(5, -1, np.int32))
    assert not flag4.any()


def test_pr34_wheel_fires_test3_only():
    # rim edges of the weighted wheel: test 3 holds with the hub as witness,
    # test 4 does not (s = (n-2) + 2 < 2n-2); accepted pairs form a matching
    n = 12
    g = gen.wheel(n)
    lam = 2 * n - 2
    assert int(oracle.degrees(g).min()) == lam
    flag1, ptr = oracle.pr12(g, lam)
    assert not flag1.any() and (ptr < 0).all()
    flag4, part, acc = oracle.pr34(g, lam, 3, ptr)
    assert not flag4.any()
    rim = [v for v in range(g.n) if g.row_ptr[v + 1] - g.row_ptr[v] == 3]
    assert len(rim) == n - 1 and all(part[v] >= 0 for v in rim)
    matched = [v for v in range(g.n) if acc[v] >= 0]
    assert matched and all(acc[acc[v]] == v for v in matched)


def two_blocks(seed):
    """Two dense random blocks (weights 1..9) joined by one to three light
    bridges: small graphs whose minimum cut is usually below the minimum
    degree, so the tests run with a bound above lambda."""
    r = np.random.default_rng(seed)
    a, b = int(r.integers(3, 8)), int(r.integers(3, 8))
    u, v, w = [], [], []
    for lo, hi in ((0, a), (a, a + b)):
        for i in range(lo, hi):
            for j in range(i + 1, hi):
                if r.random() < 0.8:
                    u.append(i); v.append(j); w.append(int(r.integers(1, 10)))
    for _ in range(int(r.integers(1, 4))):
        u.append(int(r.integers(0, a))); v.append(int(r.integers(a, a + b))); w.append(int(r.integers(1, 4)))
    return gen.from_edges(a + b, u, v, w)


@pytest.mark.parametrize("seed", range(120))
def test_pr1234_safe_contraction(seed):
    # contracting every test-1 and test-4 edge, every test-2 pointer and the
    # accepted test-3 pairs together keeps lambda whenever the bound is
    # above it (brute force on small graphs)
    g = two_blocks(7000 + seed) if seed % 2 else gen.random_small(6 + seed % 9, 0.55, 7000 + seed, 1, 9)
    lam = oracle.brute(g)[0]
    lam_hat = int(oracle.degrees(g).min())
    if seed % 3 == 0:
        # bounds between lambda and the min degree too (the solver's bound
        # never exceeds the min degree: that is what makes a trivial cut
        # impossible as a cut below the bound)
        lam_hat = min(lam_hat, lam + 1 + seed % 4)
    if lam_hat <= lam:
        return
    flag1, ptr = oracle.pr12(g, lam_hat)
    flag4, part, acc = oracle.pr34(g, lam_hat, 64, ptr)
    pairs = [(x, int(g.col[j])) for x in range(g.n) for j in range(g.row_ptr[x], g.row_ptr[x + 1])
             if flag1[j] or flag4[j]]
    pairs += [(x, int(ptr[x])) for x in range(g.n) if ptr[x] >= 0]
    pairs += [(x, int(acc[x])) for x in range(g.n) if acc[x] >= 0]
    if not pairs:
        return
    h, nc = _contract_marks(g, pairs)
    assert nc >= 2
    assert oracle.brute(h)[0] == lam


def test_pr4_is_a_connectivity_bound():
    # s(v,x) never exceeds the true connectivity of v and x
    for seed in range(30):
        g = gen.random_small(10, 0.6, 9100 + seed, 1, 7)
        flag4, part, acc = oracle.pr34(g, 1, 64, np.full(g.n, -1, np.int32))
        for v in range(g.n):
            for j in range(g.row_ptr[v], g.row_ptr[v + 1]):
                x = int(g.col[j])
                # the largest lam for which test 4 holds is s(v,x)
                lo, hi = 0, 10 ** 6
                while lo < hi:
                    mid = (lo + hi + 1) // 2
                    f, _, _ = oracle.pr34(g, mid, 64, np.full(g.n, -1, np.int32))
                    if f[j]:
                        lo = mid
                    else:
                        hi = mid - 1
                assert lo <= oracle.brute_st(g, v, x)


@pytest.mark.parametrize("seed", [103230, 105901, 106297])
def test_pr3_needs_the_matching(seed):
    # graphs (found by search) where contracting every vertex's test-3
    # partner at once loses the minimum cut, while the accepted matching
    # alone keeps it
    g = two_blocks(seed)
    lam = oracle.brute(g)[0]
    lam_hat = int(oracle.degrees(g).min())
    assert lam_hat > lam
    none = np.full(g.n, -1, np.int32)
    flag4, part, acc = oracle.pr34(g, lam_hat, 64, none)
    h, nc = _contract_marks(g, [(v, int(part[v])) for v in range(g.n) if part[v] >= 0])
    assert nc < 2 or oracle.brute(h)[0] != lam
    matched = [(v, int(acc[v])) for v in range(g.n) if acc[v] >= 0]
    if matched:
        h, nc = _contract_marks(g, matched)
        assert nc >= 2 and oracle.brute(h)[0] == lam


# ------------------------------------------- hand-worked label-propagation round
def test_lp_round_hand_example():
    # Worked by hand from the synchronous rule (own label kept unless another
    # label is strictly heavier; ties among other labels to the smallest):
    #   v0: 7 -> 3 (own), 9 -> 2+1 = 3, not heavier     -> keeps 7
    #   v1: 7 -> 3 (own), 9 -> 4                        -> 9
    #   v2: 9 -> 5 (own), 7 -> 2+4 = 6                  -> 7
    #   v3: 9 -> 5 (own), 7 -> 1, 5 -> 2, 3 -> 2; loop ignored -> keeps 9
    #   v4: 5 -> 0 (own), 9 -> 2, 3 -> 2 (tie)          -> 3
    #   v5: 3 -> 0 (own), 9 -> 2, 5 -> 2 (tie)          -> 5
    #   v6: isolated                                    -> keeps 4
    u = [0, 0, 0, 1, 2, 3, 3, 4, 3]
    v = [1, 2, 3, 2, 3, 4, 5, 5, 3]
    w = [3, 2, 1, 4, 5, 2, 2, 2, 100]
    g = gen.raw_csr(7, u, v, w)
    lab = np.array([7, 7, 9, 9, 5, 3, 4], np.int32)
    assert list(oracle.lp_round(g, lab)) == [7, 9, 7, 9, 3, 5, 4]
    # splitting an edge into parallel entries of the same total changes nothing
    g2 = gen.raw_csr(7, u + [1], v + [2], w[:3] + [1] + w[4:] + [3])
    assert list(oracle.lp_round(g2, lab)) == [7, 9, 7, 9, 3, 5, 4]


# ------------------------------------------------------- s-t cut enumeration
def test_brute_st_hand_example():
    # triangle 0-1 (3), 1-2 (5), 0-2 (1):
    #   lambda(0,2) = min({0}: 3+1, {0,1}: 5+1) = 4
    #   lambda(1,2) = min({1}: 3+5, {0,1}: 5+1) = 6
    #   lambda(0,1) = min({0}: 3+1, {0,2}: 3+5) = 4
    g = gen.from_edges(3, [0, 1, 0], [1, 2, 2], [3, 5, 1])
    assert oracle.brute_st(g, 0, 2) == 4
    assert oracle.brute_st(g, 2, 0) == 4
    assert oracle.brute_st(g, 1, 2) == 6
    assert oracle.brute_st(g, 0, 1) == 4


@pytest.mark.parametrize("seed", range(12))
def test_brute_st_equals_max_flow(seed):
    # max-flow min-cut theorem: the smallest s-t cut equals the maximum s-t
    # flow, computed here by scipy's own routine on the symmetric capacities
    from scipy.sparse.csgraph import maximum_flow
    g = gen.random_small(6 + seed % 7, 0.5, 9100 + seed, 0, 9)
    cap = sp.csr_matrix((g.w.astype(np.int32), g.col, g.row_ptr), shape=(g.n, g.n))
    r = gen.SplitMix64(seed)
    for _ in range(4):
        s = r.below(g.n)
        t = (s + 1 + r.below(g.n - 1)) % g.n
        assert oracle.brute_st(g, s, t) == maximum_flow(cap, s, t).flow_value


@pytest.mark.parametrize("seed", range(12))
def test_brute_st_minimum_over_t_is_lambda(seed):
    # every cut separates vertex 0 from some t, so the global minimum is the
    # smallest s-t cut from vertex 0
    g = gen.random_small(5 + seed % 8, 0.5, 9200 + seed, 0, 9)
    lam, _ = oracle.brute(g)
    assert min(oracle.brute_st(g, 0, t) for t in range(1, g.n)) == lam

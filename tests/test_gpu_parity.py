"""GPU parity: every step kernel against the CPU oracle, element by element,
through the C ABI (include/mincut_steps.h), and the whole solver against
the oracle's lambda. Integer work, so the bar is bit-exact; where several
answers are correct (row order, the side of the cut) the unique part is
compared and the rest checked for validity."""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

CF_SHARED, CF_SEQUENTIAL, CF_PRIVATE, CF_LEVELS = 0, 1, 2, 3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2609_07204_amd as mc
    assert torch.cuda.is_available()
    c = mc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_sort():
    """A context whose contractions merge by radix sort (contract_mode 1)."""
    import paper_2609_07204_amd as mc
    c = mc.Context(0, contract_mode=1)
    yield c
    c.close()


@pytest.fixture(params=[0, 1], ids=["hash", "sort"])
def cctx(request, ctx, ctx_sort):
    """The context of each edge-merge mode."""
    return ctx if request.param == 0 else ctx_sort


def canon_dev(ctx, g):
    """Device padded graph of g with degrees filled (identity contraction)."""
    src = ctx.dgraph(g)
    dst, dmin, darg = ctx.step_contract(src)
    return dst, dmin, darg


def assert_same_csr(dev_graph, rp, col, w):
    drp, dcol, dw, ddeg = dev_graph.to_canonical()
    assert np.array_equal(drp, rp)
    assert np.array_equal(dcol, col)
    assert np.array_equal(dw, w)
    deg = np.add.reduceat(w, rp[:-1]) if w.size else np.zeros(len(rp) - 1, np.int64)
    deg = np.where(np.diff(rp) > 0, deg, 0)
    assert np.array_equal(ddeg, deg)


# --------------------------------------------------------- contraction
def raw_graph(n, m, seed, wmax=7):
    r = gen.SplitMix64(seed)
    u = [r.below(n) for _ in range(m)]
    v = [r.below(n) for _ in range(m)]
    w = [r.below(wmax + 1) for _ in range(m)]
    return gen.raw_csr(n, u, v, w)


@pytest.mark.parametrize("n,m,seed", [(2, 1, 1), (5, 30, 2), (40, 300, 3), (700, 9000, 4), (3000, 60000, 5)])
def test_normalise_matches_oracle(cctx, n, m, seed):
    say("normalise", n, m, seed)
    g = raw_graph(n, m, seed)
    dst, dmin, darg = canon_dev(cctx, g)
    rp, col, w = oracle.contract(g, np.arange(n, dtype=np.int32), n)
    assert_same_csr(dst, rp, col, w)
    deg = oracle.degrees(g)
    assert dmin == deg.min() and darg == int(np.argmin(deg))


def test_normalise_hub_rows(cctx):
    ctx = cctx
    # rows far longer than the chunk limit take the global-table path
    say("normalise hubs")
    r = gen.SplitMix64(9)
    u, v, w = [], [], []
    for hub in (0, 1, 2):
        for _ in range(5000):
            u.append(hub)
            v.append(r.below(400))
            w.append(1 + r.below(5))
    g = gen.raw_csr(400, u, v, w)
    dst, dmin, darg = canon_dev(ctx, g)
    rp, col, ww = oracle.contract(g, np.arange(400, dtype=np.int32), 400)
    assert_same_csr(dst, rp, col, ww)


@pytest.mark.parametrize("seed,n2frac", [(1, 0.5), (2, 0.05), (3, 0.9), (4, 0.002), (5, 1.0)])
def test_contract_random_labels(cctx, seed, n2frac):
    ctx = cctx
    say("contract labels", seed, n2frac)
    g = gen.erdos_renyi(4000, 12 / 3999, seed, 1, 50, lcc=False)
    r = gen.SplitMix64(100 + seed)
    n2 = max(1, int(g.n * n2frac))
    lab = np.array([r.below(n2) for _ in range(g.n)], np.int32)
    lab[:n2] = np.arange(n2)
    import torch
    src, _, _ = canon_dev(ctx, g)
    dst, dmin, darg = ctx.step_contract(src, torch.as_tensor(lab).cuda(), n2)
    rp, col, w = oracle.contract(g, lab, n2)
    assert_same_csr(dst, rp, col, w)
    deg = np.diff(rp)
    odeg = np.array([w[rp[x]:rp[x + 1]].sum() for x in range(n2)])
    assert dmin == odeg.min() and darg == int(np.argmin(odeg))


def test_contract_mixed_group_sizes(cctx):
    ctx = cctx
    # one giant group, many tiny ones, and medium groups straddling the
    # small/large threshold
    say("contract mixed groups")
    g = gen.chung_lu(20000, 2.5, 16.0, 7, 1, 9, kcore=0, lcc=True)
    n = g.n
    lab = np.arange(n, dtype=np.int32) // 37
    lab[: n // 5] = 0
    uniq, lab = np.unique(lab, return_inverse=True)
    lab = lab.astype(np.int32)
    n2 = int(uniq.size)
    import torch
    src, _, _ = canon_dev(ctx, g)
    dst, dmin, darg = ctx.step_contract(src, torch.as_tensor(lab).cuda(), n2)
    rp, col, w = oracle.contract(g, lab, n2)
    assert_same_csr(dst, rp, col, w)


@pytest.mark.parametrize("n2,seed,giants", [(50000, 4, 8), (150000, 5, 3), (9000, 6, 20)])
def test_contract_many_giant_groups(cctx, n2, seed, giants):
    # giant groups (at least n2 / 4 entries: dense accumulators) beside many
    # small groups, their targets spread over all of n2; half of a giant
    # group's entries point into the other giant groups (a few hot targets)
    ctx = cctx
    say("contract giant groups", n2, seed, giants)
    g = gen.chung_lu(200000, 2.5, 10.0, seed, 1, 30, kcore=0, lcc=False)
    rng = np.random.default_rng(seed)
    order = rng.permutation(g.n)
    lab = rng.integers(giants, n2, g.n).astype(np.int32)
    lab[order[: n2 - giants]] = np.arange(giants, n2, dtype=np.int32)   # every small group has a member
    per = min((g.n - (n2 - giants)) // giants, g.n // (2 * giants))   # members of each giant group
    for k in range(giants):
        lab[order[n2 - giants + k * per: n2 - giants + (k + 1) * per]] = k
    deg = np.diff(g.row_ptr)
    sizes = np.bincount(lab, weights=deg, minlength=n2)
    say("giant entries", sorted(sizes[:giants].astype(int))[:3], "n2/4", n2 // 4)
    assert (sizes[:giants] >= n2 // 4).all() and (sizes[:giants] > 2048).all()
    import torch
    src, _, _ = canon_dev(ctx, g)
    dst, dmin, darg = ctx.step_contract(src, torch.as_tensor(lab).cuda(), n2)
    rp, col, w = oracle.contract(g, lab, n2)
    assert_same_csr(dst, rp, col, w)
    odeg = np.array([w[rp[x]:rp[x + 1]].sum() for x in range(n2)])
    assert dmin == odeg.min() and darg == int(np.argmin(odeg))


def test_contract_groups_around_workgroup_limits(cctx):
    ctx = cctx
    # groups of 150..1300 members at about three entries each: below, inside
    # and above the range merged by one workgroup per group (by entries, and
    # by members on both sides of 1024)
    say("contract groups around workgroup limits")
    g = gen.erdos_renyi(30000, 3 / 29999, 11, 1, 40, lcc=False)
    sizes = [150, 200, 400, 700, 1024, 1025, 1300, 90]
    lab = np.empty(g.n, np.int32)
    pos, k = 0, 0
    while pos < g.n:
        c = sizes[k % len(sizes)]
        lab[pos:pos + c] = k
        pos += c
        k += 1
    n2 = k
    import torch
    src, _, _ = canon_dev(ctx, g)
    dst, dmin, darg = ctx.step_contract(src, torch.as_tensor(lab).cuda(), n2)
    rp, col, w = oracle.contract(g, lab, n2)
    assert_same_csr(dst, rp, col, w)
    odeg = np.array([w[rp[x]:rp[x + 1]].sum() for x in range(n2)])
    assert dmin == odeg.min() and darg == int(np.argmin(odeg))


@pytest.mark.parametrize("n2,seed", [(3, 1), (50000, 2), (150000, 3)])
def test_sort_merge_large_contractions(ctx_sort, n2, seed):
    # many tiles, an even (4) and an odd (5) number of radix passes, runs of
    # thousands of parallel entries (n2 = 3), labels in random order
    say("sort merge", n2, seed)
    g = gen.chung_lu(200000, 2.5, 10.0, seed, 1, 30, kcore=0, lcc=False)
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, n2, g.n).astype(np.int32)
    lab[:n2] = rng.permutation(n2).astype(np.int32)
    import torch
    src, _, _ = canon_dev(ctx_sort, g)
    dst, dmin, darg = ctx_sort.step_contract(src, torch.as_tensor(lab).cuda(), n2)
    rp, col, w = oracle.contract(g, lab, n2)
    assert_same_csr(dst, rp, col, w)
    odeg = np.array([w[rp[x]:rp[x + 1]].sum() for x in range(n2)])
    assert dmin == odeg.min() and darg == int(np.argmin(odeg))


def test_solves_with_sort_merge(ctx_sort):
    # whole solves whose every contraction merges by sorting
    cases = [(gen.config_planted_2x1000(), 5), (gen.wheel(300), 598), (gen.two_cliques(40, 50, 3), 3),
             (gen.disjoint_union(gen.complete(6), gen.cycle([2, 3, 4])), 0)]
    for g, lam in cases:
        say("sort-merge solve", g.name)
        solve_check(ctx_sort, g, lam)
        solve_check(ctx_sort, g, lam, device_input=True)
    for g in (gen.chung_lu(30000, 2.5, 12.0, 17, 1, 50, kcore=3, lcc=True),
              gen.rhg(20000, 16, 3.0, 5, 1, 100, kcore=0, lcc=True),
              gen.mixed_graph(5000, 16, 1, 6, 1, 1000)):
        say("sort-merge solve", g.name, g.n)
        solve_check(ctx_sort, g, oracle.noi(g)[0])


# ---------------------------------------------------------- union-find
@pytest.mark.parametrize("n,k,seed", [(1, 0, 1), (10, 5, 2), (5000, 3000, 3), (200000, 150000, 4)])
def test_components(ctx, n, k, seed):
    say("components", n, k)
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, k).astype(np.int32)
    b = rng.integers(0, n, k).astype(np.int32)
    lab, n2 = ctx.step_components(n, a, b)
    ref, nref = oracle.components(n, a, b)
    assert n2 == nref
    assert np.array_equal(lab, ref)


# ------------------------------------------------- reduction tests 1-2
@pytest.mark.parametrize("seed", range(6))
def test_pr12(ctx, seed):
    say("pr12", seed)
    g = gen.erdos_renyi(3000, 6 / 2999, seed, 1, 40, lcc=True) if seed % 2 else \
        gen.chung_lu(5000, 2.5, 8.0, seed, 1, 30, lcc=True)
    lam = int(oracle.degrees(g).min()) + seed * 3
    check_pr12(ctx, g, lam)


def _cycles(k, length=4, weight=5):
    """k disjoint cycles of `length` vertices, each joined into one tree by
    the first two unions of its rows."""
    base = np.arange(k)[:, None] * length
    u = (base + np.arange(length)).ravel()
    v = (base + (np.arange(length) + 1) % length).ravel()
    return gen.from_edges(k * length, u, v, np.full(u.size, weight), "cycles%d" % k)


# The test-1 trees left by the first two unions of every row are linked
# through byte labels and a bit matrix of tree pairs when there are at most
# 255 of them, else through root snapshots: both sides of that limit, a
# geometric graph whose few dozen trees share many test-1 entries, and a
# power-law graph with hundreds of trees.
@pytest.mark.parametrize("case,lam", [("rhg", 2), ("rhg", 30), ("cycles255", 2), ("cycles256", 2),
                                      ("cl", 20), ("rhg_many", 2)])
def test_pr12_tree_linking(ctx, case, lam):
    say("pr12 tree linking", case, lam)
    if case == "rhg":
        g = gen.rhg(20000, 16, 3.0, 5, 1, 100, kcore=0, lcc=True)
    elif case == "rhg_many":
        g = gen.rhg(60000, 12, 3.0, 8, 1, 100, kcore=0, lcc=False)
    elif case.startswith("cycles"):
        g = _cycles(int(case[6:]))
    else:
        g = gen.chung_lu(5000, 2.5, 8.0, 0, 1, 30, lcc=True)
    check_pr12(ctx, g, lam)


def check_pr12(ctx, g, lam):
    dev, _, _ = canon_dev(ctx, g)
    flag, ptr, lab, n2 = ctx.step_pr12(dev, lam)
    oflag, optr = oracle.pr12(g, lam)
    assert np.array_equal(ptr, optr)
    # flags live at the device entry positions: compare per (row, target)
    off = dev.off.cpu().numpy()
    col = dev.col.cpu().numpy()
    fl = flag.cpu().numpy()
    got = set()
    for v in range(g.n):
        for j in range(off[v], off[v] + int(dev.len[v])):
            if fl[j]:
                got.add((v, int(col[j])))
    ref = {(v, int(g.col[j])) for v in range(g.n) for j in range(g.row_ptr[v], g.row_ptr[v + 1]) if oflag[j]}
    assert got == ref
    pa = [p[0] for p in ref] + [v for v in range(g.n) if optr[v] >= 0]
    pb = [p[1] for p in ref] + [int(optr[v]) for v in range(g.n) if optr[v] >= 0]
    rl, rn = oracle.components(g.n, np.array(pa, np.int32), np.array(pb, np.int32))
    assert n2 == rn and np.array_equal(lab, rl)


# ------------------------------------------------------------ CAPFOREST
def cf_oracle(g, lam, start, cap=0):
    return oracle.capforest_pass(g, lam, start, max_scan=cap)


def check_cf_equal(res, ref):
    assert np.array_equal(res["order"], ref["order"])
    assert res["n2"] == int(ref["labels"].max()) + 1
    assert np.array_equal(res["labels"], ref["labels"])
    assert res["lam"] == ref["lam"]
    if ref["best_len"] > 0:
        assert res["best_alpha"] == ref["best_alpha"] and res["best_len"] == ref["best_len"]


CF_GRAPHS = [
    ("planted", lambda: gen.planted(300, 300, 8, 3, 1, 10, 5)),
    ("er", lambda: gen.erdos_renyi(800, 10 / 799, 3, 1, 100, lcc=True)),
    ("chung_lu", lambda: gen.chung_lu(1000, 2.5, 10.0, 4, 1, 1, kcore=3, lcc=True)),
    ("wheel", lambda: gen.wheel(200)),
    ("cliques", lambda: gen.two_cliques(30, 40, 5)),
    ("cycle", lambda: gen.cycle([1 + (i * 7919) % 97 for i in range(500)])),
]


@pytest.mark.parametrize("name,mk", CF_GRAPHS)
def test_capforest_complete_pass_matches_oracle(ctx, name, mk):
    g = mk()
    say("capforest complete", name, g.n)
    dev, dmin, _ = canon_dev(ctx, g)
    for start in (0, g.n // 2, g.n - 1):
        for lam in (dmin, max(1, dmin // 2), dmin * 3):
            res = ctx.step_capforest(dev, lam, start=start, mode=CF_SEQUENTIAL)
            check_cf_equal(res, cf_oracle(g, lam, start))


@pytest.mark.parametrize("name,mk", CF_GRAPHS)
def test_capforest_lds_pass_matches_oracle(ctx, name, mk):
    g = mk()
    say("capforest lds", name, g.n)
    dev, dmin, _ = canon_dev(ctx, g)
    for start in (0, g.n // 3):
        for cap in (0, 50):
            # every graph here has n + max degree <= 1536, so the pass never
            # runs out of hash capacity and must match the oracle exactly
            assert g.n + int(np.diff(g.row_ptr).max()) <= 1536
            res = ctx.step_capforest(dev, dmin, start=start, mode=CF_SHARED, passes=1, shared=False, len_cap=cap)
            check_cf_equal(res, cf_oracle(g, dmin, start, cap))


@pytest.mark.parametrize("mode", [0, 2, 3])
def test_capforest_parallel_marks_are_safe(ctx, mode):
    for seed in range(12):
        g = gen.random_small(12 + seed % 5, 0.5, 4000 + seed, 1, 9)
        lam_min = int(oracle.degrees(g).min())
        if g.nnz == 0 or lam_min == 0:
            continue
        say("capforest parallel safety", seed)
        dev, dmin, _ = canon_dev(ctx, g)
        res = ctx.step_capforest(dev, dmin, start=-1, mode=mode, passes=64, shared=True)
        # each pass marks against its own bound, which never drops below
        # min(dmin, smallest alpha of any pass); connectivity is ultrametric,
        # so every pair joined through marks clears that threshold
        thr = min(dmin, res["best_alpha"])
        lab = res["labels"]
        for x in range(g.n):
            for y in range(x + 1, g.n):
                if lab[x] == lab[y]:
                    assert oracle.brute_st(g, x, y) >= thr


# ---------------------------------------------------------- end to end
def solve_check(ctx, g, lam_ref, device_input=False):
    lam, side = ctx.mincut(dev=ctx.upload(g)) if device_input else ctx.mincut(g)
    assert lam == lam_ref, (g.name, lam, lam_ref)
    assert side[0] == 0
    if lam > 0 or g.n > 1:
        assert 0 < int(side.sum()) < g.n
    assert oracle.cut_value(g, side) == lam
    return side


def test_closed_forms(ctx):
    cases = [(gen.complete(2, 5), 5), (gen.complete(9), 8), (gen.complete(60, 3), 177),
             (gen.cycle([4, 9, 2, 7, 5, 3]), 5), (gen.two_cliques(12, 15, 4), 4), (gen.wheel(50), 98),
             (gen.wheel(4), 6), (gen.random_tree(300, 5, 3, 90), None),
             (gen.disjoint_union(gen.complete(5), gen.cycle([3, 3, 3])), 0)]
    for g, lam in cases:
        if lam is None:
            lam = int(g.w.min())
        say("closed form", g.name)
        solve_check(ctx, g, lam)
        solve_check(ctx, g, lam, device_input=True)


def test_disconnected_side_is_component_of_zero(ctx):
    g = gen.disjoint_union(gen.cycle([2, 2, 2, 2]), gen.complete(3))
    lam, side = ctx.mincut(g)
    assert lam == 0 and list(side) == [0, 0, 0, 0, 1, 1, 1]


def _component_side(g):
    """side[v] = 1 iff v lies outside the component of vertex 0 (scipy)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    _, comp = connected_components(sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n)))
    return (comp != comp[0]).astype(np.uint8)


@pytest.mark.parametrize("case", ["two_large", "large_and_triangle", "isolated_vertex", "many_small"])
def test_disconnected_large_with_heuristic(ctx, case):
    # graphs above the heuristic's size threshold: connectivity is then
    # decided on the first coarse graph (or at once for a vertex of degree 0)
    big = gen.chung_lu(30000, 2.5, 12.0, 77, 1, 50, kcore=3, lcc=True)
    if case == "two_large":
        g = gen.disjoint_union(big, gen.erdos_renyi(12000, 10 / 11999, 78, 1, 50, lcc=True))
    elif case == "large_and_triangle":
        g = gen.disjoint_union(big, gen.complete(3, weight=5))
    elif case == "isolated_vertex":
        g = gen.disjoint_union(big, gen.complete(1))
    else:
        g = big
        for k in range(40):
            g = gen.disjoint_union(g, gen.cycle([1 + (k + i) % 7 for i in range(5 + k % 9)]))
    for seed in (3, 4):
        h = gen.permute(g, seed)[0]
        say("disconnected with heuristic", case, h.n, seed)
        assert h.n >= 10000
        ref = _component_side(h)
        for lam, side in (ctx.mincut(h), ctx.mincut(dev=ctx.upload(h))):
            assert lam == 0 and np.array_equal(side, ref)


@pytest.mark.parametrize("seed", range(120))
def test_random_small_vs_brute(ctx, seed):
    g = gen.random_small(2 + seed % 15, [0.3, 0.6, 0.95][seed % 3], 10000 + seed, 0, 9)
    lam_ref = oracle.brute(g)[0]
    solve_check(ctx, g, lam_ref)


def test_planted_two_blocks(ctx):
    g = gen.config_planted_2x1000()
    say("planted 2x1000")
    side = solve_check(ctx, g, 5)
    solve_check(ctx, g, 5, device_input=True)


@pytest.mark.parametrize("fam,seed", [(f, s) for f in range(3) for s in range(4)])
def test_mixed_medium_vs_oracle(ctx, fam, seed):
    n = [300, 1500, 5000, 12000][seed]
    g = gen.mixed_graph(n, 8 + 5 * seed, fam, 77 + seed, 1, 100)
    say("mixed", fam, seed, g.n, g.m)
    lam_ref = oracle.stoer_wagner(g)[0] if g.n <= 3000 else oracle.noi(g)[0]
    solve_check(ctx, g, lam_ref)


def test_unit_weight_chung_lu_core(ctx):
    g = gen.config_chung_lu(15)
    say("chung-lu 2^15 core", g.n, g.m)
    lam_ref = oracle.noi(g)[0]
    solve_check(ctx, g, lam_ref)


def test_bad_device_input_rejected(ctx):
    import torch
    import paper_2609_07204_amd as mc
    g = gen.complete(5)
    rp, col, w = ctx.upload(g)
    w2 = w.clone()
    w2[3] = -1
    with pytest.raises(mc.MincutError) as e:
        ctx.mincut(dev=(rp, col, w2))
    assert e.value.code == -2
    col2 = col.clone()
    col2[0] = 7
    with pytest.raises(mc.MincutError) as e:
        ctx.mincut(dev=(rp, col2, w))
    assert e.value.code == -2
    w3 = w.clone()
    w3[:] = 1 << 60
    with pytest.raises(mc.MincutError) as e:
        ctx.mincut(dev=(rp, col, w3))
    assert e.value.code == -3


@pytest.mark.parametrize("mode", [CF_PRIVATE, CF_LEVELS])
@pytest.mark.parametrize("name,mk", CF_GRAPHS)
def test_capforest_private_complete_pass_is_valid(ctx, name, mk, mode):
    # one private pass without a length cap scans every vertex once; its
    # recorded alpha is the capacity of its scanned prefix; contracting its
    # marks keeps lambda whenever the final bound is above lambda
    g = mk()
    say("capforest private complete", name, g.n)
    dev, dmin, _ = canon_dev(ctx, g)
    lam_true = oracle.stoer_wagner(g)[0]
    for start in (0, g.n // 2):
        res = ctx.step_capforest(dev, dmin, start=start, mode=mode, passes=1)
        order = res["order"]
        assert order.size == g.n and np.array_equal(np.sort(order), np.arange(g.n))
        assert order[0] == start
        if res["best_len"] > 0:
            side = np.zeros(g.n, np.uint8)
            side[order[:res["best_len"]]] = 1
            assert oracle.cut_value(g, side) == res["best_alpha"]
            assert res["lam"] == min(dmin, res["best_alpha"])
        thr = min(dmin, res["best_alpha"])
        if thr > lam_true:
            rp, col, w = oracle.contract(g, res["labels"], res["n2"])
            h = gen.Graph(res["n2"], rp, col, w)
            assert res["n2"] >= 2 and oracle.stoer_wagner(h)[0] == lam_true
        else:
            assert thr == lam_true


@pytest.mark.parametrize("mode", [CF_PRIVATE, CF_LEVELS])
def test_capforest_private_truncated_passes_valid(ctx, mode):
    g = gen.config_chung_lu(14)
    say("capforest private truncated", g.n)
    dev, dmin, _ = canon_dev(ctx, g)
    lam_true = oracle.noi(g)[0]
    res = ctx.step_capforest(dev, dmin, start=-1, mode=mode, passes=32, len_cap=300)
    assert res["n2"] < g.n  # the passes mark edges
    thr = min(dmin, res["best_alpha"])
    rp, col, w = oracle.contract(g, res["labels"], res["n2"])
    h = gen.Graph(res["n2"], rp, col, w)
    if thr > lam_true:
        assert oracle.noi(h)[0] == lam_true


@pytest.mark.parametrize("mode", ["shared", "deterministic", "levels"])
def test_solver_modes(ctx, mode):
    import paper_2609_07204_amd as mc
    c = mc.Context(0, capforest_mode=1 if mode == "shared" else 0, deterministic=1 if mode == "deterministic" else 0,
                   levels_min_n=2 if mode == "levels" else 0)
    for g in [gen.config_planted_2x1000(), gen.mixed_graph(3000, 12, 2, 5, 1, 100), gen.wheel(30)]:
        say("mode", mode, g.name)
        lam, side = c.mincut(g)
        lam_ref = oracle.stoer_wagner(g)[0]
        assert lam == lam_ref and oracle.cut_value(g, side) == lam
    c.close()


def hub_graph(n, hubs, hub_deg, d, seed, wlo=1, whi=100):
    """Random graph of mean degree d plus `hubs` vertices joined to hub_deg
    random others each: rows of at least 512 entries take the hub path of
    the level-synchronous CAPFOREST edge kernel."""
    r = np.random.default_rng(seed)
    base = gen.regular(n, d, seed, wlo, whi)
    rows = np.repeat(np.arange(n), np.diff(base.row_ptr))
    keep = rows < base.col
    u = list(rows[keep])
    v = list(base.col[keep])
    w = list(base.w[keep])
    for h in range(hubs):
        t = r.choice(n, size=hub_deg, replace=False)
        u += [h] * hub_deg
        v += list(t)
        w += list(r.integers(wlo, whi + 1, hub_deg))
    g = gen.from_edges(n, u, v, w, name="hubs(n=%d,h=%d,deg=%d,seed=%d)" % (n, hubs, hub_deg, seed))
    assert int(np.diff(g.row_ptr).max()) >= 512
    return g


@pytest.mark.parametrize("seed,wmax", [(1, 1), (2, 100), (3, 5)])
def test_capforest_levels_hub_pass_is_valid(ctx, seed, wmax):
    # complete pass through the whole-GPU form on a graph with hubs: scan
    # order is a permutation, the best alpha is its prefix's cut, and the
    # marked edges keep lambda whenever the bound stays above it
    g = hub_graph(3000, 4, 900, 6, seed, 1, wmax)
    say("capforest levels hubs", g.name)
    dev, dmin, _ = canon_dev(ctx, g)
    lam_true = oracle.noi(g)[0]
    for start in (0, 17, g.n - 1):
        res = ctx.step_capforest(dev, dmin, start=start, mode=CF_LEVELS, passes=1)
        order = res["order"]
        assert order.size == g.n and np.array_equal(np.sort(order), np.arange(g.n))
        assert order[0] == start
        if res["best_len"] > 0:
            side = np.zeros(g.n, np.uint8)
            side[order[:res["best_len"]]] = 1
            assert oracle.cut_value(g, side) == res["best_alpha"]
        thr = min(dmin, res["best_alpha"])
        assert res["n2"] < g.n
        if thr > lam_true:
            rp, col, w = oracle.contract(g, res["labels"], res["n2"])
            h = gen.Graph(res["n2"], rp, col, w)
            assert res["n2"] >= 2 and oracle.noi(h)[0] == lam_true
        else:
            assert thr == lam_true


@pytest.mark.parametrize("seed,wmax", [(4, 1), (5, 100), (6, 1000)])
def test_solver_levels_with_hubs(ctx, seed, wmax):
    import paper_2609_07204_amd as mc
    # whole-GPU steps down to graphs of 1000 vertices (smaller rounds run one
    # workgroup per pass). With unit weights (seed 4) the graph resists
    # contraction: the 20,000-vertex solve takes about 260 rounds, nearly all
    # with a complete fallback pass, about 35 s on one MI355X.
    c = mc.Context(0, levels_min_n=1000)
    for n, hubs in ((4000, 3), (20000, 12)):
        g = hub_graph(n, hubs, 1500, 6, seed, 1, wmax)
        say("levels solve with hubs", g.name)
        lam, side = c.mincut(g)
        assert lam == oracle.noi(g)[0] and oracle.cut_value(g, side) == lam
    c.close()


def test_capforest_step_graphs_match_eager_steps():
    # whole-GPU CAPFOREST steps replayed from captured HIP graphs (timing
    # off) and launched one by one (timing on): several solves in a row,
    # each with several replays per round, all equal to the oracle
    import paper_2609_07204_amd as mc
    c = mc.Context(0, levels_min_n=1000)
    graphs = [gen.chung_lu(1 << 14, 2.5, 12.0, 21, 1, 20, kcore=3, lcc=True),
              gen.mixed_graph(6000, 12, 1, 8, 1, 100), hub_graph(4000, 3, 1500, 6, 7, 1, 50)]
    for rep in range(2):
        for g in graphs:
            ref = oracle.noi(g)[0]
            c.profile(True)
            lam_e, side_e, st_e = c.mincut(g, return_stats=True)
            c.profile(False)
            lam_g, side_g, st_g = c.mincut(g, return_stats=True)
            say("step graphs", g.name, rep, lam_g, st_e["rounds"], st_g["rounds"])
            assert lam_e == lam_g == ref
            assert oracle.cut_value(g, side_e) == ref and oracle.cut_value(g, side_g) == ref
    c.close()


@pytest.mark.parametrize("log2n,seed", [(16, 3), (17, 5)])
def test_solver_levels_chung_lu_hubs(ctx, log2n, seed):
    # power-law graphs whose hubs (rows of 512 entries or more) take the
    # hub path of the whole-GPU CAPFOREST steps in the first rounds
    import paper_2609_07204_amd as mc
    g = gen.chung_lu(1 << log2n, 2.5, 20, seed, kcore=10)
    assert int(np.diff(g.row_ptr).max()) >= 512
    say("levels solve chung-lu", g.name, g.n, g.m)
    c = mc.Context(0, levels_min_n=16384)
    lam, side, st = c.mincut(g, return_stats=True)
    say("  lambda", lam, "rounds", st["rounds"], "fallback", st["fallback_passes"])
    assert lam == oracle.noi(g)[0] and oracle.cut_value(g, side) == lam
    c.close()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_raw_input_takes_merging_normalisation(ctx, seed):
    # loops, parallel entries, zero weights and unsorted rows go through the
    # merging normalisation; the same graph in normal form is used in place;
    # both give the oracle's lambda
    r = np.random.default_rng(seed)
    n, m = 600, 4000
    u = r.integers(0, n, m)
    v = r.integers(0, n, m)
    w = r.integers(0, 6, m)
    u = np.concatenate([u, np.arange(n), (np.arange(n) + 1) % n])   # a cycle keeps it connected
    v = np.concatenate([v, np.arange(n), np.arange(n)])
    w = np.concatenate([w, np.full(n, 3), np.full(n, 1)])
    raw = gen.raw_csr(n, u, v, w)
    pos = w > 0
    norm = gen.from_edges(n, u[pos], v[pos], w[pos])
    lam_ref = oracle.noi(norm)[0]
    lam1, side1, st1 = ctx.mincut(raw, return_stats=True)
    lam2, side2, st2 = ctx.mincut(norm, return_stats=True)
    say("raw vs normal", seed, lam_ref, st1["input_normal"], st2["input_normal"])
    assert st1["input_normal"] == 0 and st2["input_normal"] == 1
    assert lam1 == lam2 == lam_ref
    assert oracle.cut_value(norm, side1) == lam_ref and oracle.cut_value(norm, side2) == lam_ref


# ------------------------------------------------------ label propagation
@pytest.mark.parametrize("seed,nlab", [(1, 0), (2, 5), (3, 40), (4, 3000)])
def test_lp_round_matches_oracle(ctx, seed, nlab):
    # rows of up to ~2000 entries (hubs take the long-row path), labels from
    # singletons (nlab = 0) to a few large clusters: bit-exact
    g = hub_graph(3000, 5, 1800, 6, seed, 1, 9)
    r = np.random.default_rng(seed)
    lab = np.arange(g.n, dtype=np.int32) if nlab == 0 else r.integers(0, nlab, g.n).astype(np.int32)
    dev = ctx.dgraph(g)
    got = ctx.step_lp(dev, lab)
    want = oracle.lp_round(g, lab)
    say("lp round", seed, nlab, int(np.sum(got != lab)), "changed")
    assert np.array_equal(got, want)
    # a second round from the first round's labels
    assert np.array_equal(ctx.step_lp(dev, want), oracle.lp_round(g, want))


@pytest.mark.parametrize("seed,whi", [(11, 1), (12, 3), (13, 1000)])
def test_lp_first_round_from_singletons_matches_oracle(ctx, seed, whi):
    # the heuristic's first round (singleton labels, normal graph) takes its
    # own streaming kernels; it must equal the general rule bit for bit:
    # rows of up to 1800 entries (listed long rows), many equal weights,
    # and vertices with no edge at all (they keep their own label)
    g = hub_graph(3000, 5, 1800, 6, seed, 1, whi)
    rp, col, w = g.row_ptr, g.col, g.w
    n = g.n + 7      # seven isolated vertices at the end
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    keep = rows < col
    h = gen.from_edges(n, rows[keep], col[keep], w[keep])
    dev = ctx.dgraph(h)
    got = ctx.step_lp(dev, None)
    want = oracle.lp_round(h, np.arange(h.n, dtype=np.int32))
    say("lp first round", seed, whi, int(np.sum(got != np.arange(h.n))), "moved")
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed,nlab", [(5, 3), (6, 60), (7, 0)])
def test_lp_round_all_row_classes_match_oracle(ctx, seed, nlab):
    # a power-law graph with rows of every length class (register rows up
    # to 128 entries, LDS-table rows up to 512, long rows beyond), weights
    # 1..3 so that label weights tie often; bit-exact
    g = gen.chung_lu(20000, 2.1, 24, seed, 1, 3, kcore=0, lcc=False)
    d = np.diff(g.row_ptr)
    say("lp rows", seed, nlab, "max row", int(d.max()), "rows >128:", int((d > 128).sum()), ">512:", int((d > 512).sum()))
    assert d.max() > 512 and ((d > 128) & (d <= 512)).sum() > 0
    r = np.random.default_rng(seed)
    lab = np.arange(g.n, dtype=np.int32) if nlab == 0 else r.integers(0, nlab, g.n).astype(np.int32)
    dev = ctx.dgraph(g)
    want = oracle.lp_round(g, lab)
    assert np.array_equal(ctx.step_lp(dev, lab), want)
    assert np.array_equal(ctx.step_lp(dev, want), oracle.lp_round(g, want))


@pytest.mark.parametrize("seed,wlo,whi,hubs", [(21, 1 << 29, (1 << 29) + 2, 0), (22, 1 << 30, 1 << 33, 5),
                                               (23, (1 << 32) - 3, (1 << 32) - 1, 0)])
def test_lp_round_label_sums_near_32_bits(ctx, seed, wlo, whi, hubs):
    # short rows keep their per-label sums in 32 bits when every row's
    # weight sum is below 2^32 and in 64 bits otherwise: row sums just
    # below 2^32 (sums past 2^31, three weights so that sums tie), row sums
    # far above it with hub rows, and single weights just below 2^32
    if hubs:
        g = hub_graph(3000, hubs, 1800, 6, seed, wlo, whi)
    else:
        g = gen.regular(3000, 6 if wlo < (1 << 30) else 1, seed, wlo, whi)
    rs = np.add.reduceat(g.w.astype(object), g.row_ptr[:-1]) if len(g.w) else []
    narrow = max(rs) < (1 << 32)
    say("lp sums", seed, "max row sum", max(rs), "narrow" if narrow else "wide")
    assert narrow == (hubs == 0)
    r = np.random.default_rng(seed)
    dev = ctx.dgraph(g)
    for lab in (np.arange(g.n, dtype=np.int32), r.integers(0, 7, g.n).astype(np.int32),
                r.integers(0, 400, g.n).astype(np.int32)):
        want = oracle.lp_round(g, lab)
        assert np.array_equal(ctx.step_lp(dev, lab), want)


@pytest.mark.parametrize("seed,nlab", [(31, 3), (32, 60), (33, 0)])
def test_lp_round_general_kernel_all_row_classes(ctx, seed, nlab):
    # weights so large that row sums pass 2^32: the general LP kernel (64-bit
    # keys and sums) takes every row, with rows of every length class (chunks
    # of many short rows, chunks of a few rows cut into pieces, long rows);
    # few distinct weights, so that label sums tie; bit-exact
    g = gen.chung_lu(20000, 2.1, 24, seed, 1 << 30, (1 << 30) + 2, kcore=0, lcc=False)
    d = np.diff(g.row_ptr)
    rs = np.add.reduceat(g.w.astype(object), g.row_ptr[:-1])
    assert max(rs) >= (1 << 32) and d.max() > 256 and ((d > 32) & (d <= 256)).sum() > 0
    r = np.random.default_rng(seed)
    lab = np.arange(g.n, dtype=np.int32) if nlab == 0 else r.integers(0, nlab, g.n).astype(np.int32)
    dev = ctx.dgraph(g)
    want = oracle.lp_round(g, lab)
    assert np.array_equal(ctx.step_lp(dev, lab), want)
    assert np.array_equal(ctx.step_lp(dev, want), oracle.lp_round(g, want))


def test_lp_round_ties_and_own_label(ctx):
    # star-like rows with equal weights: ties go to the smallest label, and a
    # vertex keeps its label unless another is strictly heavier
    n = 40
    u, v, w = [], [], []
    for k in range(1, n):
        u.append(0); v.append(k); w.append(1)
    for k in range(1, n - 1):
        u.append(k); v.append(k + 1); w.append(1)
    g = gen.from_edges(n, u, v, w)
    for lab in (np.arange(n, dtype=np.int32), (np.arange(n) % 3).astype(np.int32),
                np.array([7] + [3] * 19 + [5] * 20, np.int32)):
        dev = ctx.dgraph(g)
        assert np.array_equal(ctx.step_lp(dev, lab), oracle.lp_round(g, lab))


@pytest.mark.parametrize("fam,seed", [(0, 1), (1, 2), (2, 3), (2, 4)])
def test_heuristic_solve_matches_oracle(ctx, fam, seed):
    # graphs above the heuristic threshold: the label-propagation bound is a
    # real cut (lambda <= bound <= min degree) and the exact rounds that
    # follow still reach lambda
    import paper_2609_07204_amd as mc
    g = gen.mixed_graph(30000, 10 + 4 * seed, fam, 500 + seed, 1, 100)
    lam_ref = oracle.noi(g)[0]
    c = mc.Context(0, heuristic_min_n=10000)
    lam, side, st = c.mincut(g, return_stats=True)
    say("heuristic", g.name, g.n, g.m, "levels", st["heuristic_levels"], "bound", st["lambda_heuristic"],
        "lambda", lam_ref, "min degree", st["lambda_min_degree"])
    assert lam == lam_ref and oracle.cut_value(g, side) == lam
    assert st["heuristic_levels"] >= 1
    assert lam_ref <= st["lambda_heuristic"] <= st["lambda_min_degree"]
    c.close()


# ------------------------------------------------- reduction tests 3 and 4
def tri_graph(seed, n=2000):
    """Clustered weighted graph: dense random blocks of 4..12 vertices joined
    by light edges, so many short rows share neighbours (tests 3 and 4
    fire), plus a few long rows."""
    r = np.random.default_rng(seed)
    u, v, w = [], [], []
    start = 0
    blocks = []
    while start < n:
        b = int(r.integers(4, 13))
        b = min(b, n - start)
        blocks.append((start, start + b))
        for i in range(start, start + b):
            for j in range(i + 1, start + b):
                if r.random() < 0.7:
                    u.append(i); v.append(j); w.append(int(r.integers(1, 20)))
        start += b
    for _ in range(n):
        u.append(int(r.integers(0, n))); v.append(int(r.integers(0, n))); w.append(int(r.integers(1, 4)))
    for i in range(n):   # a ring keeps it connected
        u.append(i); v.append((i + 1) % n); w.append(3)
    for h in range(3):
        t = r.choice(n, size=200, replace=False)
        u += [h] * 200; v += list(t); w += [1] * 200
    return gen.from_edges(n, u, v, w, name="tri(seed=%d)" % seed)


@pytest.mark.parametrize("seed,D", [(1, 16), (2, 8), (3, 64), (4, 24)])
def test_pr34_matches_oracle(ctx, seed, D):
    g = tri_graph(seed)
    dev, dmin, _ = canon_dev(ctx, g)
    for lam in (dmin, max(1, dmin // 2), 10 ** 9):
        _, ptr = oracle.pr12(g, lam)
        flag_t, acc, lab, n2 = ctx.step_pr34(dev, lam, D, ptr)
        f4, part, acc_ref = oracle.pr34(g, lam, D, ptr)
        # entries of the canonical device graph are the host graph's rows
        # in some order: compare per (row, target)
        off = dev.off[:g.n].cpu().numpy().astype(np.int64)
        ln = dev.len[:g.n].cpu().numpy().astype(np.int64)
        flag = flag_t.cpu().numpy()
        col_dev = dev.col.cpu().numpy()
        got = {(x, int(col_dev[j])) for x in range(g.n) for j in range(off[x], off[x] + ln[x]) if flag[j]}
        want = {(x, int(g.col[j])) for x in range(g.n) for j in range(g.row_ptr[x], g.row_ptr[x + 1]) if f4[j]}
        say("pr34", seed, D, lam, len(want), "test-4 entries", int((acc_ref >= 0).sum()), "matched")
        assert got == want
        assert np.array_equal(acc, acc_ref)
        pairs = [(a, b) for a, b in want] + [(v, int(acc_ref[v])) for v in range(g.n) if acc_ref[v] >= 0]
        a = np.array([p[0] for p in pairs], np.int32)
        b = np.array([p[1] for p in pairs], np.int32)
        lab_ref, nc = oracle.components(g.n, a, b)
        assert n2 == nc and np.array_equal(lab, lab_ref)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_solver_with_tests34_matches_oracle(ctx, seed):
    import paper_2609_07204_amd as mc
    g = tri_graph(seed, 6000)
    lam_ref = oracle.noi(g)[0]
    for D in (0, 16, 64):
        c = mc.Context(0, pr_tri_deg_cap=D)
        lam, side, st = c.mincut(g, return_stats=True)
        say("solve tri", seed, D, lam_ref, "tests 3/4 marks", st["marks_tri"])
        assert lam == lam_ref and oracle.cut_value(g, side) == lam
        if D == 0:
            assert st["marks_tri"] == 0
        c.close()


# ------------------------------------------------------------ batched form
def batch_mix(seed, count, nmax=3000):
    r = np.random.default_rng(seed)
    gs = []
    for i in range(count):
        kind = i % 7
        if kind == 0:
            gs.append(gen.random_small(int(r.integers(2, 16)), 0.5, seed * 1000 + i, 0, 9))
        elif kind == 1:
            gs.append(gen.complete(int(r.integers(2, 9))))
        elif kind == 2:
            n = int(r.integers(3, 30))
            gs.append(gen.cycle([int(x) for x in r.integers(1, 9, n)]))
        elif kind == 3:
            a, b = gen.complete(int(r.integers(2, 6))), gen.cycle([1, 2, 3])
            gs.append(gen.disjoint_union(a, b))            # disconnected: lambda 0
        elif kind == 4:
            n = int(r.integers(50, nmax))
            gs.append(gen.mixed_graph(n, int(r.integers(6, 20)), int(r.integers(0, 3)), seed * 1000 + i, 1, 100))
        elif kind == 5:
            n = int(r.integers(10, 200))
            m = 4 * n
            u = r.integers(0, n, m); v = r.integers(0, n, m); w = r.integers(0, 5, m)
            u = np.concatenate([u, np.arange(n)]); v = np.concatenate([v, (np.arange(n) + 1) % n])
            w = np.concatenate([w, np.ones(n, np.int64)])
            gs.append(gen.raw_csr(n, u, v, w))          # loops, parallel entries, zero weights
        else:
            gs.append(gen.wheel(int(r.integers(4, 40))))
    return gs


def oracle_lambda(g):
    return oracle.stoer_wagner(g)[0] if g.n <= 400 else oracle.noi(g)[0]


@pytest.mark.parametrize("seed,count", [(1, 40), (2, 200), (3, 700)])
def test_batch_matches_oracle(ctx, seed, count):
    import torch
    gs = batch_mix(seed, count)
    # a workspace full of stale bytes: nothing may rely on fresh memory
    ws = torch.full((ctx.batch_workspace_bytes(gs),), 0xA5, dtype=torch.uint8, device=ctx.device)
    lams, sides = ctx.mincut_batch(gs, workspace=ws)
    bad = []
    for i, g in enumerate(gs):
        ref = oracle_lambda(g)
        if lams[i] != ref or oracle.cut_value(g, sides[i]) != ref or sides[i][0] != 0:
            bad.append((i, g.name, int(lams[i]), int(ref)))
    say("batch", seed, count, "graphs,", sum(g.nnz for g in gs), "entries; mismatches", bad[:5])
    assert not bad


@pytest.mark.parametrize("threads,lp", [(64, 2), (128, 1), (512, 2), (1024, 1)])
def test_batch_pass_sizes_match_oracle(ctx, threads, lp):
    # every pass workgroup size the autotuner may pick, with and without
    # the admission bound, gives the oracle's lambdas and valid sides
    gs = batch_mix(20 + threads, 150)
    ctx.set_options(batch_pass_threads=threads, batch_lp=lp)
    try:
        lams, sides = ctx.mincut_batch(gs)
    finally:
        ctx.set_options(batch_pass_threads=0, batch_lp=0, finish_max_n=0, queue=0)
    bad = [(i, gs[i].name) for i, g in enumerate(gs)
           if lams[i] != oracle_lambda(g) or oracle.cut_value(g, sides[i]) != lams[i] or sides[i][0] != 0]
    assert not bad, bad[:5]


def test_batch_autotune_picks_a_setting_and_keeps_results(ctx):
    import paper_2609_07204_amd as mc
    gs = batch_mix(31, 200)
    t = ctx.batch_autotune(gs, sample=80)
    say("autotune", t["pass_threads"], t["lp"], t["finish_max_n"], t["queue"],
        [round(c["ms"], 2) for c in t["candidates"]])
    # 10 pass settings, 3 finisher limits, and the 2 other queues unless the
    # finisher lost
    assert t["sample"] == 80 and len(t["candidates"]) in (13, 15)
    assert t["pass_threads"] in (64, 128, 256, 512, 1024) and t["lp"] in (1, 2)
    assert t["finish_max_n"] in (0, 512, 256, -1) and t["queue"] in (0, 1, 2)
    assert all(c["ms"] > 0 for c in t["candidates"])
    best = min(t["candidates"], key=lambda c: c["ms"])
    assert (best["pass_threads"], best["lp"], best["finish_max_n"], best["queue"]) == \
        (t["pass_threads"], t["lp"], t["finish_max_n"], t["queue"])
    try:
        lams, sides = ctx.mincut_batch(gs)
        assert all(lams[i] == oracle_lambda(g) and oracle.cut_value(g, sides[i]) == lams[i] for i, g in enumerate(gs))
        with pytest.raises(mc.MincutError):
            ctx.set_options(batch_pass_threads=100)
    finally:
        ctx.set_options(batch_pass_threads=0, batch_lp=0, finish_max_n=0, queue=0)


def test_batch_device_input_same_as_host(ctx):
    gs = batch_mix(9, 120)
    devs = [ctx.upload(g) for g in gs]
    lam_h, _ = ctx.mincut_batch(gs, want_sides=False)
    lam_d, sides = ctx.mincut_batch(devs=devs)
    assert np.array_equal(lam_h, lam_d)
    for i, g in enumerate(gs):
        assert oracle.cut_value(g, sides[i]) == lam_d[i]


def test_batch_same_as_alone(ctx):
    # each result in the batch equals the graph's result alone
    gs = [gen.config_batch_graph(i) for i in range(0, 64)]
    lams, sides = ctx.mincut_batch(gs)
    for i, g in enumerate(gs):
        lam1, _ = ctx.mincut(g, want_side=False)
        assert lams[i] == lam1
        assert oracle.cut_value(g, sides[i]) == lam1


def test_batch_rejects_bad_graphs(ctx):
    import paper_2609_07204_amd as mc
    g = gen.complete(5)
    bad = gen.Graph(5, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    bad.col[3] = 9
    with pytest.raises(mc.MincutError) as e:
        ctx.mincut_batch([g, bad])
    assert e.value.code == -2
    devs = [ctx.upload(g), ctx.upload(bad)]
    with pytest.raises(mc.MincutError) as e:
        ctx.mincut_batch(devs=devs)
    assert e.value.code == -2


# ------------------------------------------------------------ served form
@pytest.mark.parametrize("solo_min_n", [0, 2000])
def test_server_results_same_alone_and_in_the_mix(ctx, solo_min_n):
    # requests submitted while others are in flight join their rounds (or,
    # from solo_min_n vertices on, are solved on their own between rounds);
    # every result equals the graph's result alone (and the oracle's)
    import paper_2609_07204_amd as mc
    srv = mc.Server(ctx, hbm_bytes=2 << 30, max_inflight=64, max_request_n=1 << 16, max_request_nnz=1 << 21,
                    solo_min_n=solo_min_n)
    say("server capacity", srv.capacity())
    gs = batch_mix(21, 90) + [gen.config_batch_graph(i) for i in range(8)]
    tickets = {}
    results = {}
    pending = list(range(len(gs)))
    steps = 0
    while pending or len(results) < len(gs):
        # a few arrivals per step, so later graphs join rounds in progress
        for _ in range(3):
            if pending:
                i = pending.pop(0)
                tickets[srv.submit(gs[i])] = i
        srv.step()
        steps += 1
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                results[tickets.pop(t)] = r
        assert steps < 10000
    say("served", len(gs), "graphs in", steps, "steps")
    joined_late = 0
    for i, g in enumerate(gs):
        lam, side, st = results[i]
        alone, _ = ctx.mincut(g, want_side=False)
        assert lam == alone == oracle_lambda(g), (i, g.name)
        assert oracle.cut_value(g, side) == lam and side[0] == 0
        assert st["t_submit_ms"] <= st["t_admit_ms"] <= st["t_done_ms"]
        joined_late += st["rounds"] > 0
    assert joined_late > 0
    if solo_min_n:
        assert any(results[i][2]["rounds"] == 0 for i, g in enumerate(gs) if g.n >= solo_min_n)
    srv.close()


def test_server_admits_by_memory_and_cancels(ctx):
    import paper_2609_07204_amd as mc
    srv = mc.Server(ctx, hbm_bytes=256 << 20, max_inflight=8, max_request_n=1 << 14, max_request_nnz=1 << 18)
    cap = srv.capacity()
    g_big = gen.mixed_graph(12000, 16, 2, 5, 1, 100)
    with pytest.raises(mc.MincutError):
        srv.submit(gen.mixed_graph(40000, 8, 1, 6, 1, 100))    # larger than any admission
    ts = [srv.submit(g_big) for _ in range(6)]
    t_small = srv.submit(gen.complete(6))
    srv.cancel(ts[-1])
    done = {}
    for _ in range(5000):
        a, q = srv.step()
        for t in ts[:-1] + [t_small]:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        if len(done) == len(ts):
            break
    assert len(done) == len(ts)
    ref = oracle.noi(g_big)[0]
    assert all(done[t][0] == ref for t in ts[:-1]) and done[t_small][0] == 5
    with pytest.raises(mc.MincutError) as e:
        srv.poll(ts[-1])
    assert e.value.code == -7
    say("server capacity", cap)
    srv.close()


@pytest.mark.parametrize("fill", [0x00, 0xA5, 0xFF])
def test_single_solve_ignores_stale_workspace(ctx, fill):
    import torch
    for g in (gen.config_planted_2x1000(), gen.mixed_graph(20000, 12, 2, 7, 1, 100), gen.wheel(50)):
        ws = torch.full((ctx.workspace_bytes(g.n, g.nnz),), fill, dtype=torch.uint8, device=ctx.device)
        lam, side = ctx.mincut(g, workspace=ws)
        ref = oracle_lambda(g)
        assert lam == ref and oracle.cut_value(g, side) == ref


# ------------------------------------------------ the configurations at full size
GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lambda.json")))


@pytest.mark.parametrize("name,make", [
    ("chung_lu_2^22_core10_seed1", lambda: gen.config_chung_lu(22, 1)),
    ("rhg_2^23_core32_seed1", lambda: gen.config_rhg(23, 1)),
])
def test_full_size_config_matches_oracle(ctx, name, make):
    # the workload solved at its real size, input resident on the device as
    # the benchmark times it, with the bound heuristic on (default) and off:
    # lambda equals the oracle's stored value, the side recomputes to it
    ref = GOLDEN[name]
    t = time.time()
    g = make()
    say("full size", name, g.n, g.m, "generated in %.1fs" % (time.time() - t))
    assert (g.n, g.m) == (ref["n"], ref["m"])
    dev = ctx.upload(g)
    try:
        for hmin in (10000, 0):
            ctx.set_options(heuristic_min_n=hmin)
            lam, side = ctx.mincut(dev=dev)
            say("  heuristic_min_n", hmin, "lambda", lam)
            assert lam == ref["lambda"]
            assert side[0] == 0 and 0 < int(side.sum()) < g.n
            assert oracle.cut_value(g, side) == lam
    finally:
        ctx.set_options(heuristic_min_n=10000)


def test_batch_full_config_matches_oracle(ctx):
    # all 4096 graphs of the batched configuration in one call; every lambda
    # against the oracle (run on host threads: the oracle releases the
    # interpreter lock), every side recomputed
    gen._L()
    oracle._L()     # load both libraries before the threads use them
    t = time.time()
    with ThreadPoolExecutor(16) as ex:
        gs = list(ex.map(gen.config_batch_graph, range(4096)))
    say("batch config: %d graphs, %d entries, generated in %.1fs" % (len(gs), sum(g.nnz for g in gs), time.time() - t))
    t = time.time()
    lams, sides = ctx.mincut_batch(gs)
    say("  solved in %.1fs (host input, sides)" % (time.time() - t))
    t = time.time()
    with ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(lambda g: oracle.noi(g)[0], gs))
        cuts = list(ex.map(lambda a: oracle.cut_value(a[0], a[1]), zip(gs, sides)))
    say("  oracle in %.1fs" % (time.time() - t))
    bad = [(i, gs[i].name, int(lams[i]), refs[i], cuts[i]) for i in range(len(gs))
           if lams[i] != refs[i] or cuts[i] != refs[i] or sides[i][0] != 0]
    assert not bad, bad[:5]


def test_round_timing_records_the_solve(ctx):
    # per-round records of a profiled solve: heuristic levels first, then
    # the exact rounds; sizes shrink, the first round starts from the input
    g = gen.config_chung_lu(16)
    ctx.profile(True)
    try:
        lam, _ = ctx.mincut(g)
        rounds = ctx.profile_rounds()
    finally:
        ctx.profile(False)
    say("rounds", [(r["kind"], r["n_in"], r["m_in"], r["n_out"], round(r["ms"], 3)) for r in rounds])
    assert lam == oracle.noi(g)[0]
    assert rounds and all(r["ms"] > 0 for r in rounds)
    assert rounds[0]["n_in"] == g.n and rounds[0]["m_in"] == g.nnz
    kinds = [r["kind"] for r in rounds]
    assert kinds == sorted(kinds, key=lambda k: {"level": 0, "coarse": 1, "exact": 2}[k])
    for r in rounds:
        assert r["n_out"] <= r["n_in"] and r["m_out"] <= r["m_in"]
    ex = [r for r in rounds if r["kind"] == "exact"]
    assert ex and ex[0]["n_in"] == g.n
    for a, b in zip(ex, ex[1:]):
        assert b["n_in"] == a["n_out"] and b["m_in"] == a["m_out"]

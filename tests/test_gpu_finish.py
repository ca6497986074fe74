"""GPU tests of the small-graph finisher: all remaining rounds of Algorithm 2
in one launch (one workgroup per graph), and its CAPFOREST pass with the
priority queue in LDS (Section 2.1 "Bounded priority queues"):
 - the heap pass (largest key, then smallest id) is bit-exact against the
   oracle's sequential pass: scan order, marks (canonical labels), bound and
   best alpha with its prefix;
 - the bucket pass (LIFO buckets, so another valid order) scans every
   vertex, its best alpha is the cut of its prefix, and its marks keep lambda
   whenever the bound stays above it;
 - whole solves through the finisher (each queue) equal the oracle and the
   solves without it, with sides that recompute to lambda."""
import numpy as np
import pytest

import gen
import oracle
from test_gpu_parity import canon_dev, cf_oracle, check_cf_equal, hub_graph, say

pytestmark = pytest.mark.gpu

CF_BUCKET, CF_HEAP = 4, 5

SMALL_GRAPHS = [
    ("planted", lambda: gen.planted(300, 300, 8, 3, 1, 10, 5)),
    ("er", lambda: gen.erdos_renyi(800, 10 / 799, 3, 1, 100, lcc=True)),
    ("chung_lu", lambda: gen.chung_lu(1000, 2.5, 10.0, 4, 1, 1, kcore=3, lcc=True)),
    ("wheel", lambda: gen.wheel(200)),
    ("cliques", lambda: gen.two_cliques(30, 40, 5)),
    ("cycle", lambda: gen.cycle([1 + (i * 7919) % 97 for i in range(500)])),
    ("heavy", lambda: gen.erdos_renyi(600, 12 / 599, 9, 1000, 100000, lcc=True)),
    ("hubs", lambda: hub_graph(1000, 3, 600, 6, 2, 1, 5)),
]


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2609_07204_amd as mc
    assert torch.cuda.is_available()
    c = mc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,mk", SMALL_GRAPHS)
def test_lds_heap_pass_matches_oracle(ctx, name, mk):
    g = mk()
    assert g.n <= 1024
    say("lds heap pass", name, g.n)
    dev, dmin, _ = canon_dev(ctx, g)
    for start in (0, g.n // 2, g.n - 1):
        for lam in (dmin, max(1, dmin // 2), dmin * 3):
            res = ctx.step_capforest(dev, lam, start=start, mode=CF_HEAP)
            check_cf_equal(res, cf_oracle(g, lam, start))


@pytest.mark.parametrize("name,mk", SMALL_GRAPHS)
def test_lds_bucket_pass_is_valid(ctx, name, mk):
    g = mk()
    say("lds bucket pass", name, g.n)
    dev, dmin, _ = canon_dev(ctx, g)
    lam_true = oracle.stoer_wagner(g)[0]
    for start in (0, g.n // 3):
        for lam in (dmin, dmin * 2):
            res = ctx.step_capforest(dev, lam, start=start, mode=CF_BUCKET)
            order = res["order"]
            assert order.size == g.n and np.array_equal(np.sort(order), np.arange(g.n))
            assert order[0] == start
            if res["best_len"] > 0:
                side = np.zeros(g.n, np.uint8)
                side[order[:res["best_len"]]] = 1
                assert oracle.cut_value(g, side) == res["best_alpha"]
                assert res["lam"] == min(lam, res["best_alpha"])
            thr = res["lam"]
            if thr > lam_true:
                rp, col, w = oracle.contract(g, res["labels"], res["n2"])
                h = gen.Graph(res["n2"], rp, col, w)
                assert res["n2"] >= 2 and oracle.stoer_wagner(h)[0] == lam_true
            else:
                assert thr == lam_true
            if thr == lam:
                assert res["n2"] < g.n   # a complete pass at a fixed bound marks an edge


@pytest.mark.parametrize("queue", [0, 1, 2])
def test_finisher_solves_match_oracle(ctx, queue):
    import paper_2609_07204_amd as mc
    on = mc.Context(0, queue=queue)
    off = mc.Context(0, finish_max_n=-1)
    graphs = [mk() for _, mk in SMALL_GRAPHS]
    graphs += [gen.random_small(n, 0.5, 300 + n, 1, 9) for n in (3, 5, 8, 13, 19)]
    graphs += [gen.mixed_graph(900, 10, f, 40 + f, 1, 100) for f in range(3)]
    for g in graphs:
        ref = oracle.stoer_wagner(g)[0] if g.n <= 1200 else oracle.noi(g)[0]
        lam, side, st = on.mincut(g, return_stats=True)
        assert lam == ref, (g.name, lam, ref)
        assert side[0] == 0 and 0 < int(side.sum()) < g.n and oracle.cut_value(g, side) == lam
        if g.n > 2 and ref > 0:
            assert st["finish_rounds"] == st["rounds"] >= 1
        lam2, _ = off.mincut(g, want_side=False)
        assert lam2 == lam
    on.close()
    off.close()


def test_finisher_takes_over_after_large_rounds(ctx):
    # graphs larger than the finisher shrink by host-driven rounds, then the
    # finisher completes them; results equal the solves without it
    import paper_2609_07204_amd as mc
    off = mc.Context(0, finish_max_n=-1)
    for g in [gen.config_planted_2x1000(), gen.mixed_graph(20000, 12, 2, 5, 1, 100),
              gen.mixed_graph(5000, 16, 1, 6, 1, 1000), hub_graph(4000, 3, 1500, 6, 4, 1, 1)]:
        ref = oracle.noi(g)[0]
        lam, side, st = ctx.mincut(g, return_stats=True)
        say("finisher after rounds", g.name, "rounds", st["rounds"], "in finisher", st["finish_rounds"])
        assert lam == ref and oracle.cut_value(g, side) == lam
        assert off.mincut(g, want_side=False)[0] == ref
    off.close()


def test_deterministic_solves_repeat_exactly(ctx):
    import paper_2609_07204_amd as mc
    c = mc.Context(0, deterministic=1)
    for g in [gen.mixed_graph(700, 12, 2, 9, 1, 100), gen.wheel(60), gen.config_planted_2x1000()]:
        lam1, side1 = c.mincut(g)
        lam2, side2 = c.mincut(g)
        assert lam1 == lam2 == oracle.stoer_wagner(g)[0]
        assert np.array_equal(side1, side2)
    c.close()

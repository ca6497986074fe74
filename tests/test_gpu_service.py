"""GPU tests of the batched and served forms at the served workload's sizes
and of their error handling: graphs of the served pool (up to 1.7 M
vertices, 9.5 M edges, weights 1-1000) through the server alone, in a mix
and against the plain solve and the oracle's lambda (tests/golden); per-
graph statuses of the batched call; malformed, cancelled and late requests.
Integer results, so the bar is equality; sides must recompute to lambda."""
import ctypes
import json
import os
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lambda.json")))
POOL = [13, 145, 178, 66, 22, 248, 150, 147, 226, 131, 211, 104]


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
def pool():
    return {j: gen.config_served_graph(j) for j in POOL}


def run_server(srv, gs, per_step=1, max_steps=200000):
    """Submit gs (a list of (key, graph)) per_step at a time, one step after
    each group of arrivals, until every result is in. Returns key -> result."""
    tickets, results = {}, {}
    pending = list(gs)
    steps = 0
    while pending or tickets:
        for _ in range(per_step):
            if pending:
                key, g = pending.pop(0)
                tickets[srv.submit(g)] = key
        srv.step()
        steps += 1
        for t in list(tickets):
            r = srv.poll(t)
            if r is not None:
                results[tickets.pop(t)] = r
        assert steps < max_steps
    return results


@pytest.mark.timeout(600)
def test_served_pool_alone_in_mix_and_plain(ctx, pool):
    # default solo_min_n (65536): graphs with n >= 65536 run on solo slots
    # while the others go through the engine's rounds
    import paper_2609_07204_amd as mc
    maxn = max(g.n for g in pool.values())
    maxe = max(g.nnz for g in pool.values())
    srv = mc.Server(ctx, hbm_bytes=32 << 30, max_inflight=256, max_request_n=maxn, max_request_nnz=maxe,
                    solo_slots=2)
    say("server capacity", srv.capacity())
    mix = run_server(srv, [(j, pool[j]) for j in POOL], per_step=2)
    alone = {}
    for j in POOL:
        alone[j] = run_server(srv, [(j, pool[j])])[j]
    for j in POOL:
        g = pool[j]
        ref = GOLDEN["served_pool_%d" % j]
        assert (g.n, g.m) == (ref["n"], ref["m"])
        lam_plain, side_plain = ctx.mincut(g)
        for tag, (lam, side, st) in (("mix", mix[j]), ("alone", alone[j])):
            assert lam == ref["lambda"], (j, tag, lam, ref["lambda"])
            assert side[0] == 0 and 0 < int(side.sum()) < g.n
            assert oracle.cut_value(g, side) == lam, (j, tag)
            assert st["t_submit_ms"] <= st["t_admit_ms"] <= st["t_done_ms"]
            if g.n >= 65536:
                assert st["rounds"] == 0   # solved on a solo slot
        assert lam_plain == ref["lambda"] and oracle.cut_value(g, side_plain) == lam_plain
        say("pool", j, "n", g.n, "m", g.m, "lambda", ref["lambda"], "mix ms",
            round(mix[j][2]["t_done_ms"] - mix[j][2]["t_submit_ms"], 1))
    srv.close()


def test_small_requests_finish_while_a_large_one_runs(ctx, pool):
    # the large request (n >= solo_min_n) runs on its own stream; small
    # requests submitted after it complete in the engine before it does
    import paper_2609_07204_amd as mc
    big = pool[13]
    srv = mc.Server(ctx, hbm_bytes=24 << 30, max_inflight=64, max_request_n=big.n, max_request_nnz=big.nnz)
    t_big = srv.submit(big)
    smalls = [gen.config_batch_graph(i) for i in range(0, 30, 3)]
    ts = [srv.submit(g) for g in smalls]
    done_order = []
    res = {}
    for _ in range(200000):
        srv.step()
        for t in [t_big] + ts:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r
                    done_order.append(t)
        if len(res) == len(ts) + 1:
            break
    assert len(res) == len(ts) + 1
    assert res[t_big][0] == GOLDEN["served_pool_13"]["lambda"]
    for t, g in zip(ts, smalls):
        assert res[t][0] == oracle.noi(g)[0]
    say("completion order of the large request:", done_order.index(t_big), "of", len(done_order))
    srv.close()


def test_batch_per_graph_statuses(ctx):
    # each graph is checked on its own: bad ones get their status and are
    # skipped, their outputs untouched, and the rest are solved
    import paper_2609_07204_amd as mc
    good = [gen.complete(6), gen.wheel(12), gen.config_batch_graph(5), gen.cycle([3, 1, 4, 1, 5])]
    neg = gen.Graph(good[0].n, good[0].row_ptr.copy(), good[0].col.copy(), good[0].w.copy())
    neg.w[2] = -1
    oob = gen.Graph(good[1].n, good[1].row_ptr.copy(), good[1].col.copy(), good[1].w.copy())
    oob.col[4] = good[1].n + 3
    heavy = gen.from_edges(3, [0, 1], [1, 2], [1 << 60, 1 << 60])   # total 2^62
    gs = [good[0], neg, good[1], oob, good[2], heavy, good[3]]
    expect = [0, -2, 0, -2, 0, -3, 0]
    refs = {i: oracle_lambda(g) for i, g in enumerate(gs) if expect[i] == 0}
    for where in ("host", "device"):
        kw = {"graphs": gs} if where == "host" else {"devs": [ctx.upload(g) for g in gs]}
        lams, sides, st = ctx.mincut_batch(per_graph=True, **kw)
        assert list(st) == expect, (where, list(st))
        for i in range(len(gs)):
            if expect[i] == 0:
                assert lams[i] == refs[i] and oracle.cut_value(gs[i], sides[i]) == refs[i]
            else:
                assert lams[i] == 0 and not sides[i].any()   # untouched (zero-initialised)
        with pytest.raises(mc.MincutError) as e:
            ctx.mincut_batch(**kw)
        assert e.value.code == -2   # the first bad graph fails a call without per_graph


def oracle_lambda(g):
    return oracle.stoer_wagner(g)[0] if g.n <= 400 else oracle.noi(g)[0]


def test_batch_weight_bound_is_per_graph(ctx):
    # each graph's total weight is below 2^62; together they are not
    a = gen.from_edges(3, [0, 1, 0], [1, 2, 2], [1 << 59, 3 << 58, 5])
    b = gen.from_edges(4, [0, 1, 2, 3], [1, 2, 3, 0], [1 << 59, 1 << 59, 7, 9])
    assert 2 * (int(a.w.sum()) // 2) < (1 << 62) and int(a.w.sum()) + int(b.w.sum()) >= (1 << 62)
    for kw in ({"graphs": [a, b]}, {"devs": [ctx.upload(a), ctx.upload(b)]}):
        lams, sides = ctx.mincut_batch(**kw)
        assert lams[0] == oracle.brute(a)[0] and lams[1] == oracle.brute(b)[0]
        assert oracle.cut_value(a, sides[0]) == lams[0] and oracle.cut_value(b, sides[1]) == lams[1]


def test_batch_validate_option_checks_symmetry(ctx):
    import paper_2609_07204_amd as mc
    g = gen.complete(5)
    asym = gen.Graph(5, g.row_ptr.copy(), g.col.copy(), g.w.copy())
    asym.w[0] += 1
    ctx.set_options(validate=1)
    try:
        _, _, st = ctx.mincut_batch([g, asym], per_graph=True)
        assert list(st) == [0, -2]
        with pytest.raises(mc.MincutError) as e:
            ctx.mincut(asym)
        assert e.value.code == -2
    finally:
        ctx.set_options(validate=0)


def test_mincut_outputs_untouched_on_error(ctx):
    import torch
    import paper_2609_07204_amd as mc
    g = gen.complete(6)
    rp, col, w = ctx.upload(g)
    ws = torch.empty(ctx.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device=ctx.device)
    cases = []
    w2 = w.clone()
    w2[1] = -4
    cases.append(((rp, col, w2), -2))
    col2 = col.clone()
    col2[5] = -1
    cases.append(((rp, col2, w), -2))
    w3 = torch.full_like(w, 1 << 58)
    cases.append(((rp, col, w3), -3))
    for (r, c, x), code in cases:
        csr = mc.CSR(g.n, g.nnz, r.data_ptr(), c.data_ptr(), x.data_ptr(), mc.MC_DEVICE)
        lam = ctypes.c_int64(-99)
        side = np.full(g.n, 7, np.uint8)
        st = mc.Stats()
        st.rounds = -3
        rc = mc.lib().mc_mincut(ctx.h, ctypes.byref(csr), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.byref(lam), side.ctypes.data, ctypes.byref(st))
        assert rc == code
        assert lam.value == -99 and (side == 7).all() and st.rounds == -3
    # too small a workspace
    csr = mc.CSR(g.n, g.nnz, rp.data_ptr(), col.data_ptr(), w.data_ptr(), mc.MC_DEVICE)
    lam = ctypes.c_int64(-99)
    rc = mc.lib().mc_mincut(ctx.h, ctypes.byref(csr), ctypes.c_void_p(ws.data_ptr()), 1024, ctypes.byref(lam),
                            None, None)
    assert rc == -1 and lam.value == -99


def test_server_rejects_malformed_requests_at_submit(ctx):
    import paper_2609_07204_amd as mc
    srv = mc.Server(ctx, hbm_bytes=512 << 20, max_inflight=16, max_request_n=1 << 14, max_request_nnz=1 << 18)
    good = [gen.complete(7), gen.wheel(20), gen.config_batch_graph(4)]
    bad = gen.Graph(good[1].n, good[1].row_ptr.copy(), good[1].col.copy(), good[1].w.copy())
    bad.col[0] = 10 ** 6
    heavy = gen.from_edges(3, [0, 1], [1, 2], [1 << 60, 1 << 60])
    ts = [srv.submit(good[0])]
    with pytest.raises(mc.MincutError) as e:
        srv.submit(bad)
    assert e.value.code == -2
    with pytest.raises(mc.MincutError) as e:
        srv.submit(heavy)
    assert e.value.code == -3
    ts += [srv.submit(good[1]), srv.submit(good[2])]
    res = {}
    for _ in range(10000):
        srv.step()
        for t in ts:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r
        if len(res) == len(ts):
            break
    assert [res[t][0] for t in ts] == [oracle_lambda(g) for g in good]
    srv.close()


def test_server_deadline_and_cancel_in_flight(ctx):
    import paper_2609_07204_amd as mc
    g = gen.config_batch_graph(11)
    # a deadline no request can meet: every request times out
    srv = mc.Server(ctx, hbm_bytes=512 << 20, max_inflight=16, max_request_n=1 << 16, max_request_nnz=1 << 21,
                    deadline_ms=1e-6)
    ts = [srv.submit(g) for _ in range(3)]
    for _ in range(20):
        srv.step()
    for t in ts:
        assert srv.state(t) == 5
        with pytest.raises(mc.MincutError) as e:
            srv.poll(t)
        assert e.value.code == -8
    srv.close()
    # cancel after admission: the request leaves at the next step, the
    # others finish with their results
    srv = mc.Server(ctx, hbm_bytes=512 << 20, max_inflight=16, max_request_n=1 << 16, max_request_nnz=1 << 21,
                    deadline_ms=600000.0)
    big = gen.config_batch_graph(2)   # several rounds
    t0 = srv.submit(big)
    t1 = srv.submit(g)
    srv.step()
    assert srv.state(t0) in (1, 2)
    was_running = srv.state(t0) == 1
    srv.cancel(t0)
    res = None
    for _ in range(10000):
        srv.step()
        res = srv.poll(t1)
        if res is not None:
            break
    assert res is not None and res[0] == oracle_lambda(g)
    with pytest.raises(mc.MincutError) as e:
        srv.poll(t0)
    assert e.value.code == -7
    say("cancelled while in flight:", was_running)
    srv.close()

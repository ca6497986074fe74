"""Benchmark: exact minimum cut on one MI355X.

One step = one full exact solve (Algorithm 2 of the paper: normalisation,
minimum-degree bound, connectivity check, the label-propagation bound,
rounds of reduction tests, CAPFOREST passes, union-find relabel and
contraction until at most two vertices remain) of a graph already resident
in HBM.

Default workload (the largest single-graph configuration): a random
hyperbolic graph, n = 2^23, mean degree 64, power-law exponent 5, largest
component of its 32-core, int64 weights in [1,100], seed 1 (1.65 M vertices,
52.8 M edges). metric: edges contracted per second = input edges / solve
time (every input edge is contracted away or ends in the final cut during
one solve). The same JSON line carries, as context:
  - the same graph solved with the heuristic off (the multi-round
    contraction regime at full size), with every round's sizes, time and
    algorithmic GB/s;
  - the Chung-Lu graph (n = 2^22, exponent 2.5, mean degree 20, 10-core);
  - the batch of 4,096 mixed graphs: batched solves/s against plain
    per-graph solves and the oracle on every host core.
Timing is taken with kernel profiling off; one extra profiled solve fills
the roofline and the per-round records.

Other modes: --workload chung_lu | batch | served (see --help).
Prints one JSON line. --gpus > 1 is refused: the solver runs on one GPU.
"""
import argparse
import json
import multiprocessing as mp
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def worker_count():
    # the GPU machine gives one GPU's share of 16 host cores
    return max(1, min(16, host_info()[1]))


def traffic_for(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size),
    or None when there is none for this workload or the kernel's source has
    changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    tab = json.load(open(path)).get(workload)
    if not tab:
        return None
    rec = tab.get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


# ------------------------------------------------------------ generation
def _gen_config(which, log2n, seed):
    import gen
    g = gen.config_rhg(log2n, seed) if which == "rhg" else gen.config_chung_lu(log2n, seed)
    return g.n, g.row_ptr, g.col, g.w, g.name


def _batch_graph(args):
    i, seed0 = args
    import gen
    g = gen.config_batch_graph(i, seed0)
    return g.n, g.row_ptr, g.col, g.w, g.name


def _to_graph(t):
    import gen
    n, rp, col, w, name = t
    return gen.Graph(n, rp, col, w, name)


def _noi_lambda(t):
    import oracle
    return oracle.noi(_to_graph(t))[0]


# ------------------------------------------------------------ single solves
def round_record(r):
    """One round of the last profiled solve: undirected edges in and out,
    device time, edges contracted per second and algorithmic GB/s. A round of
    Algorithm 2 moves about 40 B per entry in (reduction tests 12, CAPFOREST
    12, contraction 16), 12 B per entry out and 40 B per vertex; a coarsening
    level of the heuristic about 44 B per entry in (two LP rounds 28,
    contraction 16), 24 B per entry out (written, then read by the tests)
    and 60 B per vertex."""
    m_in, m_out, n = r["m_in"], r["m_out"], r["n_in"]
    if r["kind"] == "level":
        alg = 44 * m_in + 24 * m_out + 60 * n
    else:
        alg = 40 * m_in + 12 * m_out + 40 * n
    ms = r["ms"]
    return {"kind": r["kind"], "n": n, "n_out": r["n_out"], "m": m_in // 2, "m_out": m_out // 2,
            "ms": round(ms, 4), "edges_per_s": (m_in / 2) / (ms / 1000.0) if ms > 0 else 0.0,
            "alg_gbps": alg / (ms * 1e6) if ms > 0 else 0.0}


def time_solves(ctx, dev, ws, steps, warmup, label):
    """W untimed then K timed solves, each bracketed by a stream
    synchronisation (mc_mincut synchronises before it returns). Returns
    (lambda, per-step ms, stats of the last step)."""
    import torch
    lam0, st = None, None
    for i in range(warmup):
        lam0, _, st = ctx.mincut(dev=dev, workspace=ws, want_side=False, return_stats=True)
        log("%s warmup %d: lambda=%d rounds=%d heuristic levels=%d bound=%d %.2f ms" % (
            label, i, lam0, st["rounds"], st["heuristic_levels"], st["lambda_heuristic"], st["ms_total"]))
    torch.cuda.synchronize()
    per = []
    for i in range(steps):
        t0 = time.perf_counter()
        lam, _, st = ctx.mincut(dev=dev, workspace=ws, want_side=False, return_stats=True)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) * 1000.0)
        assert lam0 is None or lam == lam0
        lam0 = lam
    log("%s: %d steps, median %.3f ms, mean %.3f ms, lambda=%d rounds=%d" % (
        label, steps, statistics.median(per), statistics.mean(per), lam0, st["rounds"]))
    return lam0, per, st


def profiled_solve(ctx, dev, ws, label):
    """One solve with kernel timing on: per-round records and per-kernel
    totals (HIP events on the library's stream around each timed launch)."""
    ctx.profile(True)
    lam, _, st = ctx.mincut(dev=dev, workspace=ws, want_side=False, return_stats=True)
    ctx.profile(False)
    rounds = [round_record(r) for r in ctx.profile_rounds()]
    for r in rounds:
        log("  %s round %-6s n %9d -> %9d  edges %10d -> %10d  %8.3f ms  %6.2f G edges/s  %7.1f GB/s algorithmic" % (
            label, r["kind"], r["n"], r["n_out"], r["m"], r["m_out"], r["ms"], r["edges_per_s"] / 1e9, r["alg_gbps"]))
    kt = ctx.profile_read()
    for name, r in sorted(kt.items(), key=lambda kv: -kv[1]["ms"]):
        if r["launches"]:
            log("  %s %-16s %4d launches %8.3f ms  avg %8.1f us  %7.1f GB/s algorithmic" % (
                label, name, r["launches"], r["ms"], 1000.0 * r["ms"] / r["launches"],
                r["bytes"] / (r["ms"] * 1e6) if r["ms"] > 0 else 0.0))
    return lam, st, rounds, kt


def roofline_of(kt, workload):
    name, r = max(kt.items(), key=lambda kv: kv[1]["ms"])
    achieved = r["bytes"] / (r["ms"] * 1e6)          # GB/s = bytes per launch / avg launch time
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_for(name, workload),
            "kernel": name, "launches_per_step": r["launches"], "avg_launch_us": 1000.0 * r["ms"] / r["launches"],
            "bytes_per_launch": r["bytes"] / r["launches"], "kernel_ms_per_step": r["ms"]}


def golden_check(key, lam):
    gpath = os.path.join(ROOT, "tests", "golden", "lambda.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else {}
    if key in golden:
        assert golden[key]["lambda"] == lam, ("lambda differs from the oracle's", lam, golden[key])
        return True
    return False


# ------------------------------------------------------------ batch
def batch_run(ctx, gs, tune_gs, steps, warmup, plain=True, cpu_seconds=15.0, fixed=None):
    """Batched solves of gs (one mc_mincut_batch per step) after autotuning
    on a separate batch tune_gs (same generators, other seeds), plain
    per-graph solves of the same graphs, and the oracle on every host core.
    Returns a dict of the measurements."""
    import numpy as np
    import torch
    out = {"graphs": len(gs), "vertices": sum(g.n for g in gs), "entries": sum(g.nnz for g in gs)}
    devs = [ctx.upload(g) for g in gs]
    ws_bytes = ctx.batch_workspace_bytes(devs=devs)
    tuning = None
    if fixed is not None:
        ctx.set_options(batch_pass_threads=fixed[0], batch_lp=fixed[1])
        tuning = {"fixed": True, "pass_threads": fixed[0] or 256, "lp": fixed[1]}
    elif tune_gs:
        tdevs = [ctx.upload(g) for g in tune_gs]
        ws_bytes = max(ws_bytes, ctx.batch_workspace_bytes(devs=tdevs))
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=ctx.device)
        t = time.time()
        tuning = ctx.batch_autotune(devs=tdevs, workspace=ws, sample=len(tdevs))
        tuning["seconds"] = time.time() - t
        log("autotune on a separate batch (%d graphs, %.1fs): pass threads %d, admission bound %s, "
            "finisher limit %d, queue %d" % (tuning["sample"], tuning["seconds"], tuning["pass_threads"],
                                             "on" if tuning["lp"] == 1 else "off", tuning["finish_max_n"],
                                             tuning["queue"]))
        del tdevs, ws
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=ctx.device)
    torch.cuda.synchronize()
    lams = None
    for _ in range(warmup):
        lams, _ = ctx.mincut_batch(devs=devs, workspace=ws, want_sides=False)
    per = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        l2, _ = ctx.mincut_batch(devs=devs, workspace=ws, want_sides=False)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) * 1000.0)
        assert lams is None or np.array_equal(l2, lams)
        lams = l2
    ms = statistics.median(per)
    out.update({"batched_ms": ms, "batched_ms_mean": statistics.mean(per), "solves_per_s": len(gs) / (ms / 1000.0)})
    log("batched: median %.2f ms per batch, %.1f solves/s" % (ms, out["solves_per_s"]))
    if tuning is not None:
        out["tuning"] = {k: (round(v, 2) if isinstance(v, float) else v) for k, v in tuning.items()
                         if k != "candidates"}
    if plain:
        wsp = torch.empty(max(ctx.workspace_bytes(g.n, g.nnz) for g in gs), dtype=torch.uint8, device=ctx.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl = np.zeros(len(gs), np.int64)
        for i, d in enumerate(devs):
            pl[i], _ = ctx.mincut(dev=d, workspace=wsp, want_side=False)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - t0) * 1000.0
        assert np.array_equal(pl, lams), "batched and plain lambdas differ"
        out.update({"plain_solves_per_s": len(gs) / (ms_plain / 1000.0), "batched_over_plain": ms_plain / ms})
        log("plain: %.1f ms for %d solves, %.1f solves/s" % (ms_plain, len(gs), out["plain_solves_per_s"]))
        del wsp
    if cpu_seconds > 0:
        # the oracle on every host core: one process per core over the
        # graphs in order, for about cpu_seconds
        procs = worker_count()
        t = time.perf_counter()
        done = 0
        with mp.get_context("fork").Pool(procs) as pool:
            it = pool.imap(_noi_lambda, ((g.n, g.row_ptr, g.col, g.w, g.name) for g in gs), chunksize=1)
            for i, lam in enumerate(it):
                assert lam == lams[i], ("oracle and GPU differ on batch graph", i)
                done += 1
                if time.perf_counter() - t > cpu_seconds:
                    break
            pool.terminate()
        tc = time.perf_counter() - t
        out["cpu"] = {"value": done / tc, "unit": "solves/s", "cores": procs, "kind": "oracle",
                      "sample": "the first %d graphs of the batch, one NOI solve each, one process per core, "
                                "%.1f s" % (done, tc)}
        log("oracle on %d cores: %d graphs in %.1f s, %.1f solves/s" % (procs, done, tc, done / tc))
    return out, lams


def gen_batch(count, seed0, pool):
    return [_to_graph(t) for t in pool.map(_batch_graph, [(i, seed0) for i in range(count)], chunksize=8)]


def batch_main(args):
    import paper_2609_07204_amd as mc
    t = time.time()
    with mp.get_context("fork").Pool(worker_count()) as pool:
        gs = gen_batch(args.batch_count, 1000, pool)
        tune = gen_batch(args.batch_count, 5000, pool) if args.tune and not (args.batch_threads or args.batch_lp) \
            else None
    log("generated %d graphs (+%d for tuning) in %.1fs" % (len(gs), len(tune or []), time.time() - t))
    ctx = mc.Context(0, pass_len_cap=args.len_cap, heuristic_min_n=args.heuristic_min_n)
    fixed = (args.batch_threads, args.batch_lp) if (args.batch_threads or args.batch_lp) else None
    res, _ = batch_run(ctx, gs, tune, args.steps, args.warmup, plain=not args.no_plain,
                       cpu_seconds=0 if args.no_cpu_baseline else 15.0, fixed=fixed)
    model, _ = host_info()
    out = {
        "metric": "min-cut solves/sec (batched)", "value": res["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["batched_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batch of %d graphs: planted / Erdos-Renyi / Chung-Lu, n log-uniform in "
                               "[64, 65536], mean degree 8-32, weights 1-100, seeds 1000+i" % len(gs),
                   **{k: v for k, v in res.items() if k != "cpu"}, "host_cpu": model},
        "cpu_baseline": res.get("cpu"),
    }
    print(json.dumps(out))


# ------------------------------------------------------------ served
def _served_graph(j):
    import gen
    g = gen.config_served_graph(j)
    return g.n, g.row_ptr, g.col, g.w, g.name


def served_main(args):
    """Served workload: Poisson arrivals (seed 7) at each rate of --rates,
    each request a graph drawn from a pool of pre-generated graphs (edge
    counts log-uniform in [10^3, 10^7], the three families, weights 1-1000).
    The same arrival trace goes to the continuous-batching server
    (mc_server_*) and to plain per-graph solves (mc_mincut, one request at a
    time in arrival order). Latency = completion - arrival. Prints one JSON
    line; value = served solves per second at the highest rate."""
    import numpy as np
    import paper_2609_07204_amd as mc

    t = time.time()
    with mp.get_context("fork").Pool(worker_count()) as pool:
        raw = pool.map(_served_graph, range(args.pool), chunksize=2)
    gs = [_to_graph(r) for r in raw]
    log("pool of %d graphs: %d entries in %.1fs" % (len(gs), sum(g.nnz for g in gs), time.time() - t))
    ctx = mc.Context(0)
    alone = {}
    srv = mc.Server(ctx, hbm_bytes=int(args.hbm_gb * (1 << 30)), max_inflight=args.max_inflight,
                    max_request_n=max(g.n for g in gs), max_request_nnz=max(g.nnz for g in gs),
                    solo_slots=args.solo_slots)
    log("server capacity", srv.capacity())
    rates = [float(x) for x in args.rates.split(",")]
    per_rate = []
    rng = np.random.default_rng(7)
    traces = []
    for rate in rates:
        picks = rng.integers(0, len(gs), args.requests)
        arrive = np.cumsum(rng.exponential(1.0 / rate, args.requests))
        traces.append((rate, picks, arrive))

    def record(kind, rate, lat, el, steps=None):
        lat_ms = np.array(lat) * 1000.0
        rec = {"solves_per_s": len(lat) / el, "p50_ms": float(np.percentile(lat_ms, 50)),
               "p99_ms": float(np.percentile(lat_ms, 99))}
        if steps is not None:
            rec["steps"] = steps
        log("%s rate %.0f/s: %.1f solves/s, p50 %.1f ms, p99 %.1f ms" % (kind, rate, rec["solves_per_s"],
                                                                       rec["p50_ms"], rec["p99_ms"]))
        return rec

    for rate, picks, arrive in traces:
        # served: submit on arrival, one step at a time
        t0 = time.perf_counter()
        nxt, out, lat, steps = 0, {}, [], 0
        while len(lat) < args.requests:
            now = time.perf_counter() - t0
            while nxt < args.requests and arrive[nxt] <= now:
                out[srv.submit(gs[picks[nxt]])] = nxt
                nxt += 1
            if out:
                srv.step()
                steps += 1
                tdone = time.perf_counter() - t0
                for tk in list(out):
                    r = srv.poll(tk)
                    if r is not None:
                        i = out.pop(tk)
                        lat.append(tdone - arrive[i])
                        j = int(picks[i])
                        alone.setdefault(j, r[0])
                        assert r[0] == alone[j], "served result differs between requests of one graph"
            elif nxt < args.requests:
                time.sleep(max(0.0, min(0.001, arrive[nxt] - now)))
        served = record("served", rate, lat, time.perf_counter() - t0, steps)
        plain = None
        if not args.no_plain:
            # plain: the same arrivals, each solved alone as soon as the GPU
            # is free (host input, as the server gets it)
            t0 = time.perf_counter()
            lat = []
            for i in range(args.requests):
                now = time.perf_counter() - t0
                if arrive[i] > now:
                    time.sleep(arrive[i] - now)
                lam, _ = ctx.mincut(gs[picks[i]], want_side=False)
                lat.append(time.perf_counter() - t0 - arrive[i])
                j = int(picks[i])
                alone.setdefault(j, lam)
                assert lam == alone[j], "plain and served results differ"
            plain = record("plain", rate, lat, time.perf_counter() - t0)
        per_rate.append({"rate_per_s": rate, "requests": args.requests, "served": served, "plain": plain})
    cpu = None
    if not args.no_cpu_baseline:
        procs = worker_count()
        js = sorted(alone)
        t = time.perf_counter()
        done = 0
        with mp.get_context("fork").Pool(procs) as pool:
            for q, lam in enumerate(pool.imap(_noi_lambda, ((gs[j].n, gs[j].row_ptr, gs[j].col, gs[j].w, "")
                                                            for j in js), chunksize=1)):
                assert lam == alone[js[q]]
                done += 1
                if time.perf_counter() - t > 15.0:
                    break
            pool.terminate()
        tc = time.perf_counter() - t
        cpu = {"value": done / tc, "unit": "solves/s", "cores": procs, "kind": "oracle",
               "sample": "%d distinct pool graphs, one NOI solve each, one process per core, %.1f s" % (done, tc)}
    top = per_rate[-1]
    model, _ = host_info()
    out = {
        "metric": "served min-cut solves/sec", "value": top["served"]["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": args.requests, "warmup": 0, "ms_per_step": 1000.0 / top["served"]["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "served: Poisson arrivals, pool of %d graphs (m log-uniform [1e3, 1e7], planted / "
                               "Erdos-Renyi / Chung-Lu, weights 1-1000, seeds 2000000+j)" % len(gs),
                   "hbm_gb": args.hbm_gb, "max_inflight": args.max_inflight, "solo_slots": args.solo_slots,
                   "rates": per_rate, "host_cpu": model},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


# ------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=None, help="graph size (default 2^23 hyperbolic, 2^22 Chung-Lu)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-context", action="store_true",
                    help="single-graph workloads: only the headline solves (no heuristic-off solve, Chung-Lu or "
                         "batch context)")
    ap.add_argument("--passes", type=int, default=0)
    ap.add_argument("--len-cap", type=int, default=0)
    ap.add_argument("--workload", choices=["rhg", "chung_lu", "batch", "served"], default="rhg",
                    help="rhg: one exact solve of the random hyperbolic graph (default); chung_lu: of the "
                         "Chung-Lu graph; batch: the mixed batch, batched against plain per-graph solves; "
                         "served: Poisson requests to the server and to plain per-graph solves")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-plain", action="store_true", help="batch/served: skip the plain per-graph comparison")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="batch: no autotuning (default: tune on a separate batch, seeds 5000+i)")
    ap.add_argument("--batch-threads", type=int, default=0, choices=[0, 64, 128, 256, 512, 1024],
                    help="batch: fixed pass workgroup size instead of autotuning (0: autotune)")
    ap.add_argument("--batch-lp", type=int, default=0, choices=[0, 1, 2],
                    help="batch: fixed admission bound (1 on, 2 off) instead of autotuning (0: autotune)")
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--rates", default="50,100,200,500,1000,2000", help="served: arrival rates per second")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--hbm-gb", type=float, default=48.0)
    ap.add_argument("--max-inflight", type=int, default=256)
    ap.add_argument("--solo-slots", type=int, default=2)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the solves, one device-to-device copy of this many MiB (the known-size kernel "
                         "that scales hardware byte counters)")
    ap.add_argument("--lp-iters", type=int, default=0, help="label-propagation rounds per level (0: default)")
    ap.add_argument("--contract-mode", type=int, default=0, choices=[0, 1],
                    help="edge merge of the contractions: 0 hash (default), 1 radix sort")
    ap.add_argument("--tri-cap", type=int, default=-1, help="row-length cap of reduction tests 3 and 4 (-1: default)")
    ap.add_argument("--heuristic-min-n", type=int, default=10000,
                    help="run the label-propagation bound on graphs with at least this many vertices (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (it has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return batch_main(args)
    if args.workload == "served":
        return served_main(args)

    import torch
    import paper_2609_07204_amd as mc

    which = args.workload
    log2n = args.log2n or (23 if which == "rhg" else 22)
    context = not args.no_context and which == "rhg" and args.log2n is None
    t = time.time()
    # the context graphs are generated in worker processes meanwhile (no
    # pool at all without context, so profiler runs see one process)
    pool = mp.get_context("fork").Pool(worker_count()) if context else None
    cl_job = pool.apply_async(_gen_config, ("chung_lu", 22, args.seed)) if context else None
    batch_job = pool.map_async(_batch_graph, [(i, 1000) for i in range(args.batch_count)], chunksize=8) \
        if context else None
    tune_job = pool.map_async(_batch_graph, [(i, 5000) for i in range(args.batch_count)], chunksize=8) \
        if context else None
    g = _to_graph(_gen_config(which, log2n, args.seed))
    if which == "rhg":
        key = "rhg_2^%d_core32_seed%d" % (log2n, args.seed)
        wname = "rhg n=2^%d avg_deg=64 gamma=5 32-core LCC weights 1-100 seed=%d" % (log2n, args.seed)
    else:
        key = "chung_lu_2^%d_core10_seed%d" % (log2n, args.seed)
        wname = "chung_lu n=2^%d beta=2.5 avg_deg=20 10-core LCC unit weights seed=%d" % (log2n, args.seed)
    log("generated %s: n=%d m=%d in %.1fs" % (g.name, g.n, g.m, time.time() - t))
    extra = {}
    if args.lp_iters > 0:
        extra["lp_iters"] = args.lp_iters
    if args.contract_mode:
        extra["contract_mode"] = args.contract_mode
    if args.tri_cap >= 0:
        extra["pr_tri_deg_cap"] = args.tri_cap
    ctx = mc.Context(0, capforest_passes=args.passes, pass_len_cap=args.len_cap,
                     heuristic_min_n=args.heuristic_min_n, **extra)
    dev = ctx.upload(g)
    ws = torch.empty(ctx.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device=ctx.device)
    torch.cuda.synchronize()
    if context:
        # a solve waits on the host between rounds: time it with the host's
        # cores quiet, after the context graphs are generated
        for job in (cl_job, batch_job, tune_job):
            job.wait()
    lam, per, st = time_solves(ctx, dev, ws, args.steps, args.warmup, which)
    ms = statistics.median(per)
    lam_p, st_p, rounds, kt = profiled_solve(ctx, dev, ws, which)
    assert lam_p == lam
    roofline = roofline_of(kt, which)
    oracle_checked = golden_check(key, lam)

    ctxinfo = {}
    if context:
        # the same graph with the heuristic off: Algorithm 2's rounds alone,
        # the multi-round contraction regime at full size
        ctx.set_options(heuristic_min_n=0)
        t0 = time.perf_counter()
        lam_x, _, st_x = ctx.mincut(dev=dev, workspace=ws, want_side=False, return_stats=True)
        torch.cuda.synchronize()
        ms_x = (time.perf_counter() - t0) * 1000.0
        lam_xp, _, rounds_x, _ = profiled_solve(ctx, dev, ws, which + "/no-heuristic")
        ctx.set_options(heuristic_min_n=args.heuristic_min_n)
        assert lam_x == lam and lam_xp == lam
        ctxinfo["rhg_heuristic_off"] = {"ms": ms_x, "edges_per_s": g.m / (ms_x / 1000.0), "rounds": st_x["rounds"],
                                        "fallback_passes": st_x["fallback_passes"], "round_records": rounds_x}
        log("heuristic off: %.1f ms, %d rounds" % (ms_x, st_x["rounds"]))
        del dev, ws
        torch.cuda.empty_cache()
        # Chung-Lu n = 2^22 (context)
        gc = _to_graph(cl_job.get())
        dc = ctx.upload(gc)
        wsc = torch.empty(ctx.workspace_bytes(gc.n, gc.nnz), dtype=torch.uint8, device=ctx.device)
        lam_c, per_c, st_c = time_solves(ctx, dc, wsc, 3, 1, "chung_lu")
        golden_check("chung_lu_2^22_core10_seed%d" % args.seed, lam_c)
        ms_c = statistics.median(per_c)
        ctxinfo["chung_lu"] = {"n": gc.n, "m": gc.m, "lambda": lam_c, "ms": ms_c, "edges_per_s": gc.m / (ms_c / 1e3),
                               "rounds": st_c["rounds"], "heuristic_levels": st_c["heuristic_levels"]}
        del dc, wsc, gc
        torch.cuda.empty_cache()
        # the batch of 4,096 graphs (context): batched vs plain vs oracle
        gs = [_to_graph(r) for r in batch_job.get()]
        tune = [_to_graph(r) for r in tune_job.get()]
        res, _ = batch_run(mc.Context(0), gs, tune, 3, 1, plain=True,
                           cpu_seconds=0 if args.no_cpu_baseline else 15.0)
        ctxinfo["batch"] = res
        del gs, tune
        torch.cuda.empty_cache()
        pool.close()

    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=ctx.device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB device to device" % args.calibrate_copy)
        del src, dst

    cpu = None
    model, cores = host_info()
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        lam_cpu, _ = oracle.noi(g)
        tc = time.perf_counter() - t
        assert lam_cpu == lam
        cpu = {"value": g.m / tc, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "full workload, one NOI solve (repeated full CAPFOREST + contraction) on one core of "
                         "%s, %.1f s" % (model, tc)}

    out = {
        "metric": "edges contracted/sec",
        "value": g.m / (ms / 1000.0),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wname, "n": g.n, "m": g.m, "lambda": lam, "lambda_checked_against_oracle":
                   oracle_checked, "rounds": st["rounds"], "heuristic_levels": st["heuristic_levels"],
                   "ms_median": ms, "ms_mean": statistics.mean(per), "ms_steps": [round(x, 3) for x in per],
                   "host_cpu": model, "host_cores": cores, "context": ctxinfo or None},
        "roofline": roofline,
        "rounds": rounds,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

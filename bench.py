"""Benchmark: exact minimum cut of the Chung-Lu workload on one MI355X.

One step = one full exact solve (Algorithm 2 of the paper: normalisation,
minimum-degree bound, connectivity check, rounds of reduction tests,
CAPFOREST passes, union-find relabel and contraction until at most two
vertices remain) of a graph already resident in HBM.

Workload: Chung-Lu, n = 2^22, exponent 2.5, mean degree 20, reduced to the
largest connected component of its 10-core, unit int64 weights, seed 1
(~1.90 M vertices, ~25.6 M edges). metric: edges contracted per second =
input edges / solve time (every input edge is contracted away or ends in the
final cut during one solve).

Prints one JSON line. --gpus > 1 is refused: the solver runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


PEAK_HBM_GBS = 8000.0   # MI355X HBM3E peak


def traffic_for(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size),
    or None when there is none, it was measured on another workload, or its
    kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    tab = json.load(open(path))
    if tab.get("_calibration", {}).get("workload", "chung_lu") != workload:
        return None
    rec = tab.get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def _batch_graph(i):
    import gen
    g = gen.config_batch_graph(i)
    return g.n, g.row_ptr, g.col, g.w, g.name


def batch_main(args, log):
    """Batched workload: `count` graphs of the mixed batch configuration
    solved in one mc_mincut_batch call (timed over the steps), against the
    same graphs solved one by one with mc_mincut (plain per-graph launches,
    one pass). Prints one JSON line; value = batched solves per second."""
    import multiprocessing as mp
    import numpy as np
    import torch
    import gen
    import paper_2609_07204_amd as mc

    t = time.time()
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        raw = pool.map(_batch_graph, range(args.batch_count), chunksize=8)
    gs = [gen.Graph(n, rp, col, w, name) for n, rp, col, w, name in raw]
    N = sum(g.n for g in gs)
    M = sum(g.nnz for g in gs)
    log("generated %d graphs: %d vertices, %d entries in %.1fs" % (len(gs), N, M, time.time() - t))
    ctx = mc.Context(0, pass_len_cap=args.len_cap, heuristic_min_n=args.heuristic_min_n)
    devs = [ctx.upload(g) for g in gs]
    ws = torch.empty(ctx.batch_workspace_bytes(devs=devs), dtype=torch.uint8, device=ctx.device)
    log("batch workspace %.2f GB" % (ws.numel() / 1e9))
    tuning = None
    if args.batch_threads or args.batch_lp:
        # a fixed setting (for comparisons): no autotuning
        ctx.set_options(batch_pass_threads=args.batch_threads, batch_lp=args.batch_lp)
        tuning = {"fixed": True, "pass_threads": args.batch_threads or 256, "lp": args.batch_lp}
        log("fixed batch setting: pass threads %d, batch_lp %d" % (tuning["pass_threads"], args.batch_lp))
    elif args.tune_sample > 0:
        # untimed: the autotuner picks the pass workgroup size and whether to
        # bound at admission, by default on the whole batch: a sample of 512
        # or even 2048 of its graphs loads the GPU with fewer passes at once
        # and favoured 512-thread passes, which run the whole batch 12 %
        # slower than 256-thread ones
        t = time.time()
        tuning = ctx.batch_autotune(devs=devs, workspace=ws, sample=args.tune_sample)
        tuning["seconds"] = time.time() - t
        log("autotune (%d graphs, %.1fs): pass threads %d, admission bound %s; %s" % (
            tuning["sample"], tuning["seconds"], tuning["pass_threads"], "on" if tuning["lp"] == 1 else "off",
            ", ".join("%d/%s %.1f ms" % (c["pass_threads"], "on" if c["lp"] == 1 else "off", c["ms"])
                      for c in tuning["candidates"])))
    torch.cuda.synchronize()
    lams = None
    for i in range(args.warmup):
        lams, _ = ctx.mincut_batch(devs=devs, workspace=ws, want_sides=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        l2, _ = ctx.mincut_batch(devs=devs, workspace=ws, want_sides=False)
        assert lams is None or np.array_equal(l2, lams)
        lams = l2
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    log("batched: %.2f ms per batch, %.1f solves/s" % (ms, len(gs) / (ms / 1000.0)))
    if args.no_plain:
        print(json.dumps({"batched_ms": ms, "solves_per_s": len(gs) / (ms / 1000.0), "len_cap": args.len_cap,
                          "heuristic_min_n": args.heuristic_min_n, "tuning": tuning}))
        return
    # plain: one mc_mincut per graph on the same stream, workspace reused
    wsp = torch.empty(max(ctx.workspace_bytes(g.n, g.nnz) for g in gs), dtype=torch.uint8, device=ctx.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = np.zeros(len(gs), np.int64)
    for i, d in enumerate(devs):
        plain[i], _ = ctx.mincut(dev=d, workspace=wsp, want_side=False)
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) * 1000.0
    log("plain: %.1f ms for %d solves, %.1f solves/s" % (ms_plain, len(gs), len(gs) / (ms_plain / 1000.0)))
    assert np.array_equal(plain, lams), "batched and plain lambdas differ"
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        done = 0
        for i, g in enumerate(gs):
            assert oracle.noi(g)[0] == lams[i]
            done += 1
            if time.perf_counter() - t > 15.0:
                break
        tc = time.perf_counter() - t
        cpu = {"value": done / tc, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "the first %d graphs of the batch, one NOI solve each, %.1f s" % (done, tc)}
    out = {
        "metric": "min-cut solves/sec (batched)",
        "value": len(gs) / (ms / 1000.0),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "batch of %d graphs: planted / Erdos-Renyi / Chung-Lu, n log-uniform in "
                               "[64, 65536], mean degree 8-32, weights 1-100, seeds 1000+i" % len(gs),
                   "vertices": N, "entries": M, "plain_solves_per_s": len(gs) / (ms_plain / 1000.0),
                   "batched_over_plain": ms_plain / ms,
                   "tuning": None if tuning is None else {
                       "sample": tuning["sample"], "seconds": round(tuning["seconds"], 2),
                       "pass_threads": tuning["pass_threads"], "admission_bound": tuning["lp"] == 1}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def _served_graph(j):
    import gen
    g = gen.config_served_graph(j)
    return g.n, g.row_ptr, g.col, g.w, g.name


def served_main(args, log):
    """Served workload: Poisson arrivals (seed 7) at each rate of --rates,
    each request a graph drawn from a pool of pre-generated graphs (edge
    counts log-uniform in [10^3, 10^7], the three families, weights 1-1000),
    handled by the continuous-batching server (mc_server_*). Latency =
    completion - arrival. Prints one JSON line; value = completed solves per
    second at the highest rate."""
    import multiprocessing as mp
    import numpy as np
    import gen
    import paper_2609_07204_amd as mc

    t = time.time()
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        raw = pool.map(_served_graph, range(args.pool), chunksize=2)
    gs = [gen.Graph(n, rp, col, w, name) for n, rp, col, w, name in raw]
    log("pool of %d graphs: %d entries in %.1fs" % (len(gs), sum(g.nnz for g in gs), time.time() - t))
    ctx = mc.Context(0)
    alone = {}
    srv = mc.Server(ctx, hbm_bytes=int(args.hbm_gb * (1 << 30)), max_inflight=args.max_inflight,
                    max_request_n=max(g.n for g in gs), max_request_nnz=max(g.nnz for g in gs))
    log("server capacity", srv.capacity())
    rates = [float(x) for x in args.rates.split(",")]
    per_rate = []
    rng = np.random.default_rng(7)
    for rate in rates:
        picks = rng.integers(0, len(gs), args.requests)
        gaps = rng.exponential(1.0 / rate, args.requests)
        arrive = np.cumsum(gaps)
        t0 = time.perf_counter()
        nxt = 0
        out = {}
        lat = []
        steps = 0
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
                        if j not in alone:
                            alone[j] = r[0]
                        assert r[0] == alone[j], "served result differs between requests of one graph"
            elif nxt < args.requests:
                time.sleep(max(0.0, min(0.001, arrive[nxt] - now)))
        el = time.perf_counter() - t0
        lat_ms = np.array(lat) * 1000.0
        rec = {"rate_per_s": rate, "requests": args.requests, "solves_per_s": args.requests / el,
               "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
               "steps": steps}
        per_rate.append(rec)
        log("rate %.0f/s: %.1f solves/s, p50 %.1f ms, p99 %.1f ms, %d steps" % (
            rate, rec["solves_per_s"], rec["p50_ms"], rec["p99_ms"], steps))
    # every distinct graph served: its result equals the graph solved alone
    for j, lam in alone.items():
        lam1, _ = ctx.mincut(gs[j], want_side=False)
        assert lam == lam1, ("served and alone differ", j)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        done = 0
        for j in sorted(alone):
            assert oracle.noi(gs[j])[0] == alone[j]
            done += 1
            if time.perf_counter() - t > 15.0:
                break
        tc = time.perf_counter() - t
        cpu = {"value": done / tc, "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": "%d distinct pool graphs, one NOI solve each, %.1f s" % (done, tc)}
    top = per_rate[-1]
    out = {
        "metric": "served min-cut solves/sec", "value": top["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.requests, "warmup": 0, "ms_per_step": 1000.0 / top["solves_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "served: Poisson arrivals, pool of %d graphs (m log-uniform [1e3, 1e7], planted / "
                               "Erdos-Renyi / Chung-Lu, weights 1-1000, seeds 2000000+j)" % len(gs),
                   "hbm_gb": args.hbm_gb, "max_inflight": args.max_inflight, "rates": per_rate},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=None, help="graph size (default 2^22 Chung-Lu, 2^23 hyperbolic)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--passes", type=int, default=0)
    ap.add_argument("--len-cap", type=int, default=0)
    ap.add_argument("--no-profile", action="store_true", help="time the steps without kernel events")
    ap.add_argument("--workload", choices=["chung_lu", "rhg", "batch", "served"], default="chung_lu",
                    help="chung_lu: one exact solve of the Chung-Lu graph (default); rhg: one exact solve of "
                         "the random hyperbolic graph; batch: the mixed batch, batched against plain per-graph "
                         "solves; served: Poisson requests to the server")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-plain", action="store_true", help="batch: time the batched call only (parameter sweeps)")
    ap.add_argument("--tune-sample", type=int, default=4096,
                    help="batch: graphs the autotuner times before the run (at least --batch-count: the whole "
                         "batch; 0: no tuning)")
    ap.add_argument("--batch-threads", type=int, default=0, choices=[0, 64, 128, 256, 512, 1024],
                    help="batch: fixed pass workgroup size instead of autotuning (0: autotune)")
    ap.add_argument("--batch-lp", type=int, default=0, choices=[0, 1, 2],
                    help="batch: fixed admission bound (1 on, 2 off) instead of autotuning (0: autotune)")
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--rates", default="20,50,200,1000,2000",
                    help="served: arrival rates per second (20/s is below the server's capacity)")
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--hbm-gb", type=float, default=48.0)
    ap.add_argument("--max-inflight", type=int, default=256)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the solves, one device-to-device copy of this many MiB (the known-size kernel "
                         "that scales hardware byte counters)")
    ap.add_argument("--lp-iters", type=int, default=0, help="label-propagation rounds per level (0: default)")
    ap.add_argument("--tri-cap", type=int, default=-1, help="row-length cap of reduction tests 3 and 4 (-1: default)")
    ap.add_argument("--heuristic-min-n", type=int, default=10000,
                    help="run the label-propagation bound on graphs with at least this many vertices (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (it has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    if args.workload == "batch":
        return batch_main(args, log)
    if args.workload == "served":
        return served_main(args, log)

    import torch
    import gen
    import paper_2609_07204_amd as mc

    t = time.time()
    if args.workload == "rhg":
        args.log2n = args.log2n or 23
        g = gen.config_rhg(args.log2n, args.seed)
        key = "rhg_2^%d_core32_seed%d" % (args.log2n, args.seed)
        wname = ("rhg n=2^%d avg_deg=64 gamma=5 32-core LCC weights 1-100 seed=%d" % (args.log2n, args.seed))
    else:
        args.log2n = args.log2n or 22
        g = gen.config_chung_lu(args.log2n, args.seed)
        key = "chung_lu_2^%d_core10_seed%d" % (args.log2n, args.seed)
        wname = ("chung_lu n=2^%d beta=2.5 avg_deg=20 10-core LCC unit weights seed=%d" % (args.log2n, args.seed))
    log("generated %s: n=%d m=%d in %.1fs" % (g.name, g.n, g.m, time.time() - t))
    extra = {}
    if args.lp_iters > 0:
        extra["lp_iters"] = args.lp_iters
    if args.tri_cap >= 0:
        extra["pr_tri_deg_cap"] = args.tri_cap
    ctx = mc.Context(0, capforest_passes=args.passes, pass_len_cap=args.len_cap,
                     heuristic_min_n=args.heuristic_min_n, **extra)
    dev = ctx.upload(g)
    ws = torch.empty(ctx.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device=ctx.device)
    torch.cuda.synchronize()
    lam0 = None
    for i in range(args.warmup):
        lam, _, st = ctx.mincut(dev=dev, workspace=ws, want_side=(i == 0), return_stats=True)
        lam0 = lam
        log("warmup %d: lambda=%d rounds=%d fallback=%d heuristic levels=%d bound=%d %.2f ms" % (
            i, lam, st["rounds"], st["fallback_passes"], st["heuristic_levels"], st["lambda_heuristic"],
            st["ms_total"]))
    torch.cuda.synchronize()
    if not args.no_profile:
        ctx.profile(True)
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        lam, _, st = ctx.mincut(dev=dev, workspace=ws, want_side=False, return_stats=True)
        stats.append(st)
        assert lam0 is None or lam == lam0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    log("timed %d steps: %.3f ms/step, lambda=%d, rounds=%d" % (args.steps, ms, lam, stats[-1]["rounds"]))
    roofline = None
    rounds = None
    if not args.no_profile:
        ctx.profile(False)
        rounds = [round_record(r) for r in ctx.profile_rounds()]
        for r in rounds:
            log("  round %-6s n %9d -> %9d  edges %10d -> %10d  %7.3f ms  %6.2f G edges/s  %7.1f GB/s algorithmic" % (
                r["kind"], r["n"], r["n_out"], r["m"], r["m_out"], r["ms"], r["edges_per_s"] / 1e9, r["alg_gbps"]))
        kt = ctx.profile_read()
        for name, r in sorted(kt.items(), key=lambda kv: -kv[1]["ms"]):
            if r["launches"]:
                log("  %-16s %4d launches/step %8.3f ms/step  avg %8.1f us  %7.1f GB/s algorithmic" % (
                    name, r["launches"] // args.steps, r["ms"] / args.steps, 1000.0 * r["ms"] / r["launches"],
                    r["bytes"] / (r["ms"] * 1e6) if r["ms"] > 0 else 0.0))
        name, r = max(kt.items(), key=lambda kv: kv[1]["ms"])
        achieved = r["bytes"] / (r["ms"] * 1e6)          # GB/s = bytes per launch / avg launch time
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_for(name, args.workload),
                    "kernel": name, "launches_per_step": r["launches"] / args.steps,
                    "avg_launch_us": 1000.0 * r["ms"] / r["launches"],
                    "bytes_per_launch": r["bytes"] / r["launches"],
                    "kernel_ms_per_step": r["ms"] / args.steps}

    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device=ctx.device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB device to device" % args.calibrate_copy)
        del src, dst

    golden = {}
    gpath = os.path.join(ROOT, "tests", "golden", "lambda.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    if key in golden:
        assert golden[key]["lambda"] == lam, ("lambda differs from the oracle's", lam, golden[key])

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        lam_cpu, _ = oracle.noi(g)
        tc = time.perf_counter() - t
        assert lam_cpu == lam
        cpu = {"value": g.m / tc, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "full workload, one NOI solve (repeated full CAPFOREST + contraction), %.1f s" % tc}

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
        "config": {"workload": wname, "n": g.n, "m": g.m, "lambda": lam,
                   "rounds": stats[-1]["rounds"], "heuristic_levels": stats[-1]["heuristic_levels"]},
        "roofline": roofline,
        "rounds": rounds,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def round_record(r):
    """One round of the last timed solve: undirected edges in and out,
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


if __name__ == "__main__":
    main()

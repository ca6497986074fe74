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

Prints one JSON line. --gpus > 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


PEAK_HBM_GBS = 8000.0   # MI355X HBM3E peak


def traffic_for(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size),
    or None when there is none or its kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=22)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--passes", type=int, default=0)
    ap.add_argument("--len-cap", type=int, default=0)
    ap.add_argument("--no-profile", action="store_true", help="time the steps without kernel events")
    ap.add_argument("--heuristic-min-n", type=int, default=10000,
                    help="run the label-propagation bound on graphs with at least this many vertices (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the solver has no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_2609_07204_amd as mc

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t = time.time()
    g = gen.config_chung_lu(args.log2n, args.seed)
    log("generated %s: n=%d m=%d in %.1fs" % (g.name, g.n, g.m, time.time() - t))
    ctx = mc.Context(0, capforest_passes=args.passes, pass_len_cap=args.len_cap,
                     heuristic_min_n=args.heuristic_min_n)
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
    if not args.no_profile:
        ctx.profile(False)
        kt = ctx.profile_read()
        for name, r in sorted(kt.items(), key=lambda kv: -kv[1]["ms"]):
            if r["launches"]:
                log("  %-16s %4d launches/step %8.3f ms/step  avg %8.1f us  %7.1f GB/s algorithmic" % (
                    name, r["launches"] // args.steps, r["ms"] / args.steps, 1000.0 * r["ms"] / r["launches"],
                    r["bytes"] / (r["ms"] * 1e6) if r["ms"] > 0 else 0.0))
        name, r = max(kt.items(), key=lambda kv: kv[1]["ms"])
        achieved = r["bytes"] / (r["ms"] * 1e6)          # GB/s = bytes per launch / avg launch time
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_for(name),
                    "kernel": name, "launches_per_step": r["launches"] / args.steps,
                    "avg_launch_us": 1000.0 * r["ms"] / r["launches"],
                    "bytes_per_launch": r["bytes"] / r["launches"],
                    "kernel_ms_per_step": r["ms"] / args.steps}

    golden = {}
    gpath = os.path.join(ROOT, "tests", "golden", "lambda.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    key = "chung_lu_2^%d_core10_seed%d" % (args.log2n, args.seed)
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
        "config": {"workload": "chung_lu n=2^%d beta=2.5 avg_deg=20 10-core LCC unit weights seed=%d"
                               % (args.log2n, args.seed), "n": g.n, "m": g.m, "lambda": lam,
                   "rounds": stats[-1]["rounds"], "heuristic_levels": stats[-1]["heuristic_levels"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

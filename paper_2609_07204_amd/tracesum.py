"""Summary of a rocprofv3 kernel trace of bench.py, per solve.

Every solve starts with the normal-form check `k_canon` (which also checks a
device input), so the trace is split into solves at each launch of that
kernel (the batched form launches it once per batch). The summary gives every solve's GPU span
(first kernel start to last kernel end before the next solve) and, over a
chosen range of solves, every kernel's launches, total and average time,
followed by rocprofv3's own statistics over the whole run.

    python -m paper_2609_07204_amd.tracesum TRACE_DIR FIRST LAST [TITLE]

FIRST and LAST (inclusive) number the solves from 0 in trace order.
Prints markdown on stdout.
"""
import csv
import glob
import os
import sys

MARKER = "k_canon"


def short(name):
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0].strip()


def load(trace_dir):
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_trace.csv under %s" % trace_dir)
    rows = []
    for f in files:
        for r in csv.DictReader(open(f)):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"])))
    rows.sort()
    return rows


def split_solves(rows):
    """[(start index, end index)) of each solve in the sorted rows."""
    starts = [i for i, r in enumerate(rows) if r[2] == MARKER]
    return [(a, starts[k + 1] if k + 1 < len(starts) else len(rows)) for k, a in enumerate(starts)]


def per_kernel(rows, spans):
    tot = {}
    for a, b in spans:
        for s, e, name in rows[a:b]:
            t = tot.setdefault(name, [0, 0.0])
            t[0] += 1
            t[1] += (e - s) / 1e6   # ms
    return tot


def stats_table(trace_dir, top=20):
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        return []
    out = []
    for r in csv.DictReader(open(files[0])):
        out.append((short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                    float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    out.sort(key=lambda x: -x[2])
    return out[:top]


def main(trace_dir, first, last, title="Kernel trace"):
    rows = load(trace_dir)
    solves = split_solves(rows)
    first, last = int(first), int(last)
    chosen = solves[first:last + 1]
    lines = ["# %s" % title, ""]
    lines.append("Solves found (split at `%s`): %d. Per-solve GPU span (first kernel start to last kernel end), "
                 "ms:" % (MARKER, len(solves)))
    spans_ms = []
    for a, b in solves[: max(last + 1, 0) + 4]:
        spans_ms.append("%.3f" % ((max(r[1] for r in rows[a:b]) - rows[a][0]) / 1e6))
    lines.append(", ".join(spans_ms))
    lines.append("")
    tot = per_kernel(rows, chosen)
    launches = sum(v[0] for v in tot.values())
    ksum = sum(v[1] for v in tot.values())
    lines.append("## Solves %d to %d: kernel time by kernel, per solve (%d launches per solve, kernel sum %.3f ms "
                 "per solve)" % (first, last, launches // max(1, len(chosen)), ksum / max(1, len(chosen))))
    lines.append("")
    lines.append("| kernel | launches per solve | ms per solve | avg us |")
    lines.append("|---|---:|---:|---:|")
    for name, (c, ms) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:30]:
        lines.append("| %s | %.1f | %.3f | %.1f |" % (name, c / len(chosen), ms / len(chosen), 1000.0 * ms / c))
    st = stats_table(trace_dir)
    if st:
        lines += ["", "## rocprofv3 --stats over the whole run (top 20 by total time)", "",
                  "| kernel | calls | total ms | avg us | percent |", "|---|---:|---:|---:|---:|"]
        for name, calls, ms, avg, pct in st:
            lines.append("| %s | %d | %.2f | %.1f | %.2f |" % (name, calls, ms, avg, pct))
    print("\n".join(lines))


if __name__ == "__main__":
    if len(sys.argv) < 4:
        raise SystemExit(__doc__)
    main(*sys.argv[1:5])

"""HBM traffic per launch of the timed kernels, from two rocprofv3 counter
runs of bench.py (FETCH_SIZE, then WRITE_SIZE, with --calibrate-copy MIB).

The counters are scaled by what they read for the calibration copy, a
device-to-device copy of known size (MIB MiB read and MIB MiB written), so
the result is in bytes. Writes profiles/traffic.json: for every kernel, the
average bytes per launch, the factors, and the SHA-256 of the source file
that holds the kernel (bench.py reports the figure only while that file is
unchanged).

    python -m paper_2609_07204_amd.traffic FETCH_DIR WRITE_DIR MIB [WORKLOAD]

WORKLOAD (default chung_lu) is the bench.py workload the counter runs
measured; bench.py reports the figure for that workload only.
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)

def kernel_sources():
    """{kernel name: source file relative to the repository root} for every
    __global__ function under csrc/."""
    out = {}
    d = os.path.join(PKG, "csrc")
    for f in sorted(glob.glob(os.path.join(d, "*.hip"))):
        rel = os.path.relpath(f, ROOT)
        for m in re.finditer(r"__global__\s+(?:__launch_bounds__\([^)]*\)\s+)?void\s+(k_\w+)\s*\(", open(f).read()):
            out.setdefault(m.group(1), rel)
    return out


def per_kernel(d, counter):
    """{short kernel name: [values per dispatch]} from a rocprofv3 counter
    collection directory."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    out = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0].strip()
            if name.startswith("void "):   # template instances are named with their return type
                name = name[5:]
            out.setdefault(name, []).append(float(r["Counter_Value"]))
    return out


def main(fetch_dir, write_dir, mib, workload="rhg", path=None):
    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k or "copy" in k.lower()]
    if not copy:
        raise SystemExit("no copy kernel among the dispatches")
    ck = max(copy, key=lambda k: max(fetch[k]))
    nbytes = float(mib) * (1 << 20)
    f_fetch = nbytes / max(fetch[ck])             # bytes per counter unit
    f_write = nbytes / max(write.get(ck, [0.0]) or [1.0])
    res = {"_calibration": {"copy_kernel": ck, "copy_bytes": nbytes, "fetch_factor": f_fetch,
                            "write_factor": f_write, "workload": workload}}
    srcs = kernel_sources()
    for k in sorted(fetch):
        # a template's dispatches are named with their arguments (k_x<2048>)
        src = srcs.get(k.split("<")[0])
        if src is None or k not in write:
            continue
        fb = sum(fetch[k]) / len(fetch[k]) * f_fetch
        wb = sum(write[k]) / len(write[k]) * f_write
        res[k] = {"bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                  "launches": len(fetch[k]), "source": src,
                  "source_sha256": hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()}
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    tab = json.load(open(path)) if os.path.exists(path) else {}
    tab[workload] = res
    json.dump(tab, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps(res, indent=1, sort_keys=True))
    return res


if __name__ == "__main__":
    main(*sys.argv[1:5])

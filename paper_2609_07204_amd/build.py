"""Build libmincut.so (HIP for gfx950) in-tree with hipcc.

Every translation unit under csrc/ is compiled for gfx950 only, with packed
FP32 instructions disabled (-Xclang -target-feature -Xclang -packed-fp32-ops),
and linked into one shared library with a plain C ABI (include/mincut.h,
include/mincut_steps.h).
"""
import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmincut.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["mc_host.cpp", "mc_scan.hip", "mc_finish.hip", "mc_contract.hip", "mc_sort.hip", "mc_graph_ops.hip", "mc_capforest.hip",
           "mc_capforest_private.hip", "mc_capforest_steps.hip", "mc_heuristic.hip", "mc_batch.hip", "mc_solver.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "feature flag" not in l and l.strip())
    return src, p.returncode, out, obj


def build(verbose=False):
    """Compile every source and link libmincut.so. Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = []
    for src, rc, out, obj in results:
        if verbose and out:
            print(out, file=sys.stderr)
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, out))
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    p = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Write expected minimum cuts of the seeded workloads, computed by the CPU
oracle only (never by the GPU path). Run: python tests/golden/make_golden.py
[names...]. Output: tests/golden/lambda.json."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402

WORKLOADS = {
    "planted_2x1000_seed1": lambda: gen.config_planted_2x1000(1),
    "chung_lu_2^22_core10_seed1": lambda: gen.config_chung_lu(22, 1),
    "chung_lu_2^20_core10_seed1": lambda: gen.config_chung_lu(20, 1),
    "rhg_2^20_core32_seed1": lambda: gen.config_rhg(20, 1),
    "rhg_2^23_core32_seed1": lambda: gen.config_rhg(23, 1),
}
# graphs of the served pool (m log-uniform in [1e3, 1e7], weights 1-1000):
# the three heaviest Erdos-Renyi ones, four with n >= 65536, small ones of
# each family and mid-size ones
SERVED_POOL = [13, 145, 178, 66, 22, 248, 150, 147, 226, 131, 211, 104]
for _j in SERVED_POOL:
    WORKLOADS["served_pool_%d" % _j] = (lambda j: lambda: gen.config_served_graph(j))(_j)


def main(names):
    path = os.path.join(HERE, "lambda.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    for name in names or list(WORKLOADS):
        t = time.time()
        g = WORKLOADS[name]()
        tg = time.time() - t
        t = time.time()
        lam, side = oracle.noi(g) if g.n > 3000 else oracle.stoer_wagner(g)
        assert oracle.cut_value(g, side) == lam
        data[name] = {"lambda": lam, "n": g.n, "m": g.m, "oracle": "noi" if g.n > 3000 else "stoer_wagner",
                      "oracle_seconds": round(time.time() - t, 2), "gen_seconds": round(tg, 2)}
        print(name, data[name], flush=True)
        json.dump(data, open(path, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])

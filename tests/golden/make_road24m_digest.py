"""Writes road24m_digest.json: the oracle's contraction hierarchy of the
clustered road-like 24M-vertex graph (seed 0, default labels of seed 0,
exact witness searches, plain priority), as an order-independent digest.

Calls only the oracle and the seeded input generator; a full oracle build
of this graph takes tens of minutes on one core and about 30 GB of memory.

    python tests/golden/make_road24m_digest.py [out.json]
"""
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
from paper_2412_18008_amd import synth  # noqa: E402
from ch_digest import digest  # noqa: E402


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main(out):
    oracle.build()
    t0 = time.time()
    off, dst, w = synth.config_road24m(seed=0)
    print(f"generated n={len(off) - 1} m={len(dst)} in {time.time() - t0:.0f} s", flush=True)
    t1 = time.time()
    o = oracle.OracleCH(off, dst, w, seed=0)
    while o.round():
        if o.rounds % 20 == 0:
            print(f"round {o.rounds}: {o.alive_count} alive, {time.time() - t1:.0f} s",
                  flush=True)
    o.finish()
    build_s = time.time() - t1
    print(f"oracle build {build_s:.0f} s, {o.rounds} rounds", flush=True)
    vs = o.vertex_state()
    up, dn = o.up(), o.down()
    rs = o.round_stats()
    d = digest(vs["level"], vs["pc"], o.rank(),
               (up["tail"], up["head"], up["w"], up["mid"]),
               (dn["tail"], dn["head"], dn["w"], dn["mid"]), rs)
    d["m"] = int(len(dst))
    d["shortcuts"] = int(sum(r["n_shortcuts"] for r in rs))
    d["oracle_build_s"] = round(build_s, 1)
    d["host"] = {"cpu": cpu_model(), "nproc": os.cpu_count(), "threads_used": 1,
                 "date": time.strftime("%Y-%m-%d")}
    d["workload"] = ("clustered road-like 24M: 24,000,000 points (64 Gaussian cities, 70% of "
                     "the points, 30% uniform), 3-nearest-neighbour edges symmetrised, "
                     "travel-time weights, 10% one-way, seed 0")
    with open(out, "w") as f:
        json.dump(d, f, indent=1)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "road24m_digest.json"))

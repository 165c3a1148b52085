"""Autotuner for the speed knobs of ch_build and ch_query_batch.

Build knobs (``ch_params_t``): the first-tier witness-search kernel (lanes
per source x LDS table slots) for sparse and for dense rounds, the average
out-degree that separates the two, the lanes per item of the other round
kernels, and the overlay size below which exact-mode searches use the
all-pairs table (``dense_tail``), and the distance-bucket width of an
exact-mode search step (``ls_step``).  Query knobs (flags of ch_query_batch): the
waves per query of the first query tier and the level window.  None of them
may change the result: every build configuration tried must give a CH
identical to the default one and every query configuration the same
distances; a configuration that differs is an error, not a candidate.  The
build knobs are tuned one at a time from the default (coordinate descent),
then the query knobs on the tuned CH.

The best configuration per size class (graph size and average degree) is
kept in a JSON cache: ``$SPOCH_AUTOTUNE_CACHE`` if set, else
``tuned.json`` next to this file.

Usage: ``python -m paper_2412_18008_amd.autotune --workload road1m``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")
KNOBS = ("ls_sparse", "ls_dense", "dense_deg10", "group", "dense_tail", "ls_step")
QUERY_KNOBS = ("waves", "window")
# values tried per knob (0 = the library's default)
# (dense_tail 1 = off: no all-pairs table)
CHOICES = {"ls_sparse": (0, 2, 3), "ls_dense": (0, 1, 2, 3), "dense_deg10": (0, 40, 70),
           "group": (0, 8, 16, 32), "dense_tail": (0, 1, 2048, 4096), "ls_step": (0, 1, 2, 5, 32)}
QUERY_CHOICES = {"waves": (0, 1, 2, 8), "window": (0, 16, 48, 128)}


def cache_path():
    return os.environ.get("SPOCH_AUTOTUNE_CACHE", DEFAULT_CACHE)


def size_class(n, m):
    """Graphs within a factor ~1.4 in size and 0.5 in average degree share a class."""
    d = m / n if n else 0.0
    return f"n2^{round(math.log2(max(n, 1)) * 2) / 2:g}_deg{round(d * 2) / 2:g}"


def load(path=None):
    path = path or cache_path()
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(entries, path=None):
    path = path or cache_path()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def params_for(n, m, path=None):
    """Tuned build knobs for a graph of n vertices and m arcs ({} if none)."""
    e = load(path).get(size_class(n, m))
    return {k: e["params"][k] for k in KNOBS if k in e["params"]} if e else {}


def query_params_for(n, m, path=None):
    """Tuned query knobs (waves, window) for the size class ({} if none)."""
    e = load(path).get(size_class(n, m))
    q = e.get("query") if e else None
    return {k: q["params"][k] for k in QUERY_KNOBS} if q else {}


def _digest(ch):
    """SHA-256 over the exported CH (level, score, rank, both arc lists)."""
    import hashlib

    e = ch.export()
    h = hashlib.sha256()
    for k in sorted(e):
        h.update(k.encode())
        h.update(np.ascontiguousarray(e[k]).view(np.uint8))
    return h.hexdigest()


def tune(off, dst, w, qs, qt, reps=2, log=print):
    """Coordinate descent over the build knobs from the default (median of
    `reps` device-resident builds per configuration), then the query knobs on
    the tuned CH (median of `reps` batches).  Returns (best build knobs and
    time, best query knobs and time, table).  Raises if a configuration
    changes the CH or a distance."""
    import torch

    from . import binding

    dev = torch.device("cuda:0")
    t_off = torch.from_numpy(np.asarray(off, np.int64)).to(dev)
    t_dst = torch.from_numpy(np.asarray(dst, np.int64).astype(np.int32)).to(dev)
    t_w = torch.from_numpy(np.asarray(w, np.int64).astype(np.int32)).to(dev)
    t_s = torch.from_numpy(np.asarray(qs, np.int64).astype(np.int32)).to(dev)
    t_t = torch.from_numpy(np.asarray(qt, np.int64).astype(np.int32)).to(dev)
    ref = None
    table = []
    seen = {}

    def run(c):
        key = tuple(sorted(c.items()))
        if key in seen:
            return seen[key]
        nonlocal ref
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch = binding.build(t_off, t_dst, t_w, **c)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            dig = _digest(ch)
            ch.free()
            if ref is None:
                ref = dig
            elif dig != ref:
                raise RuntimeError(f"configuration {c} changed the CH")
        ms = float(np.median(times)) * 1e3
        table.append(dict(params=dict(c), ms=ms))
        log(f"[autotune] build {c} -> {ms:.1f} ms")
        seen[key] = ms
        return ms

    cur = {k: 0 for k in KNOBS}
    best_ms = run(cur)
    for k in KNOBS:
        for v in CHOICES[k]:
            c = dict(cur, **{k: v})
            ms = run(c)
            if ms < best_ms:
                best_ms, cur = ms, c
    # queries on the CH of the tuned knobs
    ch = binding.build(t_off, t_dst, t_w, **cur)
    dref = ch.query(t_s, t_t).cpu().numpy()
    qbest, qbest_ms = {"waves": 0, "window": 0}, None
    qtable = []
    for wv in QUERY_CHOICES["waves"]:
        for win in QUERY_CHOICES["window"]:
            times = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                d = ch.query(t_s, t_t, waves=wv, window=win)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                if not np.array_equal(d.cpu().numpy(), dref):
                    raise RuntimeError(f"query waves={wv} window={win} changed a distance")
            ms = float(np.median(times)) * 1e3
            qtable.append(dict(params=dict(waves=wv, window=win), ms=ms))
            log(f"[autotune] query waves={wv} window={win} -> {ms:.1f} ms")
            if qbest_ms is None or ms < qbest_ms:
                qbest, qbest_ms = dict(waves=wv, window=win), ms
    ch.free()
    return dict(params=cur, ms=best_ms), dict(params=qbest, ms=qbest_ms, table=qtable), table


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="road1m",
                    choices=("road1m", "grid64", "road24m", "road100k", "knn5"))
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--queries", type=int, default=100_000)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    from . import synth

    g = {"road1m": lambda: synth.config_road1m(0), "grid64": lambda: synth.config_grid64(0),
         "road24m": lambda: synth.config_road24m(0),
         "road100k": lambda: synth.road_like(100_000, seed=0),
         "knn5": lambda: synth.knn_graph(1_000_000, 5, seed=5)}[args.workload]()
    off, dst, w = g
    n, m = len(off) - 1, len(dst)
    qs, qt = synth.queries(n, args.queries, seed=3)
    best, qbest, table = tune(off, dst, w, qs, qt, reps=args.reps)
    entries = load(args.cache)
    entries[size_class(n, m)] = dict(params=best["params"], ms=best["ms"], workload=args.workload,
                                     n=n, m=m, table=table, query=qbest,
                                     date=time.strftime("%Y-%m-%d"))
    save(entries, args.cache)
    print(json.dumps(dict(size_class=size_class(n, m), best=best, query=qbest["params"],
                          query_ms=qbest["ms"])))
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Autotuner for the speed knobs of ch_build.

The knobs (``ch_params_t``): the first-tier witness-search kernel (lanes per
source x LDS table slots) for sparse and for dense rounds, the average
out-degree that separates the two, and the lanes per item of the other round
kernels.  None of them may change the result: every configuration tried is
checked to give a CH identical to the default one, and a configuration that
differs is an error, not a candidate.

The best configuration per size class (graph size and average degree) is
kept in a JSON cache: ``$SPOCH_AUTOTUNE_CACHE`` if set, else
``tuned.json`` next to this file.

Usage: ``python -m paper_2412_18008_amd.autotune --workload road1m``.
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")
KNOBS = ("ls_sparse", "ls_dense", "dense_deg10", "group")


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
    """Tuned knobs for a graph of n vertices and m arcs ({} if none)."""
    e = load(path).get(size_class(n, m))
    return {k: e["params"][k] for k in KNOBS} if e else {}


def candidates(full=False):
    """The configurations tried (the default first)."""
    out = [dict(ls_sparse=0, ls_dense=0, dense_deg10=0, group=0)]
    sparse = (1, 2, 3) if full else (1, 2)
    dense = (2, 3, 4) if full else (3, 4)
    thr = (40, 50, 70) if full else (50, 70)
    for a, b, t in itertools.product(sparse, dense, thr):
        out.append(dict(ls_sparse=a, ls_dense=b, dense_deg10=t, group=0))
    out.append(dict(ls_sparse=1, ls_dense=4, dense_deg10=50, group=16))
    out.append(dict(ls_sparse=1, ls_dense=4, dense_deg10=50, group=64))
    return out


def _export_digest(ch):
    e = ch.export()
    h = 0
    for k in sorted(e):
        h = hash((h, k, e[k].tobytes()))
    return h


def tune(off, dst, w, reps=2, full=False, log=print):
    """Times every candidate (median of `reps` builds, device-resident input)
    and returns (best knobs, table).  Raises if a candidate changes the CH."""
    import torch

    from . import binding

    dev = torch.device("cuda:0")
    t_off = torch.from_numpy(np.asarray(off, np.int64)).to(dev)
    t_dst = torch.from_numpy(np.asarray(dst, np.int64).astype(np.int32)).to(dev)
    t_w = torch.from_numpy(np.asarray(w, np.int64).astype(np.int32)).to(dev)
    ref = None
    table = []
    for c in candidates(full):
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch = binding.build(t_off, t_dst, t_w, **c)
            times.append(time.perf_counter() - t0)
            dig = _export_digest(ch)
            ch.free()
            if ref is None:
                ref = dig
            elif dig != ref:
                raise RuntimeError(f"configuration {c} changed the CH")
        ms = float(np.median(times)) * 1e3
        table.append(dict(params=c, ms=ms))
        log(f"[autotune] {c} -> {ms:.1f} ms")
    best = min(table, key=lambda r: r["ms"])
    return best, table


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="road1m", choices=("road1m", "grid64", "road24m",
                                                             "road100k"))
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    from . import synth

    g = {"road1m": lambda: synth.config_road1m(0), "grid64": lambda: synth.config_grid64(0),
         "road24m": lambda: synth.config_road24m(0),
         "road100k": lambda: synth.road_like(100_000, seed=0)}[args.workload]()
    off, dst, w = g
    n, m = len(off) - 1, len(dst)
    best, table = tune(off, dst, w, reps=args.reps, full=args.full)
    entries = load(args.cache)
    entries[size_class(n, m)] = dict(params=best["params"], ms=best["ms"], workload=args.workload,
                                     n=n, m=m, table=table)
    save(entries, args.cache)
    print(json.dumps(dict(size_class=size_class(n, m), best=best)))
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python3
"""Benchmark of the GPU contraction-hierarchy build and query batch.

One step = the whole path on one synthetic graph already resident in HBM:
ch_build (ingest, every contraction round, postprocessing) followed by one
ch_query_batch of the workload's queries.  Prints one JSON line.

The dominant kernel is the fast-path witness search (k_local_search); its
achieved bandwidth is the algorithmic bytes it must move (8 B per adjacency
row's offset pair, 8 B per arc read, 16 B per memo slot read or written),
counted on the device, divided by its HIP-event time on the build stream.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


WORKLOADS = {
    "road1m": dict(
        desc=("road-like 1M: 1,000,000 uniform points in the unit square, edges to the "
              "3 nearest neighbours symmetrised, weight round(1e4*length)+1, 10% of "
              "edges one-way, seed 0; 100,000 uniform s-t queries, seed 3"),
        queries=100_000),
    "grid64": dict(
        desc=("64x64 grid, 4-neighbour arcs both ways, uint32 weights uniform in "
              "[1,1000], seed 0; 1,000 uniform s-t queries, seed 1"),
        queries=1_000),
    "road24m": dict(
        desc=("clustered road-like 24M: 64 Gaussian cities + 30% uniform points, "
              "3-NN symmetrised, travel-time weights by length quartile speed class, "
              "10% one-way, seed 0; 1,000,000 uniform s-t queries, seed 3"),
        queries=1_000_000),
}


def make_graph(name):
    from paper_2412_18008_amd import synth

    if name == "road1m":
        g = synth.config_road1m(seed=0)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=3)
    elif name == "grid64":
        g = synth.config_grid64(seed=0)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=1)
    else:
        g = synth.config_road24m(seed=0)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=3)
    return g, q


def ls_bytes(r):
    return 8 * r["rows_expanded"] + 8 * r["arcs_scanned"] + 16 * r["memo_probes"] + \
        16 * r["memo_inserts"]


def cpu_baseline(g, budget_note):
    """The oracle (plain sequential C) timed on this host on the same graph."""
    import oracle

    off, dst, w = g
    oracle.build()
    t0 = time.perf_counter()
    o = oracle.OracleCH(off, dst, w, seed=0).run()
    el = time.perf_counter() - t0
    sc = sum(r["n_shortcuts"] for r in o.round_stats())
    return {"value": sc / el, "unit": "shortcuts/s", "cores": 1, "kind": "oracle",
            "sample": f"{budget_note}; oracle build {el:.2f} s, {sc} shortcuts, "
                      f"{o.rounds} rounds, 1 thread on {platform.processor() or 'host CPU'}",
            "build_s": el}


MLP_FLOP_PER_ROW = 2 * (8 * 64 + 64 * 64 + 64)  # multiply-adds of the three layers


def mlp_throughput(binding, w_host, dev, rows=1 << 20, reps=20):
    """GFLOP/s of the learned priority's forward kernel (fp32 and bf16) on
    `rows` device-resident feature vectors, timed with HIP events."""
    import numpy as np
    import torch

    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.rand(rows, 8, generator=g).to(dev)
    w = torch.from_numpy(np.asarray(w_host, np.float32)).to(dev)
    out = {}
    for tag, bf16 in (("fp32", False), ("bf16", True)):
        binding.mlp_forward(x, w, bf16=bf16)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            binding.mlp_forward(x, w, bf16=bf16)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[tag] = {"ms_per_launch": ms, "rows": rows,
                    "gflop_s": rows * MLP_FLOP_PER_ROW / (ms / 1e3) / 1e9}
    return out


def plain_vs_learned(binding, args, t_off, t_dst, t_w, qs, qt, knobs, dev):
    """Same graph and knobs, priority plain vs learned: build time, shortcuts,
    CH arcs, mean vertices visited per query (the two upward search spaces,
    counted by the query kernel) and the number of distances that differ."""
    import numpy as np
    import torch

    wts = np.load(args.learned).astype(np.float32)
    nq = min(len(qs), 20_000)
    rep = {"weights": os.path.basename(args.learned), "queries": nq}
    dist = {}
    for tag, mlp in (("plain", None), ("learned", wts)):
        print(f"[bench] {tag} build for the comparison", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch = binding.build(t_off, t_dst, t_w, seed=0, mlp=mlp, **knobs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d, vis = ch.query_stats(qs[:nq], qt[:nq])
        dist[tag] = d
        sm = ch.summary
        rep[tag] = {"build_s": el, "rounds": sm["rounds"], "shortcuts": sm["shortcuts"],
                    "ch_arcs": sm["up_arcs"] + sm["down_arcs"],
                    "mean_visited_per_query": float(vis.mean())}
        ch.free()
    rep["distance_errors"] = int(np.count_nonzero(dist["plain"] != dist["learned"]))
    rep["mlp_forward"] = mlp_throughput(binding, wts, dev)
    return rep


# Kernel sources whose change invalidates the committed HBM counter totals.
TRAFFIC_SOURCES = ("paper_2412_18008_amd/csrc/search.hpp", "paper_2412_18008_amd/csrc/common.hpp",
                   "paper_2412_18008_amd/csrc/round_kernels.hpp",
                   "paper_2412_18008_amd/csrc/dense_tail.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_local_search_road1m.md")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel):
    """Measured HBM bytes per launch of `kernel` from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or
    None when there is none for it or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("traffic:"):
                k, _, v = line[len("traffic:"):].strip().rpartition("=")
                rec[k.strip()] = v.strip()
    if rec.get("source_hash") != kernel_source_hash() or kernel not in rec:
        return None
    return float(rec[kernel])


def copy_calibration(dev, nbytes):
    """One plain device copy of nbytes (reads nbytes, writes nbytes): the
    reference for scaling the HBM counters of a profiled run."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)  # a streaming kernel: reads nbytes, writes nbytes
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: {nbytes} bytes", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="road1m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--untuned", action="store_true",
                    help="ignore the autotuner cache (default knobs)")
    ap.add_argument("--learned", default=os.path.join(ROOT, "paper_2412_18008_amd",
                                                      "learned_weights.npy"),
                    help="weights (.npy, 4801 float32) of the learned priority; the plain vs "
                         "learned comparison runs after the timed steps when the file exists")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after the steps, copy BYTES once on the device (a reference "
                         "kernel for HBM counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the build is a single-GPU path "
              "(the multi-GPU sharding is described, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2412_18008_amd import binding

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    binding.lib()

    g, (qs, qt) = make_graph(args.workload)
    off, dst, w = g
    n, m = len(off) - 1, len(dst)
    print(f"[bench] workload {args.workload}: n={n} m={m} queries={len(qs)}", file=sys.stderr,
          flush=True)
    t_off = torch.from_numpy(off.astype(np.int64)).to(dev)
    t_dst = torch.from_numpy(dst.astype(np.int32)).to(dev)
    t_w = torch.from_numpy(w.astype(np.int32)).to(dev)
    t_s = torch.from_numpy(qs.astype(np.int32)).to(dev)
    t_t = torch.from_numpy(qt.astype(np.int32)).to(dev)
    torch.cuda.synchronize()

    from paper_2412_18008_amd import autotune

    knobs = {} if args.untuned else autotune.params_for(n, m)
    print(f"[bench] knobs {knobs or 'default'}", file=sys.stderr, flush=True)

    def step():
        tb = time.perf_counter()
        ch = binding.build(t_off, t_dst, t_w, seed=0, stats=True, **knobs)
        tq = time.perf_counter()
        d = ch.query(t_s, t_t)
        te = time.perf_counter()
        rec = dict(build_s=tq - tb, query_s=te - tq, summary=dict(ch.summary),
                   rounds=ch.round_stats(), dist_sum=None)
        ch.free()
        del d
        return rec

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        recs.append(step())
        print(f"[bench] step {i + 1}/{args.steps}: build {recs[-1]['build_s']:.3f} s, "
              f"query {recs[-1]['query_s'] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    shortcuts = recs[-1]["summary"]["shortcuts"]
    build_s = float(np.median([r["build_s"] for r in recs]))
    query_s = float(np.median([r["query_s"] for r in recs]))
    # first-tier witness-search launches, per kernel instance; the roofline
    # is reported for the instance with the largest total time
    per = {}
    for r in recs:
        for x in r["rounds"]:
            # rounds of the device-driven tail have no separately timed
            # search launch (their searches are part of a five-launch round)
            if x["n_sources"] == 0 or x["ls_tier1"] == binding.CH_LS_TAIL:
                continue
            k = binding.LS_KERNELS[x["ls_tier1"]]
            a = per.setdefault(k, [0, 0.0, 0])
            a[0] += 1
            a[1] += x["ms_local_search"]
            a[2] += ls_bytes(x)
    dom = max(per, key=lambda k: per[k][1]) if per else binding.LS_KERNELS[1]
    ls_launches, ls_ms, ls_b = per.get(dom, [0, 0.0, 0])
    achieved = (ls_b / 1e9) / (ls_ms / 1e3) if ls_ms > 0 else 0.0

    line = {
        "metric": "CH build time (s) + shortcuts/s + HBM roofline %, plain priority",
        "value": shortcuts / (ms_per_step / 1e3),
        "unit": "shortcuts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload]["desc"], "n": n, "m": m,
                   "queries": int(len(qs)), "priority": "plain (edge difference)",
                   "wps": "exact, radius D_s", "knobs": knobs or "default"},
        "build_time_s": build_s,
        "query_batch_ms": query_s * 1e3,
        "queries_per_s": len(qs) / query_s,
        "rounds": recs[-1]["summary"]["rounds"],
        "shortcuts": shortcuts,
        "shortcuts_per_build_s": shortcuts / build_s,
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom} (first-tier witness search)",
            "all_first_tier": {k: {"launches": v[0], "ms": v[1], "bytes": v[2]}
                               for k, v in per.items()},
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": committed_traffic(dom),
            "launches": ls_launches,
            "avg_launch_ms": ls_ms / max(ls_launches, 1),
            "algorithmic_bytes_per_launch": ls_b / max(ls_launches, 1),
        },
    }
    if os.path.exists(args.learned):
        line["plain_vs_learned"] = plain_vs_learned(binding, args, t_off, t_dst, t_w, qs, qt,
                                                    knobs, dev)
    if args.copy_calibration:
        copy_calibration(dev, args.copy_calibration)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(g, f"the full {args.workload} build (same graph)")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

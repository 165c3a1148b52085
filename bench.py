#!/usr/bin/env python3
"""Benchmark of the GPU contraction-hierarchy build and query batch.

One step = the whole path on one synthetic graph already resident in HBM:
ch_build (ingest, every contraction round, postprocessing) followed by one
ch_query_batch of the workload's queries.  Prints one JSON line.

Default workload: the clustered road-like 24M graph with a 1M-query batch.
`value` is shortcuts per second of step time (build + query batch).

Rooflines (HBM-bound integer work, 8 TB/s peak):
* `roofline`: the kernel with the most device time per step.  Its achieved
  bandwidth is its algorithmic bytes per launch divided by its average
  launch time (HIP events inside the library, on the build or query
  stream).  Witness searches: 8 B per adjacency row (offset pair), 8 B per
  arc read, 16 B per memo slot read or written, counted on the device.
  Queries: 8 B per vertex expanded (offset pair) + 8 B per arc relaxed,
  counted by the query kernels in one extra (untimed) batch.
* `roofline_wps`: every witness-search launch of the build together (the
  first tier, the block tier and the global tier), the same way.
`traffic` (HBM bytes per launch from rocprofv3 counters) comes from the
committed counter summary of the same workload while the kernel sources
still hash to the recorded value, else null.
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
    "road24m": dict(
        desc=("clustered road-like 24M: 24,000,000 points (64 Gaussian cities with 70% of the "
              "points, 30% uniform), edges to the 3 nearest neighbours symmetrised, "
              "travel-time weights round(1.1e6*length/speed)+1 with the speed class by "
              "length quartile, 10% of edges one-way, seed 0; 1,000,000 uniform s-t "
              "queries, seed 3"),
        queries=1_000_000),
    "road1m": dict(
        desc=("road-like 1M: 1,000,000 uniform points in the unit square, edges to the "
              "3 nearest neighbours symmetrised, weight round(1e4*length)+1, 10% of "
              "edges one-way, seed 0; 100,000 uniform s-t queries, seed 3"),
        queries=100_000),
    "batch512": dict(
        desc=("batched construction: 512 road-like graphs (the road-like 1M recipe), vertex "
              "counts log-uniform in [1e4, 5e5] from PCG64(512) (68,749,675 vertices in all), "
              "graph i from seed i, built by one ch_build_batch; 1,000 uniform s-t queries "
              "per graph"),
        queries=1_000),
    **{f"knn{k}": dict(
        desc=(f"k-NN k={k}: 1,000,000 uniform points in the unit square, arcs from every "
              f"point to its {k} nearest neighbours (m = {k},000,000), weights uniform in "
              f"[1,32], seed {k}; 100,000 uniform s-t queries, seed 3"),
        queries=100_000) for k in (2, 5, 10)},
    "grid64": dict(
        desc=("64x64 grid, 4-neighbour arcs both ways, uint32 weights uniform in "
              "[1,1000], seed 0; 1,000 uniform s-t queries, seed 1"),
        queries=1_000),
}

# bounded CPU sample of each workload for the oracle (same generator)
CPU_SAMPLES = {
    **{f"knn{k}": (f"k-NN k={k} at 50,000 points (seed {k})",
                   lambda synth, k=k: synth.knn_graph(50_000, k, seed=k)) for k in (2, 5, 10)},
    "road24m": ("clustered road-like 1M (the 24M recipe at 1,000,000 points, seed 0)",
                lambda synth: synth.clustered_road(1_000_000, seed=0)),
    "road1m": ("the road-like 1M graph itself", lambda synth: synth.config_road1m(seed=0)),
    "grid64": ("the 64x64 grid itself", lambda synth: synth.config_grid64(seed=0)),
}


def make_graph(name):
    from paper_2412_18008_amd import synth

    if name == "road1m":
        g = synth.config_road1m(seed=0)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=3)
    elif name == "grid64":
        g = synth.config_grid64(seed=0)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=1)
    elif name.startswith("knn"):
        k = int(name[3:])
        g = synth.knn_graph(1_000_000, k, seed=k)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=3)
    else:
        g = synth.config_road24m(seed=0)
        q = synth.queries(len(g[0]) - 1, WORKLOADS[name]["queries"], seed=3)
    return g, q


def ls_bytes(rows, arcs, probes, inserts):
    return 8 * rows + 8 * arcs + 16 * probes + 16 * inserts


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(workload, settle=0):
    """The oracle (plain sequential C, one thread) timed on this host on a
    bounded sample of the workload, plus the committed record of its full
    build of the 24M graph (run once, elsewhere) for context."""
    import oracle
    from paper_2412_18008_amd import synth

    desc, gen = CPU_SAMPLES[workload]
    off, dst, w = gen(synth)
    oracle.build()
    t0 = time.perf_counter()
    o = oracle.OracleCH(off, dst, w, seed=0,
                        **(dict(wps_mode=oracle.WPS_SETTLED, settle_limit=settle)
                           if settle else {})).run()
    el = time.perf_counter() - t0
    sc = sum(r["n_shortcuts"] for r in o.round_stats())
    rep = {"value": sc / el, "unit": "shortcuts/s", "cores": 1, "kind": "oracle",
           "sample": (f"{desc}: n={len(off) - 1}, m={len(dst)}; oracle build {el:.2f} s, "
                      f"{sc} shortcuts, {o.rounds} rounds, 1 thread of {os.cpu_count()} on "
                      f"{cpu_model()}"),
           "build_s": el, "host_cpu": cpu_model(), "host_nproc": os.cpu_count()}
    dig = os.path.join(ROOT, "tests", "golden", "road24m_digest.json")
    if workload == "road24m" and not settle and os.path.exists(dig):
        with open(dig) as f:
            d = json.load(f)
        rep["full_workload_recorded"] = {
            "build_s": d["oracle_build_s"], "shortcuts": d["shortcuts"], "rounds": d["rounds"],
            "shortcuts_per_s": d["shortcuts"] / d["oracle_build_s"], "host": d["host"],
            "note": "the oracle's full build of this workload, recorded once with its output "
                    "digest (tests/golden/road24m_digest.json); another host"}
    return rep


MLP_FLOP_PER_ROW = 2 * (8 * 64 + 64 * 64 + 64)  # multiply-adds of the three layers


def mlp_throughput(binding, w_host, dev, rows=1 << 24, reps=5):
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
        gf = rows * MLP_FLOP_PER_ROW / (ms / 1e3) / 1e9
        peak = 2.5e6 if bf16 else 157.3e3  # GFLOP/s: bf16 MFMA dense, fp32 vector
        out[tag] = {"ms_per_launch": ms, "rows": rows, "gflop_s": gf,
                    "peak_gflop_s": peak, "frac_of_peak": gf / peak}
    # training: 100 Adam steps of 4096 samples (forward, backward, gradient
    # sums, update), host-timed around the whole call
    xt = np.random.default_rng(3).random((1 << 18, 8)).astype(np.float32)
    tt = xt[:, 0].copy()
    for tag, bf16 in (("fp32", False), ("bf16", True)):
        binding.mlp_train(xt, tt, np.asarray(w_host, np.float32), batch=4096, steps=5, bf16=bf16)
        t0 = time.perf_counter()
        binding.mlp_train(xt, tt, np.asarray(w_host, np.float32), batch=4096, steps=100,
                          bf16=bf16)
        out[tag]["train_ms_per_step_4096"] = (time.perf_counter() - t0) * 1e3 / 100
    return out


def plain_vs_learned(binding, args, dev, workload, graph):
    """On `workload` (device tensors off, dst, w and host queries in
    `graph`), priority plain vs learned: build time, rounds, shortcuts, CH
    arcs, mean vertices visited per query (the two upward search spaces,
    counted by the query kernel), the time of a pruned 100k-query batch and
    the number of distances that differ."""
    import numpy as np
    import torch

    from paper_2412_18008_amd import autotune

    t_off, t_dst, t_w, qs, qt = graph
    knobs = autotune.params_for(t_off.numel() - 1, t_dst.numel())
    wts = np.load(args.learned).astype(np.float32)
    nq = min(len(qs), 20_000)
    nb = min(len(qs), 100_000)
    ts = torch.from_numpy(qs[:nb].astype(np.int32)).to(dev)
    tt = torch.from_numpy(qt[:nb].astype(np.int32)).to(dev)
    rep = {"graph": WORKLOADS[workload]["desc"], "workload": workload,
           "weights": os.path.basename(args.learned), "queries": nq}
    dist = {}
    for tag, mlp in (("plain", None), ("learned", wts)):
        print(f"[bench] {tag} build for the comparison", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch = binding.build(t_off, t_dst, t_w, seed=0, mlp=mlp, progress=True, **knobs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d, vis = ch.query_stats(qs[:nq], qt[:nq])
        dist[tag] = d
        ch.query(ts, tt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.query(ts, tt)
        torch.cuda.synchronize()
        qms = (time.perf_counter() - t0) * 1e3
        sm = ch.summary
        rep[tag] = {"build_s": el, "rounds": sm["rounds"], "shortcuts": sm["shortcuts"],
                    "ch_arcs": sm["up_arcs"] + sm["down_arcs"],
                    "mean_visited_per_query": float(vis.mean()),
                    f"query_batch_{nb}_ms": qms}
        ch.free()
        print(f"[bench] {tag}: {rep[tag]}", file=sys.stderr, flush=True)
    rep["distance_errors"] = int(np.count_nonzero(dist["plain"] != dist["learned"]))
    rep["mlp_forward"] = mlp_throughput(binding, wts, dev)
    return rep


# Kernel sources whose change invalidates the committed HBM counter totals.
TRAFFIC_SOURCES = ("paper_2412_18008_amd/csrc/search.hpp", "paper_2412_18008_amd/csrc/common.hpp",
                   "paper_2412_18008_amd/csrc/round_kernels.hpp",
                   "paper_2412_18008_amd/csrc/dense_tail.hpp",
                   "paper_2412_18008_amd/csrc/post.hip")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(workload, kernel):
    """Measured HBM bytes per launch of `kernel` on `workload` from the
    committed counter summary profiles/pmc_<workload>.md (FETCH_SIZE +
    WRITE_SIZE, calibrated against a plain copy), or None when there is no
    record for that workload and kernel or the kernel sources changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("traffic:"):
                k, _, v = line[len("traffic:"):].strip().rpartition("=")
                rec[k.strip()] = v.strip()
    if rec.get("workload") != workload or rec.get("source_hash") != kernel_source_hash():
        return None
    if kernel not in rec:
        return None
    return float(rec[kernel])


def query_sizes(ch, qs, qt, dev, sizes=(1, 1000, 10_000, 100_000, 1_000_000), qknobs=None):
    """Latency and throughput of one ch_query_batch call per batch size
    (device-resident s, t; the median of 5 calls after one warm-up call,
    each timed from launch to completion on the host)."""
    import numpy as np
    import torch

    out = {}
    for k in sizes:
        k = min(k, len(qs))
        s = torch.from_numpy(qs[:k].astype(np.int32)).to(dev)
        t = torch.from_numpy(qt[:k].astype(np.int32)).to(dev)
        ch.query(s, t, **(qknobs or {}))
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            ch.query(s, t, **(qknobs or {}))
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = float(np.median(ts)) * 1e3
        out[str(k)] = {"latency_ms": ms, "queries_per_s": k / (ms / 1e3)}
    return out


def hbm_probe(dev, nbytes=1 << 30, gathers=1 << 26):
    """Practical HBM rates on this GPU: a streaming kernel (reads and writes
    nbytes) and a scattered one (`gathers` random 8-byte reads from a 2 GiB
    array, with their indices read and results written in order), each the
    median of 5 runs timed with events.  The scattered kernel is also the
    check of the counter calibration: its FETCH_SIZE per launch, scaled like
    the search kernels', should be near its 64-byte lines touched plus the
    index bytes."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    src = torch.arange((2 << 30) // 8, dtype=torch.int64, device=dev)
    g = torch.Generator(device=dev).manual_seed(11)
    idx = torch.randint(0, src.numel(), (gathers,), device=dev, generator=g)
    out = torch.empty(gathers, dtype=torch.int64, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return sorted(ms)[2]

    ms_s = timed(lambda: torch.neg(a, out=b))
    ms_g = timed(lambda: torch.index_select(src, 0, idx, out=out))
    stream_gbs = 2 * nbytes / (ms_s / 1e3) / 1e9
    useful = gathers * (8 + 8 + 8)  # value, index, result
    lines = gathers * (64 + 8 + 8)   # a 64-byte line per random read
    return {"stream": {"bytes": 2 * nbytes, "ms": ms_s, "gbs": stream_gbs,
                       "frac_of_peak": stream_gbs / HBM_PEAK_GBS},
            "scattered_8B": {"gathers": gathers, "ms": ms_g,
                             "useful_gbs": useful / (ms_g / 1e3) / 1e9,
                             "line_gbs": lines / (ms_g / 1e3) / 1e9,
                             "gathers_per_s": gathers / (ms_g / 1e3)}}


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


QUERY_KERNELS = ("k_query<4, QTier1>", "k_query<16, QTier2>", "k_query<8, QTier3>",
                 "k_query_global")
BLK_KERNEL = "k_local_search_blk<8192>"
GLOBAL_KERNEL = "k_local_search_global"


def search_kernels(binding, recs):
    """Per witness-search kernel over the timed steps: launches, device ms,
    algorithmic bytes (rounds of the device-driven tail have no separately
    timed search launch and are left out)."""
    per = {}

    def add(k, ms, b):
        a = per.setdefault(k, [0, 0.0, 0])
        a[0] += 1
        a[1] += ms
        a[2] += b

    for r in recs:
        for x in r["rounds"]:
            if x["n_sources"] == 0 or x["ls_tier1"] == binding.CH_LS_TAIL:
                continue
            add(binding.LS_KERNELS[x["ls_tier1"]], x["ms_local_search"],
                ls_bytes(x["rows_expanded"], x["arcs_scanned"], x["memo_probes"],
                         x["memo_inserts"]))
            if x["ms_ls_blk"] > 0:
                add(BLK_KERNEL, x["ms_ls_blk"],
                    ls_bytes(x["rows2"], x["arcs2"], x["probes2"], x["inserts2"]))
            if x["n_ls_global"]:
                add(GLOBAL_KERNEL, x["ms_ls_global"],
                    ls_bytes(x["rows3"], x["arcs3"], x["probes3"], x["inserts3"]))
    return per


def roofline_obj(workload, name, launches, ms, nbytes, bound_note):
    achieved = (nbytes / 1e9) / (ms / 1e3) if ms > 0 else 0.0
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": committed_traffic(workload, name),
            "launches": launches, "avg_launch_ms": ms / max(launches, 1),
            "algorithmic_bytes_per_launch": nbytes / max(launches, 1), "units": bound_note}


def bench_batch512(args, binding, dev):
    """ch_build_batch of the 512-graph workload plus a 1000-query batch per
    graph as one step; aggregate shortcuts/s over the step and over the
    batched build, and per-graph shortcuts/s of each graph built alone."""
    import numpy as np
    import torch

    from paper_2412_18008_amd import synth

    t_gen = time.perf_counter()
    graphs = synth.config_batch512()
    sizes = np.array([len(g[0]) - 1 for g in graphs])
    print(f"[bench] batch512: {len(graphs)} graphs, {int(sizes.sum())} vertices "
          f"(generated in {time.perf_counter() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    dgraphs = [(torch.from_numpy(o.astype(np.int64)).to(dev),
                torch.from_numpy(d.astype(np.int32)).to(dev),
                torch.from_numpy(w.astype(np.int32)).to(dev)) for o, d, w in graphs]
    queries = []
    for i, n in enumerate(sizes):
        s, t = synth.queries(int(n), 1000, seed=i)
        queries.append((torch.from_numpy(s.astype(np.int32)).to(dev),
                        torch.from_numpy(t.astype(np.int32)).to(dev)))
    torch.cuda.synchronize()

    def step():
        tb = time.perf_counter()
        chs = binding.build_batch(dgraphs)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        for c, (s, t) in zip(chs, queries):
            c.query(s, t)
        torch.cuda.synchronize()
        te = time.perf_counter()
        sc = [c.summary["shortcuts"] for c in chs]
        for c in chs:
            c.free()
        return tq - tb, te - tq, sc

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    recs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        recs.append(step())
        print(f"[bench] step {i + 1}/{args.steps}: batch build {recs[-1][0]:.3f} s, "
              f"queries {recs[-1][1] * 1e3:.0f} ms", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    sc = np.array(recs[-1][2], np.float64)
    build_s = float(np.median([r[0] for r in recs]))
    print("[bench] each graph alone (per-graph shortcuts/s)", file=sys.stderr, flush=True)
    alone = []
    for (o, d, w), n, k in zip(dgraphs, sizes, sc):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        c = binding.build(o, d, w)
        torch.cuda.synchronize()
        alone.append(k / (time.perf_counter() - ta))
        c.free()
    alone = np.array(alone)
    line = {
        "metric": "CH build time (s) + shortcuts/s + HBM roofline %, plain priority",
        "value": float(sc.sum()) / (ms_per_step / 1e3), "unit": "shortcuts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["batch512"]["desc"], "graphs": len(graphs),
                   "n": int(sizes.sum()), "m": int(sum(len(g[1]) for g in graphs)),
                   "step": "ch_build_batch + 512 ch_query_batch calls of 1000 queries"},
        "batch_build_s": build_s,
        "shortcuts": int(sc.sum()),
        "aggregate_shortcuts_per_build_s": float(sc.sum()) / build_s,
        "per_graph_alone_shortcuts_per_s": {
            "min": float(alone.min()), "median": float(np.median(alone)),
            "max": float(alone.max()), "sum_of_alone_build_s": float((sc / alone).sum())},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="road24m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--one-to-all", type=int, default=64, metavar="K",
                    help="after the steps, time ch_one_to_all from K sources to every vertex "
                         "(0 = skip)")
    ap.add_argument("--settle", type=int, default=0, metavar="THETA",
                    help="witness searches in the paper's settled(theta) mode instead of "
                         "exact")
    ap.add_argument("--untuned", action="store_true",
                    help="ignore the autotuner cache (default knobs)")
    ap.add_argument("--learned", default=os.path.join(ROOT, "paper_2412_18008_amd",
                                                      "learned_weights.npy"),
                    help="weights (.npy, 4801 float32) of the learned priority; the plain vs "
                         "learned comparison runs after the timed steps when the file exists")
    ap.add_argument("--learned-on", default="road1m", choices=("road1m", "road24m", "none"),
                    help="workload of the plain vs learned comparison (after the timed steps)")
    ap.add_argument("--no-query-sweep", action="store_true",
                    help="skip the query latency / throughput sweep over batch sizes")
    ap.add_argument("--no-hbm-probe", action="store_true",
                    help="skip the streaming / scattered HBM probe")
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
    if args.workload == "batch512":
        bench_batch512(args, binding, dev)
        return

    t_gen = time.perf_counter()
    g, (qs, qt) = make_graph(args.workload)
    off, dst, w = g
    n, m = len(off) - 1, len(dst)
    print(f"[bench] workload {args.workload}: n={n} m={m} queries={len(qs)} "
          f"(generated in {time.perf_counter() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    t_off = torch.from_numpy(off.astype(np.int64)).to(dev)
    t_dst = torch.from_numpy(dst.astype(np.int32)).to(dev)
    t_w = torch.from_numpy(w.astype(np.int32)).to(dev)
    t_s = torch.from_numpy(qs.astype(np.int32)).to(dev)
    t_t = torch.from_numpy(qt.astype(np.int32)).to(dev)
    torch.cuda.synchronize()

    from paper_2412_18008_amd import autotune

    knobs = {} if args.untuned else autotune.params_for(n, m)
    qknobs = {} if args.untuned else autotune.query_params_for(n, m)
    if args.settle:
        knobs = dict(knobs, settle=args.settle)
    print(f"[bench] knobs {knobs or 'default'}, query {qknobs or 'default'}", file=sys.stderr,
          flush=True)

    def step():
        tb = time.perf_counter()
        ch = binding.build(t_off, t_dst, t_w, seed=0, stats=True, **knobs)
        tq = time.perf_counter()
        d = ch.query(t_s, t_t, **qknobs)
        te = time.perf_counter()
        rec = dict(build_s=tq - tb, query_s=te - tq, summary=dict(ch.summary),
                   rounds=ch.round_stats(), query=ch.last_query_stats())
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

    # query kernels: device time per tier from the timed batches; their
    # algorithmic units from one more batch with the stats counters
    print("[bench] counting the query kernels' units in one more batch", file=sys.stderr,
          flush=True)
    ch = binding.build(t_off, t_dst, t_w, seed=0, **knobs)
    ch.query(t_s, t_t, count=True, **qknobs)  # a fresh CH, as in the timed steps
    torch.cuda.synchronize()
    qstat = ch.last_query_stats()
    first = qstat["first_tier"]
    ch.free()
    qper = {}
    for r in recs:
        for ti in range(4):
            if r["query"]["tier_queries"][ti]:
                a = qper.setdefault(QUERY_KERNELS[ti], [0, 0.0])
                a[0] += 1
                a[1] += r["query"]["tier_ms"][ti]
    q_bytes_batch = 8 * qstat["rows"] + 8 * qstat["arcs"]

    per = search_kernels(binding, recs)
    cands = {k: v[1] for k, v in per.items()}
    for k, v in qper.items():
        cands[k] = v[1]
    dom = max(cands, key=cands.get)
    if dom in per:
        la, ms, b = per[dom]
        roof = roofline_obj(args.workload, dom, la, ms, b,
                            "8 B per row + 8 B per arc + 16 B per memo slot read or written")
    else:
        la, ms = qper[dom]
        # bytes of the whole batch, all tiers; attributed to the dominant tier
        roof = roofline_obj(args.workload, dom, la, ms, q_bytes_batch * la,
                            "8 B per adjacency row read (expanded or stall-checked) + 8 B per "
                            "arc or core-table entry read, the whole batch (counted in one more "
                            "batch)")
    wl, wms, wb = (sum(v[i] for v in per.values()) for i in range(3))
    roof_wps = roofline_obj(args.workload, "all witness-search launches", wl, wms, wb,
                            "8 B per row + 8 B per arc + 16 B per memo slot read or written")
    roof_wps["per_kernel"] = {k: {"launches": v[0], "ms": v[1], "bytes": v[2],
                                  "achieved_gbs": (v[2] / 1e9) / (v[1] / 1e3) if v[1] else 0.0}
                              for k, v in per.items()}
    roof_wps["ms_per_build"] = wms / args.steps

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
                   "wps": (f"settled(theta={args.settle}), radius D_s" if args.settle
                           else "exact, radius D_s"),
                   "step": "ch_build + one ch_query_batch",
                   "knobs": knobs or "default", "query_knobs": qknobs or "default"},
        "build_time_s": build_s,
        "query_batch_ms": query_s * 1e3,
        "queries_per_s": len(qs) / query_s,
        "query_first_tier": first,
        "query_units": {"rows": qstat["rows"], "arcs": qstat["arcs"],
                        "tier_queries": qstat["tier_queries"]},
        "rounds": recs[-1]["summary"]["rounds"],
        "shortcuts": shortcuts,
        "shortcuts_per_build_s": shortcuts / build_s,
        "roofline": roof,
        "roofline_wps": roof_wps,
        "kernel_ms_per_step": {k: v / args.steps for k, v in sorted(cands.items(),
                                                                  key=lambda x: -x[1])},
    }
    if not args.no_query_sweep:
        print("[bench] query latency and throughput per batch size", file=sys.stderr, flush=True)
        ch = binding.build(t_off, t_dst, t_w, seed=0, **knobs)
        line["query_batch_sizes"] = query_sizes(ch, qs, qt, dev, qknobs=qknobs)
        ch.free()
    if not args.no_hbm_probe:
        print("[bench] HBM probe (streaming and scattered)", file=sys.stderr, flush=True)
        line["hbm_probe"] = hbm_probe(dev)
    if args.one_to_all:
        print(f"[bench] one-to-all from {args.one_to_all} sources", file=sys.stderr, flush=True)
        ch = binding.build(t_off, t_dst, t_w, seed=0, **knobs)
        srcs = torch.from_numpy(qs[:args.one_to_all].astype(np.int32)).to(dev)
        ch.one_to_all(srcs[:1])  # scratch sized once
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = ch.one_to_all(srcs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        line["one_to_all"] = {"sources": args.one_to_all, "ms": el * 1e3,
                              "ms_per_source": el * 1e3 / args.one_to_all,
                              "levels": recs[-1]["summary"]["rounds"],
                              "distances_per_s": args.one_to_all * n / el}
        del rows
        ch.free()
    if os.path.exists(args.learned) and args.learned_on != "none":
        if args.learned_on == args.workload:
            lg = (t_off, t_dst, t_w, qs, qt)
        else:
            (lo, ld, lw), (lqs, lqt) = make_graph(args.learned_on)
            lg = (torch.from_numpy(lo.astype(np.int64)).to(dev),
                  torch.from_numpy(ld.astype(np.int32)).to(dev),
                  torch.from_numpy(lw.astype(np.int32)).to(dev), lqs, lqt)
        line["plain_vs_learned"] = plain_vs_learned(binding, args, dev, args.learned_on, lg)
    if args.copy_calibration:
        copy_calibration(dev, args.copy_calibration)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample ...", file=sys.stderr,
              flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, args.settle)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Host logic that needs no GPU: the seeded input recipes (the shapes and
value distributions of the paper's workload families, Sec. "Experimental
Setup"), the autotuner's cache, the counter-summary lookup of bench.py and
its one-GPU guard."""
import importlib.util
import json
import math
import os
import subprocess
import sys

import numpy as np

from paper_2412_18008_amd import autotune, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _arcs(off, dst, w):
    src, d, ww = synth.arcs_of(off, dst, w)
    return src.astype(np.int64), d.astype(np.int64), ww.astype(np.int64)


def test_csr_round_trip_and_permutation():
    src = np.array([3, 0, 3, 1, 0], np.int64)
    dst = np.array([1, 2, 0, 3, 3], np.int64)
    w = np.array([5, 6, 7, 8, 9], np.int64)
    off, d, ww = synth.to_csr(4, src, dst, w)
    assert off.tolist() == [0, 2, 3, 3, 5]
    # stable within a row: arcs of 0 keep their input order
    assert d.tolist() == [2, 3, 3, 1, 0] and ww.tolist() == [6, 9, 8, 5, 7]
    s2, d2, w2 = _arcs(off, d, ww)
    assert sorted(zip(s2.tolist(), d2.tolist(), w2.tolist())) == \
        sorted(zip(src.tolist(), dst.tolist(), w.tolist()))
    perm = np.array([2, 0, 3, 1])
    po, pd, pw = synth.permute(off, d, ww, perm)
    ps, pd2, pw2 = _arcs(po, pd, pw)
    assert sorted(zip(ps.tolist(), pd2.tolist(), pw2.tolist())) == \
        sorted(zip(perm[src].tolist(), perm[dst].tolist(), w.tolist()))


def _undirected_stats(off, dst, w):
    s, d, ww = _arcs(off, dst, w)
    n = len(off) - 1
    key = s * n + d
    rev = d * n + s
    has_rev = np.isin(key, rev)
    # an edge with both directions is two arcs; a one-way edge is one
    edges = has_rev.sum() // 2 + (~has_rev).sum()
    return s, d, ww, edges, (~has_rev).sum() / edges


def test_road_like_recipe():
    n = 20_000
    a = synth.road_like(n, seed=5)
    b = synth.road_like(n, seed=5)
    for x, y in zip(a, b):  # deterministic per seed
        assert np.array_equal(x, y)
    assert not np.array_equal(a[1], synth.road_like(n, seed=6)[1])
    s, d, w, edges, oneway = _undirected_stats(*a)
    assert np.all(s != d) and np.all(w >= 1)
    # 3-NN symmetrised: between 3 and 6 neighbours per vertex, ~1.8 n edges
    assert 1.5 * n < edges < 2.2 * n
    assert 0.07 < oneway < 0.13  # 10% of the edges one-way
    # weight = round(1e4 * length) + 1; typical 3-NN length ~ 0.5 / sqrt(n)
    med = np.median(w)
    assert 0.2 * 1e4 / math.sqrt(n) < med < 2.0 * 1e4 / math.sqrt(n)


def test_clustered_road_recipe():
    n = 30_000
    off, dst, w = synth.clustered_road(n, seed=1)
    s, d, ww, edges, oneway = _undirected_stats(off, dst, w)
    assert np.all(s != d) and np.all(ww >= 1)
    assert 1.5 * n < edges < 2.2 * n
    assert 0.07 < oneway < 0.13
    # the cities (70% of the points in small Gaussians) widen the spread of
    # edge weights well beyond that of uniform points
    def spread(x):
        x = x.astype(np.float64)
        return np.percentile(x, 99) / np.median(x)
    u = synth.road_like(n, seed=1, scale=1.1e6 / 50)[2]
    assert spread(ww) > 1.4 * spread(u)


def test_knn_recipe():
    for k in (2, 5, 10):
        off, dst, w = synth.knn_graph(5000, k, seed=k)
        deg = np.diff(off.astype(np.int64))
        assert np.all(deg == k)  # k out-arcs per vertex
        s, d, ww = _arcs(off, dst, w)
        assert np.all(s != d)
        assert ww.min() >= 1 and ww.max() <= 32
        assert len(np.unique(ww)) == 32  # uniform over 1..32


def test_small_families():
    off, dst, w = synth.grid(3, 4, seed=0, wmin=1, wmax=1)
    assert len(dst) == 2 * (3 * 3 + 2 * 4) and np.all(w == 1)
    off, dst, w = synth.fan(10)
    s, d, ww = _arcs(off, dst, w)
    assert np.all(d[s == 10] == np.arange(10)) and np.all(ww[s == 10] == 1000)
    assert not np.any(d == 10)  # the hub has no in-arcs
    lab = synth.labels(1000, 3)
    assert sorted(lab.tolist()) == list(range(1000))
    qs, qt = synth.queries(100, 5000, seed=2)
    assert qs.max() < 100 and qt.max() < 100 and qs.min() >= 0


def test_batch512_sizes():
    sz = synth.batch512_sizes()
    assert len(sz) == 512
    assert sz.min() >= 10_000 and sz.max() < 500_000
    # log-uniform: the mean of log n is the midpoint of the log range
    mid = (math.log(1e4) + math.log(5e5)) / 2
    assert abs(np.log(sz).mean() - mid) < 0.15
    assert 55e6 < sz.sum() < 75e6  # about 64M vertices in all


def test_autotuner_cache(tmp_path):
    # the committed cache holds the benchmark size classes, each with values
    # the tuner can try
    tuned = autotune.load(autotune.DEFAULT_CACHE)
    for n, m in ((1_000_000, 3_541_000), (24_000_000, 84_985_476)):
        cls = autotune.size_class(n, m)
        assert cls in tuned, cls
        p = autotune.params_for(n, m, path=autotune.DEFAULT_CACHE)
        assert set(p) <= set(autotune.KNOBS)
        for k, v in p.items():
            assert v in autotune.CHOICES[k], (cls, k, v)
        q = autotune.query_params_for(n, m, path=autotune.DEFAULT_CACHE)
        for k, v in q.items():
            assert v in autotune.QUERY_CHOICES[k], (cls, k, v)
    # classes: a factor ~1.4 in n and 0.5 in degree
    assert autotune.size_class(1_000_000, 3_500_000) == autotune.size_class(1_100_000, 3_900_000)
    assert autotune.size_class(1_000_000, 3_500_000) != autotune.size_class(2_000_000, 7_000_000)
    assert autotune.size_class(1_000_000, 3_500_000) != autotune.size_class(1_000_000, 5_000_000)
    # save / load round trip; an unknown class gives the library's defaults
    path = str(tmp_path / "t.json")
    cls = autotune.size_class(5000, 20000)
    autotune.save({cls: {"params": {"ls_step": 5, "group": 8, "other": 1},
                         "query": {"params": {"waves": 2, "window": 16}}}}, path)
    assert json.load(open(path))[cls]["params"]["ls_step"] == 5
    assert autotune.params_for(5000, 20000, path=path) == {"ls_step": 5, "group": 8}
    assert autotune.query_params_for(5000, 20000, path=path) == {"waves": 2, "window": 16}
    assert autotune.params_for(7, 7, path=path) == {}
    assert autotune.query_params_for(7, 7, path=path) == {}


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_counter_summary_lookup():
    b = _bench()
    rec = {}
    with open(os.path.join(ROOT, "profiles", "pmc_road24m.md")) as f:
        for line in f:
            if line.startswith("traffic:"):
                k, _, v = line[len("traffic:"):].strip().rpartition("=")
                rec[k.strip()] = v.strip()
    assert rec["workload"] == "road24m"
    kern = "k_query<16, QTier2>"
    got = b.committed_traffic("road24m", kern)
    if rec["source_hash"] == b.kernel_source_hash():
        assert got == float(rec[kern])
    else:  # kernel sources changed since the counters were taken
        assert got is None
    # no record: another workload, or a kernel the summary does not hold
    assert b.committed_traffic("road1m", kern) is None
    assert b.committed_traffic("road24m", "k_not_profiled") is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_arithmetic():
    # algorithmic bytes of a witness search: 8 B per adjacency row, 8 B per
    # arc, 16 B per memo slot read or written; the roofline object divides
    # them by the summed launch time and by the 8 TB/s HBM peak
    b = _bench()
    assert b.ls_bytes(1, 0, 0, 0) == 8 and b.ls_bytes(0, 1, 0, 0) == 8
    assert b.ls_bytes(0, 0, 1, 0) == 16 and b.ls_bytes(0, 0, 0, 1) == 16
    assert b.ls_bytes(10, 20, 30, 40) == 80 + 160 + 480 + 640
    r = b.roofline_obj("nowhere", "k_x", 4, 2.0, 8e9, "units")
    assert r["achieved"] == 4000.0  # 8 GB in 2 ms
    assert r["peak"] == 8000.0 and r["frac"] == 0.5 and r["unit"] == "GB/s"
    assert r["avg_launch_ms"] == 0.5 and r["algorithmic_bytes_per_launch"] == 2e9
    assert r["traffic"] is None  # no counter summary for that workload

    # the per-kernel sums skip rounds without sources and the device-driven
    # tail, and add the block and global tiers where they ran
    class B:
        CH_LS_TAIL = 99
        LS_KERNELS = {0: "k_a", 1: "k_b"}

    def rnd(tier, ms, rows, n_sources=1, blk=0.0, glob=0):
        return dict(n_sources=n_sources, ls_tier1=tier, ms_local_search=ms,
                    rows_expanded=rows, arcs_scanned=0, memo_probes=0, memo_inserts=0,
                    ms_ls_blk=blk, rows2=1, arcs2=0, probes2=0, inserts2=0,
                    n_ls_global=glob, ms_ls_global=0.5, rows3=2, arcs3=0, probes3=0,
                    inserts3=0)
    recs = [{"rounds": [rnd(0, 1.0, 5), rnd(0, 2.0, 7, blk=0.25), rnd(1, 3.0, 1, glob=3),
                        rnd(0, 9.0, 100, n_sources=0), rnd(99, 9.0, 100)]}]
    per = b.search_kernels(B, recs)
    assert per["k_a"] == [2, 3.0, 8 * 12]
    assert per["k_b"] == [1, 3.0, 8]
    assert per[b.BLK_KERNEL] == [1, 0.25, 8]
    assert per[b.GLOBAL_KERNEL] == [1, 0.5, 16]

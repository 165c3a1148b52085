"""GPU parity of the hop-bounded witness search (CH_WPS_HOP): the CH built
with walks of at most H arcs per witness must equal the oracle's hop(H)
build bit for bit (level, score, rank, every CH arc and the per-round
counts), and its query distances must still equal Dijkstra's."""
import numpy as np
import pytest

import oracle
from paper_2412_18008_amd import synth
from parity_util import (assert_export_order, assert_same_ch, gpu_export, gpu_round_counts,
                         oracle_export, oracle_round_counts, reference_distances)
from test_gpu_parity import small_cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18008_amd import binding

    binding.lib()
    return binding


def _hop_case(name, off, dst, w, labels, gpu, H, **kw):
    print(f"[hop] {name} H={H} n={len(off) - 1} m={len(dst)} {kw}", flush=True)
    o = oracle.OracleCH(off, dst, w, labels=labels, wps_mode=oracle.WPS_HOP, hop_limit=H).run()
    ch = gpu.build(off, dst, w, labels=labels, stats=True, hop=H, **kw)
    a, b = oracle_export(o), gpu_export(ch)
    assert_same_ch(a, b, f"{name} H={H}")
    assert_export_order(b)
    assert ch.summary["rounds"] == o.rounds
    assert gpu_round_counts(ch) == oracle_round_counts(o), name
    return o, ch


def test_hop_small_graphs_bit_exact(gpu):
    for H in (1, 2, 3, 6):
        for name, off, dst, w in small_cases():
            _hop_case(name, off, dst, w, synth.labels(len(off) - 1, 17), gpu, H)


def test_hop_grid64_and_queries(gpu):
    off, dst, w = synth.config_grid64(seed=0)
    n = len(off) - 1
    for H in (2, 4):
        o, ch = _hop_case("grid64", off, dst, w, synth.labels(n, 1), gpu, H)
        s, t = synth.queries(n, 1000, seed=1)
        d = ch.query(s, t)
        assert np.array_equal(d, reference_distances(off, dst, w, s, t))
        od, _ = o.query_batch(s, t)
        assert np.array_equal(d, od)


def test_hop_road_and_kernel_invariance(gpu):
    off, dst, w = synth.road_like(30_000, seed=6)
    n = len(off) - 1
    lab = synth.labels(n, 2)
    o, ch = _hop_case("road30k", off, dst, w, lab, gpu, 3)
    ref = gpu_export(ch)
    for kw in (dict(group=4), dict(group=64), dict(ls_sparse=4, ls_dense=1),
               dict(ls_sparse=2, ls_dense=3)):
        other = gpu.build(off, dst, w, labels=lab, hop=3, **kw)
        assert_same_ch(ref, gpu_export(other), f"road30k H=3 {kw}")
    s, t = synth.queries(n, 2000, seed=8)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(ch.query(s, t), od)


def test_hop_mode_needs_a_limit(gpu):
    # CH_WPS_HOP with hop_limit 0 is rejected before any work
    import ctypes as C

    off, dst, w = synth.grid(4, 4, seed=1)
    po, ko = gpu._ptr(off, np.uint64)
    pd, kd = gpu._ptr(dst, np.uint32)
    pw, kw = gpu._ptr(w, np.uint32)
    g = gpu.Graph(len(ko) - 1, len(kd), po, pd, pw, None)
    p = gpu.Params(gpu.CH_WPS_HOP, 0, 0, 0, 0, None, 0, 0, 0, gpu.CH_PRIO_PLAIN, None, 0)
    h = C.c_void_p()
    assert gpu.lib().ch_build(C.byref(g), C.byref(p), C.byref(h)) == -1  # CH_E_INVALID


def test_hop_global_search_tier(gpu):
    # the stars' two-hop balls outgrow the first tier (3201 vertices: the
    # block tier's LDS table) and the block tier too (6601 vertices: the
    # global tables); see the exact-mode star test
    for d, tier in ((3200, "n_ls_fallback"), (6600, "n_ls_global")):
        off, dst, w = synth.star(d, seed=5)
        n = len(off) - 1
        o, ch = _hop_case(f"star{d}", off, dst, w, synth.labels(n, 3), gpu, 2)
        assert ch.round_stats()[0][tier] > 0
        s, t = synth.queries(n, 300, seed=2)
        od, _ = o.query_batch(s, t)
        assert np.array_equal(ch.query(s, t), od)


def test_hop_global_search_tier_after_pruning(gpu):
    # as the exact-mode test: the arc pruned in round 0 is still there for
    # the global-tier searches, which in hop mode may need it (a shorter
    # witness with more arcs does not replace it within H arcs)
    from test_gpu_parity import star_with_prunable_arc

    off, dst, w = star_with_prunable_arc(6600, seed=5)
    n = len(off) - 1
    o, ch = _hop_case("star6600+arc", off, dst, w, synth.labels(n, 3), gpu, 2)
    rs = ch.round_stats()[0]
    assert rs["n_ls_global"] > 0 and rs["n_pruned"] > 0, rs
    s, t = synth.queries(n, 300, seed=2)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(ch.query(s, t), od)


def test_hop_road1m_bit_exact(gpu):
    # the hop-bounded build at the benchmark's 1M size: every tier of the
    # search kernels and the table rounds, bit-exact with the oracle's
    # (H = 4: the oracle's own build takes about 35 s on one core)
    off, dst, w = synth.road_like(1_000_000, seed=6)
    n = len(off) - 1
    o, ch = _hop_case("road1m", off, dst, w, synth.labels(n, 2), gpu, 4)
    s, t = synth.queries(n, 5000, seed=9)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(ch.query(s, t), od)

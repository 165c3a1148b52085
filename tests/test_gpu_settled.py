"""GPU parity of the settled(theta) witness search -- the paper's literal
bound (Alg. 4: a search stops once theta vertices are settled or once every
target is; unsettled targets get no memo entry) -- against the oracle's
settled mode, bit for bit: level, score, rank, every CH arc and the per-round
counts, for several theta, on small graphs, a road-like graph and stars whose
searches need the block tier and the global tier."""
import numpy as np
import pytest

import oracle
from paper_2412_18008_amd import synth
from parity_util import (assert_export_order, assert_same_ch, gpu_export, gpu_round_counts,
                         oracle_export, oracle_round_counts, progress)
from test_gpu_parity import small_cases, star_with_prunable_arc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18008_amd import binding

    binding.lib()
    return binding


def _settled_case(name, off, dst, w, labels, gpu, theta, **kw):
    progress(f"[settled] {name} theta={theta} n={len(off) - 1} m={len(dst)} {kw}")
    o = oracle.OracleCH(off, dst, w, labels=labels, wps_mode=oracle.WPS_SETTLED,
                        settle_limit=theta).run()
    ch = gpu.build(off, dst, w, labels=labels, stats=True, settle=theta, **kw)
    a, b = oracle_export(o), gpu_export(ch)
    assert_same_ch(a, b, f"{name} theta={theta}")
    assert_export_order(b)
    assert ch.summary["rounds"] == o.rounds
    assert gpu_round_counts(ch) == oracle_round_counts(o), name
    return o, ch


def test_settled_small_graphs_bit_exact(gpu):
    for theta in (1, 2, 3, 10, 50):
        for name, off, dst, w in small_cases():
            _settled_case(name, off, dst, w, synth.labels(len(off) - 1, 17), gpu, theta)


def test_settled_fixture_graph(gpu):
    # the graph of tests/golden/settled_theta_memo.txt (settle order by
    # label on equal distances) through the whole build, every theta
    off, dst, w = synth.to_csr(5, [0, 0, 1, 3], [1, 3, 2, 4], [1, 1, 1, 1])
    lab = np.array([0, 1, 4, 2, 3], np.uint32)
    for theta in (1, 2, 3, 4, 5, 10):
        _settled_case("fixture", off, dst, w, lab, gpu, theta)


def test_settled_road_and_grid(gpu):
    off, dst, w = synth.road_like(30_000, seed=6)
    n = len(off) - 1
    for theta in (5, 50):
        o, ch = _settled_case("road30k", off, dst, w, None, gpu, theta)
        s, t = synth.queries(n, 2000, seed=theta)
        od, _ = o.query_batch(s, t)
        assert np.array_equal(ch.query(s, t), od)
    off, dst, w = synth.config_grid64(seed=0)
    _settled_case("grid64", off, dst, w, synth.labels(4096, 1), gpu, 20)
    # a batch of graphs in settled mode equals the oracle per graph
    graphs = [synth.road_like(2000, seed=i) for i in (1, 2, 3)]
    for g, c in zip(graphs, gpu.build_batch(graphs, settle=8)):
        o = oracle.OracleCH(*g, wps_mode=oracle.WPS_SETTLED, settle_limit=8).run()
        assert_same_ch(oracle_export(o), gpu_export(c), "settled batch")


def test_settled_block_and_global_tiers(gpu):
    # the leaves reach the whole star through its centre: 3201 vertices
    # outgrow the first tier (block tier), 6601 the block tier (global tier)
    for d, tier in ((3200, "n_ls_fallback"), (6600, "n_ls_global")):
        off, dst, w = star_with_prunable_arc(d, seed=5)
        n = len(off) - 1
        o, ch = _settled_case(f"star{d}+arc", off, dst, w, synth.labels(n, 3), gpu, 40)
        assert ch.round_stats()[0][tier] > 0
        s, t = synth.queries(n, 300, seed=2)
        od, _ = o.query_batch(s, t)
        assert np.array_equal(ch.query(s, t), od)


def test_settled_needs_a_limit(gpu):
    off, dst, w = synth.chain(10, seed=1)
    with pytest.raises(gpu.ChError) as e:
        p = gpu.Params(gpu.CH_WPS_SETTLED)
        import ctypes as C

        po, ko = gpu._ptr(off, np.uint64)
        pd, kd = gpu._ptr(dst, np.uint32)
        pw, kw = gpu._ptr(w, np.uint32)
        g = gpu.Graph(len(ko) - 1, len(kd), po, pd, pw, None)
        h = C.c_void_p()
        gpu._check(gpu.lib().ch_build(C.byref(g), C.byref(p), C.byref(h)), "ch_build")
    assert e.value.code == gpu.CH_E_INVALID


def test_settled_road1m_bit_exact(gpu):
    # the paper's settled(theta) bound at the benchmark's 1M size (theta =
    # 1000: the oracle's own build takes about 45 s on one core)
    off, dst, w = synth.road_like(1_000_000, seed=6)
    n = len(off) - 1
    o, ch = _settled_case("road1m", off, dst, w, None, gpu, 1000)
    s, t = synth.queries(n, 5000, seed=10)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(ch.query(s, t), od)

"""GPU parity: the HIP library, called through its C ABI, must reproduce the
oracle bit for bit -- level, score at contraction, rank, every upward and
downward CH arc with weight and middle vertex, and the per-round counts --
and its query distances must equal Dijkstra's.  Integer work, so the bar is
exact equality everywhere."""
import numpy as np
import pytest

import oracle
from paper_2412_18008_amd import synth
from parity_util import (assert_export_order, assert_same_ch, closure_sizes, gpu_export,
                         gpu_round_counts, oracle_export, oracle_round_counts,
                         reference_distances)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18008_amd import binding

    binding.lib()
    return binding


def _case(name, off, dst, w, labels, gpu, group=0, seed=0, **kw):
    print(f"[parity] {name} n={len(off) - 1} m={len(dst)} group={group}", flush=True)
    o = oracle.OracleCH(off, dst, w, labels=labels, seed=seed).run()
    ch = gpu.build(off, dst, w, labels=labels, seed=seed, stats=True, group=group, **kw)
    a, b = oracle_export(o), gpu_export(ch)
    assert_same_ch(a, b, name)
    assert_export_order(b)
    assert ch.summary["rounds"] == o.rounds
    assert gpu_round_counts(ch) == oracle_round_counts(o), name
    return o, ch


def small_cases():
    cases = []
    for s in range(8):
        cases.append((f"digraph{s}", *synth.random_digraph(40, 160, seed=s, wmax=9,
                                                            zero_frac=0.15, loops=True)))
    for s in range(4):
        cases.append((f"road{s}", *synth.random_geometric_small(300, seed=s)))
    cases.append(("grid7x9", *synth.grid(7, 9, seed=3)))
    cases.append(("unitgrid6", *synth.grid(6, 6, seed=0, wmin=1, wmax=1)))
    cases.append(("chain", *synth.chain(257, seed=1, directed=True)))
    cases.append(("bichain", *synth.chain(300, seed=2, directed=False)))
    cases.append(("star", *synth.star(70, seed=3)))
    cases.append(("sparse", *synth.random_digraph(200, 60, seed=9, wmax=5)))
    cases.append(("dense", *synth.random_digraph(60, 1500, seed=4, wmax=3)))
    return cases


def test_small_graphs_bit_exact(gpu):
    for name, off, dst, w in small_cases():
        n = len(off) - 1
        _case(name, off, dst, w, synth.labels(n, 17), gpu)


def test_grid64_bit_exact_and_queries(gpu):
    off, dst, w = synth.config_grid64(seed=0)
    n = len(off) - 1
    lab = synth.labels(n, 1)
    o, ch = _case("grid64", off, dst, w, lab, gpu)
    s, t = synth.queries(n, 1000, seed=1)
    d = ch.query(s, t)
    ref = reference_distances(off, dst, w, s, t)
    assert np.array_equal(d, ref)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(d, od)
    # query cost: the sizes of the two upward search spaces
    cs = closure_sizes(o, s[:300], t[:300])
    for nw in (1, 2, 4, 8):
        assert np.array_equal(ch.query(s, t, waves=nw), ref), nw
        d2, vis = ch.query_stats(s[:300], t[:300], waves=nw)
        assert np.array_equal(d2, d[:300])
        assert np.array_equal(vis.astype(np.int64), cs), nw
    # the level window orders the expansions; distances and the reached
    # sets do not depend on it (255 = none)
    # complete search spaces (no pruning by the best path met) give the same
    assert np.array_equal(ch.query(s, t, full=True), ref)
    for win in (1, 2, 7, 64, 255):
        assert np.array_equal(ch.query(s, t, window=win), ref), win
        assert np.array_equal(ch.query(s, t, window=win, full=True), ref), win
        d2, vis = ch.query_stats(s[:300], t[:300], waves=1, window=win)
        assert np.array_equal(d2, d[:300]), win
        assert np.array_equal(vis.astype(np.int64), cs), win


def test_group_split_invariance(gpu):
    off, dst, w = synth.grid(20, 25, seed=5)
    n = len(off) - 1
    lab = synth.labels(n, 2)
    ref = gpu_export(gpu.build(off, dst, w, labels=lab))
    for g in (4, 8, 16, 32, 64):
        assert_same_ch(ref, gpu_export(gpu.build(off, dst, w, labels=lab, group=g)), f"G={g}")


def test_default_labels_match_oracle(gpu):
    off, dst, w = synth.random_geometric_small(500, seed=7)
    for seed in (0, 12345, 0xDEADBEEF12345678):
        _case(f"default-labels seed={seed}", off, dst, w, None, gpu, seed=seed)


def test_device_input_and_device_queries(gpu):
    import torch

    off, dst, w = synth.road_like(5000, seed=3)
    n = len(off) - 1
    lab = synth.labels(n, 4)
    dev = torch.device("cuda:0")
    t_off = torch.from_numpy(off.astype(np.int64)).to(dev)
    t_dst = torch.from_numpy(dst.astype(np.int32)).to(dev)
    t_w = torch.from_numpy(w.astype(np.int32)).to(dev)
    t_lab = torch.from_numpy(lab.astype(np.int32)).to(dev)
    ch = gpu.build(t_off, t_dst, t_w, labels=t_lab)
    o = oracle.OracleCH(off, dst, w, labels=lab).run()
    assert_same_ch(oracle_export(o), gpu_export(ch), "device-input")
    s, t = synth.queries(n, 2000, seed=5)
    ds = ch.query(torch.from_numpy(s.astype(np.int32)).to(dev),
                  torch.from_numpy(t.astype(np.int32)).to(dev))
    torch.cuda.synchronize()
    got = ds.cpu().numpy().view(np.uint64)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(got, od)


def test_queries_unreachable_and_self(gpu):
    off, dst, w = synth.random_digraph(300, 250, seed=11, wmax=7)
    n = len(off) - 1
    ch = gpu.build(off, dst, w, labels=synth.labels(n, 3))
    s = np.repeat(np.arange(0, n, 7, dtype=np.uint32), 5)
    t = np.tile(np.arange(0, 5 * 7, 7, dtype=np.uint32), len(s) // 5)
    s = np.concatenate([s, np.arange(20, dtype=np.uint32)])
    t = np.concatenate([t, np.arange(20, dtype=np.uint32)])
    d = ch.query(s, t)
    assert np.array_equal(d, reference_distances(off, dst, w, s, t))
    assert np.all(d[-20:] == 0)
    assert np.any(d == np.uint64(0xFFFFFFFFFFFFFFFF))


def test_empty_and_isolated(gpu):
    ch = gpu.build(np.zeros(1, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert ch.summary["rounds"] == 0
    off = np.zeros(9, np.uint64)
    ch = gpu.build(off, np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                   labels=synth.labels(8, 0))
    assert ch.summary["rounds"] == 1
    d = ch.query(np.array([0, 3], np.uint32), np.array([0, 5], np.uint32))
    assert d[0] == 0 and d[1] == np.uint64(0xFFFFFFFFFFFFFFFF)


def test_errors(gpu):
    off, dst, w = synth.to_csr(3, [0, 1], [1, 2], [1, 2])
    with pytest.raises(gpu.ChError) as e:
        gpu.build(off, np.array([1, 3], np.uint32), w)
    assert e.value.code == gpu.CH_E_INVALID
    with pytest.raises(gpu.ChError) as e:
        gpu.build(off, dst, np.array([1, 0xFFFFFFFF], np.uint32))
    assert e.value.code == gpu.CH_E_INVALID
    with pytest.raises(gpu.ChError) as e:
        gpu.build(off, dst, w, labels=np.array([1, 1, 2], np.uint32))
    assert e.value.code == gpu.CH_E_INVALID
    bad_off = np.array([0, 2, 1, 2], np.uint64)
    with pytest.raises(gpu.ChError) as e:
        gpu.build(bad_off, dst, w)
    assert e.value.code == gpu.CH_E_INVALID
    off2, dst2, w2 = synth.to_csr(3, [0, 1], [1, 2], [0xFFFFFFFE, 1])
    with pytest.raises(gpu.ChError) as e:
        gpu.build(off2, dst2, w2, labels=np.array([5, 0, 9], np.uint32))
    assert e.value.code == gpu.CH_E_OVERFLOW
    off3, dst3, w3 = synth.chain(50, seed=1, directed=False)
    with pytest.raises(gpu.ChError) as e:
        gpu.build(off3, dst3, w3, max_rounds=2)
    assert e.value.code == gpu.CH_E_LIMIT
    ch = gpu.build(off, dst, w)
    with pytest.raises(gpu.ChError) as e:
        ch.query(np.array([0], np.uint32), np.array([3], np.uint32))
    assert e.value.code == gpu.CH_E_INVALID
    # inputs large enough for the locality renumbering are validated the same
    # way (the renumbering reads them first and must skip bad rows and heads)
    offb, dstb, wb = synth.grid(64, 64, seed=1)
    bad_dst = dstb.copy()
    bad_dst[len(bad_dst) // 2] = len(offb) + 5
    with pytest.raises(gpu.ChError) as e:
        gpu.build(offb, bad_dst, wb)
    assert e.value.code == gpu.CH_E_INVALID
    bad_off = offb.copy()
    bad_off[100] = bad_off[101] + 1  # not non-decreasing
    with pytest.raises(gpu.ChError) as e:
        gpu.build(bad_off, dstb, wb)
    assert e.value.code == gpu.CH_E_INVALID


def test_road_100k_bit_exact(gpu):
    off, dst, w = synth.road_like(100_000, seed=0)
    n = len(off) - 1
    lab = synth.labels(n, 7)
    o, ch = _case("road100k", off, dst, w, lab, gpu)
    s, t = synth.queries(n, 20_000, seed=3)
    d = ch.query(s, t)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(d, od)
    ref = reference_distances(off, dst, w, s[:20], t[:20])
    assert np.array_equal(d[:20], ref)
    # the same build on the input's own numbering (no locality renumbering)
    # and on the per-step table rounds gives the same CH and round counts
    a = oracle_export(o)
    for kw in (dict(keep_order=True), dict(tail_stepwise=True)):
        print(f"[parity] road100k {kw}", flush=True)
        ch2 = gpu.build(off, dst, w, labels=lab, stats=True, **kw)
        assert_same_ch(a, gpu_export(ch2), f"road100k {kw}")
        assert gpu_round_counts(ch2) == oracle_round_counts(o), kw
        assert np.array_equal(ch2.query(s, t), od), kw


def test_query_tiers(gpu):
    # Upward search spaces of every size: the hub of a fan graph reaches the
    # whole path (the k highest ranks), so its queries need the second LDS
    # tier (k = 3000: more than the first tier's 2048 rank slots + 448 table
    # entries), the 16384-slot tier in global memory (k = 13000: more than
    # the second tier's 8192 rank slots + 3584 table entries) and the last
    # tier with tables of 2n slots (k = 60000); the path's own queries stay in
    # the first tier.  Batches made only of hub queries move the CH's first
    # tier up, which must not change any result.
    for k in (3000, 13000, 60000):
        off, dst, w = synth.fan(k)
        n = len(off) - 1
        print(f"[parity] fan k={k}", flush=True)
        o, ch = _case(f"fan{k}", off, dst, w, synth.labels(n, 9), gpu)
        rs, rt = synth.queries(n, 200, seed=k)
        s = np.concatenate([np.full(40, k, np.uint32), rs, np.arange(0, k, k // 20, dtype=np.uint32)])
        t = np.concatenate([rt[:40], rt, np.full(20, k, np.uint32)])
        od, _ = o.query_batch(s, t)
        cs = closure_sizes(o, s, t)
        assert cs.max() > {3000: 2048 + 448, 13000: 8192 + 3584, 60000: 14336}[k]
        for nw in (1, 2, 4, 8):
            d, vis = ch.query_stats(s, t, waves=nw)
            assert np.array_equal(d, od), nw
            assert np.array_equal(vis.astype(np.int64), cs), nw
            assert np.array_equal(ch.query(s, t, waves=nw), od), nw
            assert np.array_equal(ch.query(s, t, waves=nw, full=True), od), nw
        for win in (1, 255):
            d, vis = ch.query_stats(s, t, window=win)
            assert np.array_equal(d, od), win
            assert np.array_equal(vis.astype(np.int64), cs), win
        for _ in range(2):
            d, vis = ch.query_stats(s[:40], t[:40])
            assert np.array_equal(d, od[:40])
            assert np.array_equal(vis.astype(np.int64), cs[:40])
        d, vis = ch.query_stats(s, t)
        assert np.array_equal(d, od)
        assert np.array_equal(vis.astype(np.int64), cs)
    # unit-weight grids have large upward search spaces too
    off, dst, w = synth.grid(100, 100, seed=1, wmin=1, wmax=1)
    n = len(off) - 1
    ch = gpu.build(off, dst, w, labels=synth.labels(n, 2))
    s, t = synth.queries(n, 300, seed=4)
    ref = reference_distances(off, dst, w, s, t)
    for nw in (1, 2, 4, 8):
        assert np.array_equal(ch.query(s, t, waves=nw), ref), nw
    for win in (1, 5, 255):
        assert np.array_equal(ch.query(s, t, window=win), ref), win


def test_query_core_table(gpu):
    # The first and second query tiers stop both searches at the 1024 or
    # 4096 highest ranks and finish with the table of exact distances among
    # them: every result
    # equals the oracle's (and Dijkstra's) with and without the table, on a
    # CH smaller than the core (every vertex in it), larger ones, random
    # digraphs with unreachable pairs, self queries, and a fan whose hub
    # queries overflow to the third tier; a second batch reuses the table.
    cases = [("grid64", *synth.config_grid64(seed=0)),
             ("road30k", *synth.road_like(30_000, seed=9)),
             ("digraph", *synth.random_digraph(6000, 15000, seed=4, wmax=30)),
             ("fan13000", *synth.fan(13000))]
    for name, off, dst, w in cases:
        n = len(off) - 1
        lab = synth.labels(n, 41)
        print(f"[parity] core {name}", flush=True)
        o = oracle.OracleCH(off, dst, w, labels=lab).run()
        ch = gpu.build(off, dst, w, labels=lab)
        s, t = synth.queries(n, 5000, seed=7)  # a batch that builds the table
        s[:50] = t[:50]  # self queries
        if name == "fan13000":
            s[50:90] = 13000  # the hub: overflows the second tier
        od, _ = o.query_batch(s, t)
        for tier in (1, 2):  # cores of 1024 and 4096 ranks
            # a small batch first: no table yet, searched to the top
            assert np.array_equal(ch.query(s[:100], t[:100], tier=tier), od[:100]), name
            for rep in range(2):
                d = ch.query(s, t, tier=tier)
                assert np.array_equal(d, od), (name, tier, rep)
            # a small batch now uses the table
            assert np.array_equal(ch.query(s[:100], t[:100], tier=tier), od[:100]), name
            assert np.array_equal(ch.query(s, t, tier=tier, core=False), od), name
            assert np.array_equal(ch.query(s, t, tier=tier, full=True), od), name
        if name != "fan13000":
            ref = reference_distances(off, dst, w, s[:200], t[:200])
            assert np.array_equal(d[:200], ref), name


def test_query_distances_past_32_bits(gpu):
    # a one-way path with increasing labels is contracted from its source
    # end without shortcuts, so one upward search passes 2^32 on its own
    k = 7
    off, dst, w = synth.to_csr(k, np.arange(k - 1), np.arange(1, k),
                               np.full(k - 1, 0x7FFFFFFF, np.int64))
    ch = gpu.build(off, dst, w, labels=np.arange(k, dtype=np.uint32))
    assert ch.summary["shortcuts"] == 0
    s, t = (a.ravel().astype(np.uint32) for a in np.meshgrid(np.arange(k), np.arange(k)))
    ref = reference_distances(off, dst, w, s, t)
    assert ref.max(initial=0, where=ref != np.uint64(2**64 - 1)) == 6 * 0x7FFFFFFF
    for nw in (1, 2, 4, 8):
        assert np.array_equal(ch.query(s, t, waves=nw), ref), nw
    for win in (1, 255):
        assert np.array_equal(ch.query(s, t, window=win), ref), win


def test_global_search_tier(gpu):
    # every leaf's witness search covers the whole star: 3201 vertices pass
    # the first tier's table and fit the block tier's 8192-slot LDS table
    # (3/4 of it); 6601 vertices pass that too, so round 0 finishes its
    # searches in global memory and prunes, scores and selects a second time
    # (with the all-pairs table off: the smaller star fits the table)
    for d, tier in ((3200, "n_ls_fallback"), (6600, "n_ls_global")):
        off, dst, w = synth.star(d, seed=5)
        n = len(off) - 1
        o, ch = _case(f"star{d}", off, dst, w, synth.labels(n, 3), gpu,
                      dense_tail=gpu.CH_DENSE_TAIL_OFF)
        r0 = ch.round_stats()[0]
        assert r0[tier] > 0, r0
        if tier == "n_ls_fallback":
            assert r0["n_ls_global"] == 0, r0
        s, t = synth.queries(n, 500, seed=2)
        od, _ = o.query_batch(s, t)
        assert np.array_equal(ch.query(s, t), od)


def _wcase(name, off, dst, w, labels, gpu, okw, gkw):
    """Oracle and GPU builds with their own keyword sets, compared whole."""
    print(f"[parity] {name} n={len(off) - 1} m={len(dst)} {okw}", flush=True)
    o = oracle.OracleCH(off, dst, w, labels=labels, **okw).run()
    ch = gpu.build(off, dst, w, labels=labels, stats=True, **gkw)
    a, b = oracle_export(o), gpu_export(ch)
    assert_same_ch(a, b, name)
    assert_export_order(b)
    assert ch.summary["rounds"] == o.rounds
    assert gpu_round_counts(ch) == oracle_round_counts(o), name
    return o, ch


WEIGHTS = [(1, 2, 5), (3, -1, 0), (0, 1, 0), (-1, 0, 4), (2, 0, -3)]


def test_score_weights_bit_exact(gpu):
    # integer score k_ed ED + k_cn CN + k_depth depth (the paper's combined
    # score, weights ours): same order, scores and arcs as the oracle
    for i, (name, off, dst, w) in enumerate(small_cases()):
        kw = WEIGHTS[i % len(WEIGHTS)]
        okw = dict(k_ed=kw[0], k_cn=kw[1], k_depth=kw[2])
        _wcase(f"{name} {kw}", off, dst, w, synth.labels(len(off) - 1, 17), gpu, okw,
               dict(score_weights=kw))
    # a larger graph through the general rounds, the table rounds (step by
    # step: the device-driven tail takes only the plain edge difference) and
    # with the table off; default labels; hop mode too
    off, dst, w = synth.road_like(30_000, seed=8)
    for kw in WEIGHTS[:2]:
        okw = dict(k_ed=kw[0], k_cn=kw[1], k_depth=kw[2])
        _, ch = _wcase(f"road30k {kw}", off, dst, w, None, gpu, okw, dict(score_weights=kw))
        assert any(r["ls_tier1"] == gpu.CH_LS_TABLE for r in ch.round_stats())
        _wcase(f"road30k {kw} no table", off, dst, w, None, gpu, okw,
               dict(score_weights=kw, dense_tail=gpu.CH_DENSE_TAIL_OFF))
    kw = WEIGHTS[0]
    _wcase(f"road30k {kw} hop 2", off, dst, w, None, gpu,
           dict(k_ed=kw[0], k_cn=kw[1], k_depth=kw[2], wps_mode=oracle.WPS_HOP, hop_limit=2),
           dict(score_weights=kw, hop=2))
    # weights 1, 0, 0 are the plain edge difference
    o = oracle.OracleCH(off, dst, w).run()
    assert_same_ch(oracle_export(o), gpu_export(gpu.build(off, dst, w, score_weights=(1, 0, 0))),
                   "weights 1 0 0")


def test_raw_id_tiebreak_bit_exact(gpu):
    # CH_TIE_RAW_ID: label = vertex id (on the input numbering, also when the
    # library renumbers inputs of 4096 or more vertices internally)
    cases = small_cases()[:6] + [("grid64", *synth.config_grid64(seed=0)),
                                 ("road6000", *synth.road_like(6000, seed=3))]
    for name, off, dst, w in cases:
        _wcase(f"{name} raw", off, dst, w, None, gpu, dict(tiebreak=oracle.TIE_RAW_ID),
               dict(raw_id=True))
    graphs = [c[1:] for c in cases[:4]]
    outs = gpu.build_batch(graphs, raw_id=True, score_weights=WEIGHTS[0])
    for (name, off, dst, w), ch in zip(cases[:4], outs):
        o = oracle.OracleCH(off, dst, w, tiebreak=oracle.TIE_RAW_ID, k_ed=1, k_cn=2,
                            k_depth=5).run()
        assert_same_ch(oracle_export(o), gpu_export(ch), f"batch {name}")


def test_knn_graphs_bit_exact(gpu):
    # the paper's k-NN family: k out-arcs per vertex to its nearest points,
    # weights 1..32; scoring work grows with k (pairs in x out per vertex)
    for n, k in ((3000, 2), (3000, 5), (3000, 10), (50_000, 5), (20_000, 10)):
        off, dst, w = synth.knn_graph(n, k, seed=k)
        lab = synth.labels(n, k)
        o, ch = _case(f"knn n={n} k={k}", off, dst, w, lab, gpu)
        s, t = synth.queries(n, 2000, seed=k)
        od, _ = o.query_batch(s, t)
        assert np.array_equal(ch.query(s, t), od)
        assert np.array_equal(ch.query(s, t, full=True), od)


def star_with_prunable_arc(d, seed):
    """The star of synth.star plus one leaf-to-leaf arc a -> b (weight 1) with
    w(0, a) + 1 < w(0, b): the centre's round-0 search reaches b through a,
    so the arc 0 -> b is pruned in round 0, while every leaf's search (which
    spans the whole star) runs in the global tier."""
    off, dst, w = synth.star(d, seed=seed)
    src, dd, ww = synth.arcs_of(off, dst, w)
    cw = ww[src == 0]
    leaves = dd[src == 0]
    a, b = int(leaves[np.argmin(cw)]), int(leaves[np.argmax(cw)])
    assert cw.min() + 1 < cw.max()
    return synth.to_csr(d + 1, np.append(src, a), np.append(dd, b), np.append(ww, 1))


def test_global_search_tier_after_pruning(gpu):
    # the global-tier searches of round 0 must see the arc the round prunes
    # (pruning follows all searches of the round)
    off, dst, w = star_with_prunable_arc(6600, seed=5)
    n = len(off) - 1
    o, ch = _case("star6600+arc", off, dst, w, synth.labels(n, 3), gpu,
                  dense_tail=gpu.CH_DENSE_TAIL_OFF)
    rs = ch.round_stats()[0]
    assert rs["n_ls_global"] > 0 and rs["n_pruned"] > 0, rs
    s, t = synth.queries(n, 500, seed=2)
    od, _ = o.query_batch(s, t)
    assert np.array_equal(ch.query(s, t), od)


def test_batch_equals_single_builds(gpu):
    graphs = [synth.random_geometric_small(800, seed=1), synth.grid(9, 11, seed=2),
              synth.random_digraph(60, 240, seed=3, wmax=9, zero_frac=0.1, loops=True),
              (np.zeros(1, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32)),
              synth.chain(150, seed=4, directed=False), synth.star(40, seed=5),
              synth.road_like(3000, seed=6)]
    labels = [synth.labels(len(g[0]) - 1, 100 + i) for i, g in enumerate(graphs)]
    print("[parity] batch of", len(graphs), flush=True)
    outs = gpu.build_batch(graphs, labels=labels)
    for i, (g, lab, ch) in enumerate(zip(graphs, labels, outs)):
        # each member equals the oracle's build of that graph alone
        o = oracle.OracleCH(*g, labels=lab).run()
        assert_same_ch(oracle_export(o), gpu_export(ch), f"batch[{i}] vs oracle")
        assert ch.summary["rounds"] == o.rounds
        assert ch.summary["shortcuts"] == sum(r["n_shortcuts"] for r in o.round_stats())
        single = gpu.build(*g, labels=lab)
        a, b = gpu_export(single), gpu_export(ch)
        assert_same_ch(a, b, f"batch[{i}]")
        for key in ("rounds", "up_arcs", "down_arcs", "shortcuts", "m_input"):
            assert ch.summary[key] == single.summary[key], (i, key)
        n = len(g[0]) - 1
        if n:
            s, t = synth.queries(n, 300, seed=i)
            assert np.array_equal(ch.query(s, t), single.query(s, t))
    # default labels: each graph labelled by its local ids
    outs = gpu.build_batch(graphs[:3], seed=77)
    for i, g in enumerate(graphs[:3]):
        assert_same_ch(oracle_export(oracle.OracleCH(*g, seed=77).run()), gpu_export(outs[i]),
                       f"default[{i}] vs oracle")
    # labels need only be distinct within a graph
    same = [synth.labels(len(graphs[1][0]) - 1, 5)] * 2
    outs = gpu.build_batch([graphs[1], graphs[1]], labels=same)
    assert_same_ch(gpu_export(outs[0]), gpu_export(outs[1]), "twins")
    with pytest.raises(gpu.ChError) as e:
        gpu.build_batch([graphs[1], graphs[2]], labels=[labels[1], np.zeros(60, np.uint32)])
    assert e.value.code == gpu.CH_E_INVALID


def test_search_step_buckets_bit_exact(gpu):
    # exact-mode searches with distance buckets of every width (1 = D_s / 2
    # ... 32 = the whole frontier per step), in the first, block and global
    # tiers: the CH and the round counts equal the oracle's
    cases = small_cases()[:6] + [("road20k", *synth.road_like(20_000, seed=8)),
                                 ("grid64", *synth.config_grid64(seed=0)),
                                 ("star6600", *synth.star(6600, seed=3))]
    for name, off, dst, w in cases:
        n = len(off) - 1
        lab = synth.labels(n, 31)
        ref = oracle.OracleCH(off, dst, w, labels=lab).run()
        a = oracle_export(ref)
        for step in (1, 2, 5, 32):
            ch = gpu.build(off, dst, w, labels=lab, ls_step=step, stats=True, dense_tail=1)
            assert_same_ch(a, gpu_export(ch), f"{name} ls_step={step}")
            assert gpu_round_counts(ch) == oracle_round_counts(ref), (name, step)
            if name == "star6600":
                assert sum(r["n_ls_global"] for r in ch.round_stats()) > 0


def test_search_kernel_knobs_invariance(gpu):
    off, dst, w = synth.road_like(20_000, seed=8)
    n = len(off) - 1
    lab = synth.labels(n, 9)
    ref = gpu_export(gpu.build(off, dst, w, labels=lab))
    for a in (1, 2, 3, 4):
        for b in (1, 2, 3, 4):
            for t in (30, 50, 90):
                got = gpu_export(gpu.build(off, dst, w, labels=lab, ls_sparse=a, ls_dense=b,
                                           dense_deg10=t))
                assert_same_ch(ref, got, f"ls_sparse={a} ls_dense={b} thr={t}")


def test_autotuner_roundtrip(gpu, tmp_path, monkeypatch):
    from paper_2412_18008_amd import autotune

    monkeypatch.setenv("SPOCH_AUTOTUNE_CACHE", str(tmp_path / "tuned.json"))
    off, dst, w = synth.road_like(30_000, seed=2)
    n, m = len(off) - 1, len(dst)
    s, t = synth.queries(n, 4000, seed=3)
    # every configuration is checked against the default one inside tune()
    best, qbest, table = autotune.tune(off, dst, w, s, t, reps=1, log=lambda *_: None)
    distinct = {tuple(sorted(r["params"].items())) for r in table}
    assert len(distinct) == len(table) == 1 + sum(
        len([v for v in autotune.CHOICES[k] if v != 0]) for k in autotune.KNOBS)
    assert len(qbest["table"]) == len(autotune.QUERY_CHOICES["waves"]) * len(
        autotune.QUERY_CHOICES["window"])
    autotune.save({autotune.size_class(n, m): dict(params=best["params"], ms=best["ms"],
                                                   query=qbest)})
    assert autotune.params_for(n, m) == best["params"]
    assert autotune.query_params_for(n, m) == qbest["params"]
    ch = gpu.build(off, dst, w, **autotune.params_for(n, m))
    ref = oracle.OracleCH(off, dst, w, seed=0).run()
    d = ch.query(s, t, **autotune.query_params_for(n, m))
    od, _ = ref.query_batch(s[:500], t[:500])
    assert np.array_equal(d[:500], od)


def test_dense_tail_table(gpu):
    # exact-mode searches answered from the all-pairs table of the small
    # overlay: from round 0 (threshold >= n), from a late round, or never --
    # the CH and the round counts must equal the oracle's in every case
    cases = small_cases()[:10] + [("grid64", *synth.config_grid64(seed=0)),
                                  ("road30k", *synth.road_like(30_000, seed=9))]
    for name, off, dst, w in cases:
        n = len(off) - 1
        lab = synth.labels(n, 23)
        o = oracle.OracleCH(off, dst, w, labels=lab).run()
        a = oracle_export(o)
        for tail, stepwise in ((4096, False), (4096, True), (64, False), (64, True),
                               (gpu.CH_DENSE_TAIL_OFF, False)):
            ctx = f"{name} tail={tail} stepwise={stepwise}"
            print(f"[parity] {ctx}", flush=True)
            ch = gpu.build(off, dst, w, labels=lab, stats=True, dense_tail=tail,
                           tail_stepwise=stepwise)
            assert_same_ch(a, gpu_export(ch), ctx)
            assert gpu_round_counts(ch) == oracle_round_counts(o), ctx
            kinds = {r["ls_tier1"] for r in ch.round_stats() if r["n_sources"]}
            table_kind = 5 if stepwise else 6
            if tail == gpu.CH_DENSE_TAIL_OFF:
                assert not kinds & {5, 6}, ctx
            elif n <= tail:
                assert kinds <= {table_kind}, (ctx, kinds)


def test_tail_graph_replay_bit_exact(gpu):
    # the device-driven table rounds replay one captured graph per grid size
    # (batches of rounds with fixed arguments); launched directly instead
    # (CH_F_NO_GRAPH) they must give the same CH, equal to the oracle's, on
    # graphs whose tails run several batches and grid sizes, built twice in a
    # row in one process
    cases = [("grid64", *synth.config_grid64(seed=0)),
             ("road30k", *synth.road_like(30_000, seed=9)),
             ("digraph", *synth.random_digraph(3000, 12000, seed=4, wmax=30))]
    for name, off, dst, w in cases:
        n = len(off) - 1
        lab = synth.labels(n, 29)
        a = oracle_export(oracle.OracleCH(off, dst, w, labels=lab).run())
        for graph in (True, False, True):
            ch = gpu.build(off, dst, w, labels=lab, stats=True, graph=graph)
            assert_same_ch(a, gpu_export(ch), f"{name} graph={graph}")
            assert sum(1 for r in ch.round_stats() if r["ls_tier1"] == 6) > 8, name


def test_dense_tail_learned_and_batch(gpu):
    from paper_2412_18008_amd import learned

    off, dst, w = synth.road_like(6000, seed=12)
    n = len(off) - 1
    lab = synth.labels(n, 4)
    weights = learned.init_weights(5)
    o = oracle.OracleCH(off, dst, w, labels=lab, mlp=weights).run()
    ch = gpu.build(off, dst, w, labels=lab, mlp=weights, dense_tail=4096, record=True)
    assert_same_ch(oracle_export(o), gpu_export(ch), "learned tail")
    graphs = [synth.road_like(3000, seed=s) for s in (1, 2, 3)]
    chs = gpu.build_batch(graphs, dense_tail=4096)
    for (goff, gdst, gw), c in zip(graphs, chs):
        assert_same_ch(oracle_export(oracle.OracleCH(goff, gdst, gw).run()), gpu_export(c),
                       "batch tail vs oracle")

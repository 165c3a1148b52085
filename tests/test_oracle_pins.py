"""Pins of the CPU oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own code:

* the CH preserves every pairwise distance (the definition of a CH in
  Sec. "Contraction Hierarchies"), checked against brute-force
  Floyd-Warshall closures computed here in numpy;
* after every round the overlay preserves distances among live vertices;
* every shortcut equals the two-arc path it replaces, and in exact mode its
  weight is the true distance (Alg. 7 adds a shortcut only when the path
  through u is a shortest path);
* the selected set is independent and locally minimal (Alg. 6);
* closed forms of the edge difference (Alg. 5) on a unit 3x3 grid, a star
  and a chain (the chain family adds exactly one shortcut per contraction);
* pruning removes an arc longer than a two-arc detour (end of Alg. 4);
* memo values are exact distances (exact mode) or hop-bounded minima;
* equivariance under vertex renumbering when labels travel with vertices;
* termination: at least one contraction per round, logarithmic rounds on a
  chain with random labels.
"""
import numpy as np
import pytest

import oracle
from paper_2412_18008_amd import synth

INF = np.iinfo(np.int64).max // 4
MODES = [
    dict(wps_mode=oracle.WPS_EXACT),
    dict(wps_mode=oracle.WPS_HOP, hop_limit=2),
    dict(wps_mode=oracle.WPS_HOP, hop_limit=4),
    dict(wps_mode=oracle.WPS_SETTLED, settle_limit=3),
    dict(wps_mode=oracle.WPS_SETTLED, settle_limit=50),
]


def closure(n, src, dst, w):
    """All-pairs shortest distances by Floyd-Warshall (int64, INF = none)."""
    D = np.full((n, n), INF, np.int64)
    np.fill_diagonal(D, 0)
    for a, b, c in zip(src.tolist(), dst.tolist(), w.tolist()):
        if c < D[a, b]:
            D[a, b] = c
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return np.minimum(D, INF)


def graph_closure(off, dst, w):
    src, d, ww = synth.arcs_of(off, dst, w)
    return closure(len(off) - 1, src, d, ww)


def small_graphs():
    out = []
    for s in range(6):
        out.append(("digraph", synth.random_digraph(25, 90, seed=s, wmax=9, zero_frac=0.1,
                                                    loops=True)))
    for s in range(3):
        out.append(("road", synth.random_geometric_small(40, seed=s)))
    out.append(("grid", synth.grid(5, 6, seed=4, wmax=5)))
    out.append(("unitgrid", synth.grid(4, 4, seed=0, wmin=1, wmax=1)))
    out.append(("chain", synth.chain(20, seed=1, directed=True)))
    out.append(("bichain", synth.chain(20, seed=2, directed=False)))
    out.append(("star", synth.star(6, seed=3)))
    out.append(("sparse", synth.random_digraph(30, 20, seed=9, wmax=5)))
    for k in (2, 5):  # the paper's k-NN family (directed, weights 1..32)
        out.append((f"knn{k}", synth.knn_graph(36, k, seed=k)))
    return out


def ch_query_all(o, n):
    s = np.repeat(np.arange(n, dtype=np.uint32), n)
    t = np.tile(np.arange(n, dtype=np.uint32), n)
    d, _ = o.query_batch(s, t)
    return d.reshape(n, n)


@pytest.mark.parametrize("mode", MODES, ids=lambda m: str(m))
def test_query_equals_all_pairs_closure(oracle_lib, mode):
    for name, (off, dst, w) in small_graphs():
        n = len(off) - 1
        D = graph_closure(off, dst, w)
        for lseed in range(3):
            o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, lseed), **mode).run()
            Q = ch_query_all(o, n)
            expect = np.where(D >= INF, np.uint64(0xFFFFFFFFFFFFFFFF), D.astype(np.uint64))
            assert np.array_equal(Q, expect), (name, lseed, mode)


@pytest.mark.parametrize("mode", MODES[:3], ids=lambda m: str(m))
def test_overlay_preserves_distances_every_round(oracle_lib, mode):
    for name, (off, dst, w) in small_graphs()[:8]:
        n = len(off) - 1
        D = graph_closure(off, dst, w)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 11), **mode)
        while o.round() == 1:
            alive = np.nonzero(o.vertex_state()["alive"])[0]
            for s in alive:
                d = o.overlay_dijkstra(int(s))
                got = d[alive].astype(np.float64)
                exp = D[s, alive].astype(np.float64)
                got[d[alive] == np.uint64(0xFFFFFFFFFFFFFFFF)] = np.inf
                exp[D[s, alive] >= INF] = np.inf
                assert np.array_equal(got, exp), (name, s)


def _arc_map(arcs):
    return {(int(a), int(b)): (int(c), int(m)) for a, b, c, m in
            zip(arcs["tail"], arcs["head"], arcs["w"], arcs["mid"])}


@pytest.mark.parametrize("mode", MODES, ids=lambda m: str(m))
def test_shortcuts_equal_replaced_paths(oracle_lib, mode):
    for name, (off, dst, w) in small_graphs():
        n = len(off) - 1
        D = graph_closure(off, dst, w)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 2), **mode).run()
        up, down = _arc_map(o.up()), _arc_map(o.down())
        lvl = o.vertex_state()["level"]
        for arcs in (up, down):
            for (a, b), (c, mid) in arcs.items():
                assert c >= D[a, b]
                if mid == oracle.NOMID:
                    continue
                # the middle vertex was contracted earlier than both ends,
                # and its incident arcs at that time were a->mid and mid->b
                assert lvl[mid] < lvl[a] and lvl[mid] < lvl[b]
                w1, _ = down[(a, mid)]
                w2, _ = up[(mid, b)]
                assert c == w1 + w2, (name, a, b, mid)
                if mode["wps_mode"] == oracle.WPS_EXACT:
                    assert c == D[a, b]


def test_independent_set_and_local_minimum(oracle_lib):
    for name, (off, dst, w) in small_graphs():
        n = len(off) - 1
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 3))
        lab = o.labels()
        while True:
            before = o.vertex_state()["alive"]
            more = o.round()
            st = o.vertex_state()
            r = o.rounds - 1
            newly = np.nonzero(before & ~st["alive"])[0]
            assert len(newly) >= 1
            assert np.all(st["level"][newly] == r)
            up, down = o.up(), o.down()
            for arcs, own in ((up, "tail"), (down, "head")):
                other = "head" if own == "tail" else "tail"
                sel = np.isin(arcs[own], newly)
                for u, v in zip(arcs[own][sel], arcs[other][sel]):
                    # every neighbour at contraction time is still alive
                    assert st["alive"][v], (name, u, v)
                    ku = (st["pc"][u], lab[u])
                    kv = (st["p"][v], lab[v])
                    assert ku < kv, (name, u, v)
            if not more:
                break
        o.finish()
        lvl = o.vertex_state()["level"]
        up, down = o.up(), o.down()
        assert np.all(lvl[up["tail"]] < lvl[up["head"]])
        assert np.all(lvl[down["head"]] < lvl[down["tail"]])


def _golden(name):
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    for line in open(p):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split()
            vals[int(k)] = int(v)
    return vals


def test_unit_grid_3x3_edge_difference(oracle_lib):
    off, dst, w = synth.grid(3, 3, seed=0, wmin=1, wmax=1)
    exp = _golden("grid3x3_unit_round0_scores.txt")
    o = oracle.OracleCH(off, dst, w, labels=synth.labels(9, 0))
    o.round()
    p = o.vertex_state()["p"]
    for v, val in exp.items():
        assert p[v] == val, (v, p[v], val)


def test_star_edge_difference(oracle_lib):
    for d in (1, 2, 3, 5, 8):
        off, dst, w = synth.star(d, seed=d)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(d + 1, 1))
        o.round()
        p = o.vertex_state()["p"]
        assert p[0] == d * (d - 1) - d
        assert np.all(p[1:] == -1)


def test_directed_chain_one_shortcut_per_contraction(oracle_lib):
    n = 200
    off, dst, w = synth.chain(n, seed=5, directed=True)
    o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 9))
    while True:
        before = o.vertex_state()["alive"]
        alive_ids = np.nonzero(before)[0]
        more = o.round()
        st = o.vertex_state()
        newly = np.nonzero(before & ~st["alive"])[0]
        # interior contracted vertices (both path neighbours alive) add one
        # shortcut each; the overlay stays a directed path over the survivors
        pos = {int(v): i for i, v in enumerate(alive_ids)}
        interior = [u for u in newly if 0 < pos[int(u)] < len(alive_ids) - 1]
        rs = o.round_stats()[-1]
        assert rs["n_shortcuts"] == len(interior)
        ov = o.overlay()
        surv = np.nonzero(st["alive"])[0]
        assert len(ov["tail"]) == max(len(surv) - 1, 0)
        assert np.array_equal(np.sort(ov["tail"]), surv[:-1]) if len(surv) else True
        if not more:
            break


def test_pruning_triangle(oracle_lib):
    # s=0 -> v=2 weight 10; s -> u=1 -> v weights 3 + 3
    off, dst, w = synth.to_csr(3, [0, 0, 1], [2, 1, 2], [10, 3, 3])
    exp = _golden("triangle_prune.txt")
    o = oracle.OracleCH(off, dst, w, labels=np.array([5, 6, 7], np.uint32))
    o.round()
    rs = o.round_stats()[0]
    assert rs["n_pruned"] == exp[0]
    memo = o.memo()
    got = {(int(a), int(b)): int(c) for a, b, c in zip(memo["s"], memo["t"], memo["d"])}
    assert got[(0, 2)] == exp[1]
    o.run()
    for arcs in (o.up(), o.down()):
        assert not any((a, b, c) == (0, 2, 10) for a, b, c in
                       zip(arcs["tail"].tolist(), arcs["head"].tolist(), arcs["w"].tolist()))


def _hop_closure(n, src, dst, w, s, H):
    d = np.full(n, INF, np.int64)
    d[s] = 0
    for _ in range(H):
        nd = d.copy()
        for a, b, c in zip(src.tolist(), dst.tolist(), w.tolist()):
            if d[a] < INF and d[a] + c < nd[b]:
                nd[b] = d[a] + c
        d = nd
    return d


@pytest.mark.parametrize("mode", MODES[:3], ids=lambda m: str(m))
def test_memo_values(oracle_lib, mode):
    for name, (off, dst, w) in small_graphs()[:9]:
        n = len(off) - 1
        D = graph_closure(off, dst, w)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 4), **mode)
        seen = set()
        while True:
            ov = o.overlay()
            more = o.round()
            memo = o.memo()
            for a, b, c in zip(memo["s"].tolist(), memo["t"].tolist(), memo["d"].tolist()):
                if (a, b) in seen:
                    continue
                seen.add((a, b))
                assert c >= D[a, b]
                if mode["wps_mode"] == oracle.WPS_EXACT:
                    assert c == D[a, b], (name, a, b)
                else:
                    hd = _hop_closure(n, ov["tail"], ov["head"], ov["w"], a, mode["hop_limit"])
                    assert c == hd[b], (name, a, b)
            if not more:
                break


def test_no_absent_lookups_exact_and_hop(oracle_lib):
    graphs = small_graphs() + [("road2k", synth.road_like(2000, seed=3))]
    for mode in MODES[:3]:
        for name, (off, dst, w) in graphs:
            o = oracle.OracleCH(off, dst, w, labels=synth.labels(len(off) - 1, 8), **mode).run()
            assert sum(r["n_absent"] for r in o.round_stats()) == 0, (name, mode)


def _export(o):
    vs = o.vertex_state()
    up = {(a, b, c, m) for a, b, c, m in zip(*(o.up()[k].tolist() for k in
                                                ("tail", "head", "w", "mid")))}
    dn = {(a, b, c, m) for a, b, c, m in zip(*(o.down()[k].tolist() for k in
                                                ("tail", "head", "w", "mid")))}
    return vs["level"], vs["pc"], o.rank(), up, dn


def test_permutation_equivariance(oracle_lib):
    for name, (off, dst, w) in small_graphs()[:10]:
        n = len(off) - 1
        lab = synth.labels(n, 6)
        perm = np.random.default_rng(1).permutation(n)
        off2, dst2, w2 = synth.permute(off, dst, w, perm)
        lab2 = np.empty_like(lab)
        lab2[perm] = lab
        a = _export(oracle.OracleCH(off, dst, w, labels=lab).run())
        b = _export(oracle.OracleCH(off2, dst2, w2, labels=lab2).run())
        assert np.array_equal(a[0], b[0][perm])
        assert np.array_equal(a[1], b[1][perm])
        assert np.array_equal(a[2], b[2][perm])
        P = lambda x: int(perm[x]) if x != oracle.NOMID else x  # noqa: E731
        for sa, sb in ((a[3], b[3]), (a[4], b[4])):
            assert {(P(x), P(y), c, P(m)) for x, y, c, m in sa} == sb


def test_chain_rounds_logarithmic(oracle_lib):
    for n in (1000, 100_000):
        off, dst, w = synth.chain(n, seed=3, directed=False)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 5)).run()
        assert o.rounds <= 4 * int(np.log2(n))
        assert all(r["n_selected"] >= 1 for r in o.round_stats())


def test_dijkstra_against_closure(oracle_lib):
    for name, (off, dst, w) in small_graphs():
        D = graph_closure(off, dst, w)
        n = len(off) - 1
        for s in range(n):
            d = oracle.dijkstra(off, dst, w, s)
            exp = np.where(D[s] >= INF, np.uint64(0xFFFFFFFFFFFFFFFF), D[s].astype(np.uint64))
            assert np.array_equal(d, exp)


def test_dijkstra_settle_is_a_prefix_of_dijkstra(oracle_lib):
    # stopped after k settled vertices: exactly the k nearest (up to ties)
    # carry their true distances, every other entry is UINT64_MAX
    off, dst, w = synth.road_like(5000, seed=2)
    full = oracle.dijkstra(off, dst, w, 17)
    reach = int(np.count_nonzero(full != np.uint64(0xFFFFFFFFFFFFFFFF)))
    for k in (1, 10, 777, reach, reach + 50):
        d, c = oracle.dijkstra_settle(off, dst, w, 17, k)
        fin = d != np.uint64(0xFFFFFFFFFFFFFFFF)
        assert c == min(k, reach) == int(fin.sum())
        assert np.array_equal(d[fin], full[fin])
        assert d[17] == 0
        if c < reach:
            assert full[~fin].min() >= d[fin].max()


def test_default_labels_are_fmix32(oracle_lib):
    # MurmurHash3 fmix32 reference values computed here from its definition
    def fmix32(h):
        h ^= h >> 16
        h = (h * 0x85EBCA6B) & 0xFFFFFFFF
        h ^= h >> 13
        h = (h * 0xC2B2AE35) & 0xFFFFFFFF
        h ^= h >> 16
        return h
    for v in (0, 1, 2, 12345, 0xFFFFFFFE):
        for seed in (0, 7, 0x123456789ABCDEF):
            x = v ^ (seed & 0xFFFFFFFF) ^ (seed >> 32)
            assert oracle.default_label(v, seed) == fmix32(x)


def test_errors(oracle_lib):
    off, dst, w = synth.to_csr(3, [0, 1], [1, 2], [1, 2])
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleCH(off, np.array([1, 3], np.uint32), w)
    assert e.value.code == oracle.ORC_E_INVALID
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleCH(off, dst, np.array([1, 0xFFFFFFFF], np.uint32))
    assert e.value.code == oracle.ORC_E_INVALID
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleCH(off, dst, w, labels=np.array([1, 1, 2], np.uint32))
    assert e.value.code == oracle.ORC_E_INVALID
    # a shortcut 0->2 of weight 2^32 - 2 + 1 does not fit 32 bits
    off, dst, w = synth.to_csr(3, [0, 1], [1, 2], [0xFFFFFFFE, 1])
    o = oracle.OracleCH(off, dst, w, labels=np.array([5, 0, 9], np.uint32))
    with pytest.raises(oracle.OracleError) as e:
        o.run()
    assert e.value.code == oracle.ORC_E_OVERFLOW
    # a search radius D_s above 0xFFFFFFFE does not fit the 32-bit memo
    # either, even where no shortcut would need it (1 is contracted last)
    o = oracle.OracleCH(off, dst, w, labels=np.array([0, 5, 9], np.uint32))
    with pytest.raises(oracle.OracleError) as e:
        o.run()
    assert e.value.code == oracle.ORC_E_OVERFLOW
    # max_rounds
    off, dst, w = synth.chain(50, seed=1, directed=False)
    o = oracle.OracleCH(off, dst, w, max_rounds=2)
    with pytest.raises(oracle.OracleError) as e:
        o.run()
    assert e.value.code == oracle.ORC_E_LIMIT


def test_empty_and_isolated(oracle_lib):
    off = np.zeros(1, np.uint64)
    o = oracle.OracleCH(off, np.zeros(0, np.uint32), np.zeros(0, np.uint32)).run()
    assert o.rounds == 0
    off = np.zeros(6, np.uint64)
    o = oracle.OracleCH(off, np.zeros(0, np.uint32), np.zeros(0, np.uint32)).run()
    assert o.rounds == 1
    d, _ = o.query_batch(np.array([0, 1], np.uint32), np.array([0, 2], np.uint32))
    assert d[0] == 0 and d[1] == np.uint64(0xFFFFFFFFFFFFFFFF)


def test_loaded_ch_answers_like_built_ch(oracle_lib):
    for name, (off, dst, w) in small_graphs()[:8] + [("road2k", synth.road_like(2000, seed=3))]:
        n = len(off) - 1
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 4)).run()
        up, dn = o.up(), o.down()
        L = oracle.LoadedCH(o.rank(), up["tail"], up["head"], up["w"], dn["tail"], dn["head"],
                            dn["w"])
        s, t = synth.queries(n, 500, seed=2)
        a = o.query_batch(s, t)
        b = L.query_batch(s, t)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), name


def test_top_ranks_keep_their_distances_in_the_ch(oracle_lib):
    # The query's core table rests on this property of a CH: the CH arcs
    # among the K highest ranks alone give the exact distance between any
    # two of those vertices (a shortest up-down path between two of them
    # climbs from the lower one, so it never drops below it).  Checked by
    # Floyd-Warshall on those arcs against the input graph's closure, for
    # several K, and the core-finished query (searches that stop at the
    # core, then min over core pairs) against the closure for all pairs.
    for name, (off, dst, w) in small_graphs():
        n = len(off) - 1
        full = graph_closure(off, dst, w)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(n, 3)).run()
        rank = o.rank()
        up, dn = o.up(), o.down()
        tails = np.concatenate([up["tail"], dn["tail"]]).astype(np.int64)
        heads = np.concatenate([up["head"], dn["head"]]).astype(np.int64)
        ws = np.concatenate([up["w"], dn["w"]]).astype(np.int64)
        rt, rh = rank[tails], rank[heads]
        by_rank = np.argsort(rank)
        for K in sorted({1, 3, n // 2, n}):
            if K == 0:
                continue
            c0 = n - K
            sel = (rt >= c0) & (rh >= c0)
            core = closure(K, rt[sel] - c0, rh[sel] - c0, ws[sel])
            verts = by_rank[c0:]
            assert np.array_equal(core, full[np.ix_(verts, verts)]), (name, K)
            # upward closures from every vertex below the core, over arcs
            # that leave non-core vertices only
            upw = [[] for _ in range(n)]   # by rank: (higher rank, w) of upward arcs
            dnw = [[] for _ in range(n)]   # by rank: (higher rank, w) of arcs into it
            for a, b, x in zip(rt, rh, ws):
                if a < b:
                    upw[a].append((b, x))
                else:
                    dnw[b].append((a, x))

            def climb(r0, adj):
                d = {r0: 0}
                for r in range(r0, n):  # ranks in increasing order: upward arcs only
                    if r in d and r < c0:
                        for b, x in adj[r]:
                            d[b] = min(d.get(b, INF), d[r] + x)
                return d
            fw = [climb(rank[v], upw) for v in range(n)]
            bw = [climb(rank[v], dnw) for v in range(n)]
            for s in range(n):
                for t in range(n):
                    best = INF
                    for r, x in fw[s].items():
                        if r < c0 and r in bw[t]:
                            best = min(best, x + bw[t][r])
                    for a, x in fw[s].items():
                        if a >= c0:
                            for b, y in bw[t].items():
                                if b >= c0 and core[a - c0, b - c0] < INF:
                                    best = min(best, x + core[a - c0, b - c0] + y)
                    assert best == full[s, t], (name, K, s, t)

"""Pins of the oracle's finer rules against hand-derived fixtures under
tests/golden/ (each fixture states the passage it follows and its
derivation):

* rank order inside a level: by score, then label (Sec. "Postprocessing");
* two middle vertices proposing the same shortcut at the same weight: the
  smaller label wins (Alg. 7, "Step 4: Contract");
* a shortcut no lighter than an existing arc leaves the arc and its middle
  vertex (Alg. 7; "Maintaining the Overlay Graph Dynamically");
* the eight learned-priority inputs of every vertex at contraction
  (contracted neighbours, in/out degree, depth, settled count, ...);
* the settled(theta) witness search: settle order, the source counted
  first, the stop after theta settles (Alg. 4);
* the pop count of a bidirectional CH query, its stopping rule and its
  alternation on equal queue minima (Sec. "Query on Contraction
  Hierarchies");
* per-round counts, scores and memo over whole rounds: which pairs become
  targets (never the source, never a memoized pair), the radius D_s and
  what a bounded search settles or reaches (exact and hop modes), the next
  round's V_W and V_A, absent memo entries counted by the score, and the
  contracted-neighbour term counting each neighbour once (Alg. 3-7).

Each fixture was chosen so that a plausible slip in the rule it covers (a
reversed comparison, a tie broken on the wrong key, a "<" for a "<=", a
swapped operand, a dropped "+1") changes the expected values.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2412_18008_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    """Fixture lines as (keyword, [ints]) in file order; '#' starts a
    comment."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, *v = line.split()
                rows.append((k, [int(x) for x in v]))
    return rows


def graph_of(rows):
    n = next(v[0] for k, v in rows if k == "n")
    arcs = [v for k, v in rows if k == "arc"]
    src = [a[0] for a in arcs]
    dst = [a[1] for a in arcs]
    w = [a[2] for a in arcs]
    off, d, ww = synth.to_csr(n, src, dst, w)
    lab = np.zeros(n, np.uint32)
    for k, v in rows:
        if k == "label":
            lab[v[0]] = v[1]
    return off, d, ww, lab


def overlay_rows(o):
    ov = o.overlay()
    return sorted(zip(ov["tail"].tolist(), ov["head"].tolist(), ov["w"].tolist(),
                      ov["mid"].tolist()))


def test_rank_within_level_by_score(oracle_lib):
    rows = load("rank_within_level.txt")
    off, dst, w, lab = graph_of(rows)
    o = oracle.OracleCH(off, dst, w, labels=lab).run()
    vs, rank = o.vertex_state(), o.rank()
    for k, (v, level, score, r) in ((k, v) for k, v in rows if k == "expect"):
        assert vs["level"][v] == level, v
        assert vs["pc"][v] == score, v
        assert rank[v] == r, (v, rank[v], r)


def test_eplus_equal_weight_smaller_label_middle(oracle_lib):
    rows = load("eplus_equal_via_two_middles.txt")
    off, dst, w, lab = graph_of(rows)
    o = oracle.OracleCH(off, dst, w, labels=lab)
    o.round()
    exp = sorted(tuple(v) for k, v in rows if k == "expect_overlay")
    assert overlay_rows(o) == exp
    assert o.round_stats()[0]["n_shortcuts"] == 1
    assert o.round_stats()[0]["n_pairs_emitted"] == 2
    # the finished CH keeps that middle vertex on the up arc 0 -> 1
    o.run()
    up = o.up()
    sel = (up["tail"] == 0) & (up["head"] == 1)
    assert sel.sum() == 1 and up["mid"][sel][0] == exp[0][3]


def test_equal_weight_shortcut_keeps_existing_arc(oracle_lib):
    rows = load("equal_weight_shortcut_keeps_arc.txt")
    off, dst, w, lab = graph_of(rows)
    o = oracle.OracleCH(off, dst, w, labels=lab)
    o.round()
    rs = o.round_stats()[0]
    assert rs["n_pruned"] == 0
    assert rs["n_pairs_emitted"] == 1  # the tie asks for a shortcut ...
    exp = sorted(tuple(v) for k, v in rows if k == "expect_overlay")
    assert overlay_rows(o) == exp      # ... which the existing arc keeps out


def _squash(x, c):
    x = np.float32(x)
    return np.float32(x / np.float32(x + np.float32(c)))


def test_features_at_contraction(oracle_lib):
    rows = load("features_at_contraction.txt")
    off, dst, w, lab = graph_of(rows)
    o = oracle.OracleCH(off, dst, w, labels=lab, record=True).run()
    x, level = o.features(), o.vertex_state()["level"]
    for v, lv, ed, cn, din, dout, depth, ws, nb, pairs in (
            vals for k, vals in rows if k == "expect"):
        assert level[v] == lv, v
        exp = np.array([np.float32(np.float32(ed) / np.float32(abs(ed) + 8)),
                        _squash(cn, 8), _squash(din, 8), _squash(dout, 8),
                        _squash(depth, 8), _squash(ws, 64), _squash(nb, 8),
                        _squash(pairs, 8)], np.float32)
        assert np.array_equal(x[v], exp), (v, x[v], exp)


@pytest.mark.parametrize("fixture", ["settled_theta_memo.txt", "settled_theta_target_stop.txt"])
def test_settled_theta_memo_and_count(oracle_lib, fixture):
    rows = load(fixture)
    off, dst, w, lab = graph_of(rows)
    for theta, settled, *memo in (vals for k, vals in rows if k == "expect"):
        o = oracle.OracleCH(off, dst, w, labels=lab, wps_mode=oracle.WPS_SETTLED,
                            settle_limit=theta)
        o.round()
        m = o.memo()
        got = sorted(zip(m["s"].tolist(), m["t"].tolist(), m["d"].tolist()))
        exp = sorted(tuple(memo[i:i + 3]) for i in range(0, len(memo), 3))
        assert got == exp, (theta, got, exp)
        assert o.round_stats()[0]["n_settled"] == settled, theta


@pytest.mark.parametrize("fixture", ["query_pop_count.txt", "query_direction_tie.txt",
                                     "query_equal_paths.txt"])
def test_query_pop_count_on_given_ch(oracle_lib, fixture):
    rows = load(fixture)
    n = next(v[0] for k, v in rows if k == "n")
    rank = np.zeros(n, np.uint32)
    for k, v in rows:
        if k == "rank":
            rank[v[0]] = v[1]
    up = [v for k, v in rows if k == "up"]
    dn = [v for k, v in rows if k == "down"]
    col = lambda a, i: np.array([r[i] for r in a], np.uint32)  # noqa: E731
    ch = oracle.LoadedCH(rank, col(up, 0), col(up, 1), col(up, 2), col(dn, 0), col(dn, 1),
                         col(dn, 2))
    for s, t, dist, pops in (vals for k, vals in rows if k == "expect"):
        d, c = ch.query(s, t)
        exp = 0xFFFFFFFFFFFFFFFF if dist < 0 else dist
        assert (d, c) == (exp, pops), (s, t, d, c)


def test_score_weights(oracle_lib):
    rows = load("score_weights.txt")
    off, dst, w, lab = graph_of(rows)
    k_ed, k_cn, k_depth = next(v for k, v in rows if k == "weights")
    o = oracle.OracleCH(off, dst, w, labels=lab, k_ed=k_ed, k_cn=k_cn, k_depth=k_depth).run()
    vs, rank = o.vertex_state(), o.rank()
    for v, level, score, r in (vals for k, vals in rows if k == "expect"):
        assert (vs["level"][v], vs["pc"][v], rank[v]) == (level, score, r), v


def test_score_weights_closed_forms(oracle_lib):
    # round 0 has no contracted vertex, so P = k_ed * ED: on a star the
    # centre's d(d-1) - d and the leaves' -1 scale by k_ed; k_cn and k_depth
    # do not enter
    for d, k_ed in ((3, 3), (5, -2), (8, 7)):
        off, dst, w = synth.star(d, seed=d)
        o = oracle.OracleCH(off, dst, w, labels=synth.labels(d + 1, 1), k_ed=k_ed, k_cn=11,
                            k_depth=-13)
        o.round()
        p = o.vertex_state()["p"]
        assert p[0] == k_ed * (d * (d - 1) - d)
        assert np.all(p[1:] == -k_ed)
    # saturation: a weight that overflows int32 pins the score at the bound
    off, dst, w = synth.star(8, seed=1)
    o = oracle.OracleCH(off, dst, w, labels=synth.labels(9, 1), k_ed=2**31 - 1)
    o.round()
    p = o.vertex_state()["p"]
    assert p[0] == 2**31 - 1 and np.all(p[1:] == -(2**31 - 1))


def test_raw_id_tiebreak(oracle_lib):
    # CH_TIE_RAW_ID: the label of a vertex is its id, so the build equals
    # one with labels 0 .. n-1 given explicitly
    off, dst, w = synth.grid(6, 7, seed=2, wmax=4)
    n = len(off) - 1
    o = oracle.OracleCH(off, dst, w, tiebreak=oracle.TIE_RAW_ID).run()
    assert np.array_equal(o.labels(), np.arange(n, dtype=np.uint32))
    r = oracle.OracleCH(off, dst, w, labels=np.arange(n, dtype=np.uint32)).run()
    assert np.array_equal(o.rank(), r.rank())
    # raw ids and explicit labels together are rejected
    with pytest.raises(oracle.OracleError):
        oracle.OracleCH(off, dst, w, labels=np.arange(n, dtype=np.uint32),
                        tiebreak=oracle.TIE_RAW_ID)


# per-round counters a round-counts fixture may name (orc_round_stats)
ROUND_COUNTERS = ("alive_before", "n_sources", "n_affected", "n_searched", "n_targets",
                  "n_pruned", "n_selected", "n_pairs_emitted", "n_shortcuts", "n_absent",
                  "n_settled", "overlay_arcs")
PARAMS = ("wps_mode", "hop_limit", "settle_limit", "k_ed", "k_cn", "k_depth")


@pytest.mark.parametrize("fixture", ["round_counts_two_rounds.txt", "self_target.txt",
                                     "hop_absent_score.txt", "affected_middles_hop.txt",
                                     "contracted_neighbours_once.txt",
                                     "memo_at_largest_distance.txt",
                                     "stale_entry_and_prune.txt", "hop_radius.txt"])
def test_round_counts_scores_and_memo(oracle_lib, fixture):
    rows = load(fixture)
    off, dst, w, lab = graph_of(rows)
    kw = {k: v[0] for k, v in rows if k in PARAMS}
    o = oracle.OracleCH(off, dst, w, labels=lab, **kw)
    last = max(v[0] for k, v in rows if k in ROUND_COUNTERS or k == "p")
    for r in range(last + 1):
        assert o.round() == 1, (fixture, r)
        p = o.vertex_state()["p"]
        for v, val in (vals[1:] for k, vals in rows if k == "p" and vals[0] == r):
            assert p[v] == val, (fixture, r, v, p[v], val)
    stats = o.round_stats()
    for k, (r, val) in ((k, v) for k, v in rows if k in ROUND_COUNTERS):
        assert stats[r][k] == val, (fixture, r, k, stats[r][k], val)
    exp = sorted(tuple(v) for k, v in rows if k == "memo")
    if exp:
        m = o.memo()
        assert sorted(zip(m["s"].tolist(), m["t"].tolist(), m["d"].tolist())) == exp, fixture

"""Helpers shared by the GPU parity tests: canonical forms of a CH export so
that the GPU library and the oracle can be compared element by element."""
import os
import time

import numpy as np

import oracle

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_T0 = time.time()


def progress(msg):
    """A progress line on stdout and, when SPOCH_TEST_LOG_DIR names a folder
    (relative to the repository root), appended to test_progress.log there,
    for runs whose output pytest captures."""
    line = f"[{time.time() - _T0:8.1f}s] {msg}"
    print(line, flush=True)
    sub = os.environ.get("SPOCH_TEST_LOG_DIR")
    if not sub:
        return
    d = os.path.join(_ROOT, sub)
    try:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "test_progress.log"), "a") as f:
            f.write(line + "\n")
    except OSError:
        pass


def oracle_export(o):
    vs = o.vertex_state()
    up, dn = o.up(), o.down()
    return dict(level=vs["level"], score=vs["pc"], rank=o.rank(),
                up=np.stack([up["tail"], up["head"], up["w"], up["mid"]], 1),
                down=np.stack([dn["tail"], dn["head"], dn["w"], dn["mid"]], 1))


def gpu_export(ch):
    e = ch.export()
    return dict(level=e["level"], score=e["score"], rank=e["rank"],
                up=np.stack([e["up_tail"], e["up_head"], e["up_w"], e["up_mid"]], 1),
                down=np.stack([e["down_tail"], e["down_head"], e["down_w"], e["down_mid"]], 1))


def canon(arcs):
    """Rows sorted lexicographically (tail, head, w, mid)."""
    if len(arcs) == 0:
        return arcs.reshape(0, 4)
    idx = np.lexsort(arcs.T[::-1])
    return arcs[idx]


def assert_same_ch(a, b, ctx=""):
    for k in ("level", "score", "rank"):
        assert np.array_equal(a[k], b[k]), f"{ctx}: {k} differs at " \
            f"{np.nonzero(a[k] != b[k])[0][:10]}"
    for k in ("up", "down"):
        ca, cb = canon(a[k]), canon(b[k])
        assert ca.shape == cb.shape, f"{ctx}: {k} arc count {ca.shape[0]} vs {cb.shape[0]}"
        assert np.array_equal(ca, cb), f"{ctx}: {k} arcs differ"


def assert_export_order(e):
    """Upward arcs sorted by (rank tail, rank head); downward by (rank head,
    rank tail); every arc goes from lower to higher rank."""
    r = e["rank"]
    up, dn = e["up"], e["down"]
    if len(up):
        kt, kh = r[up[:, 0]].astype(np.int64), r[up[:, 1]].astype(np.int64)
        assert np.all(kt < kh)
        key = kt * (1 << 32) + kh
        assert np.all(np.diff(key) > 0)
    if len(dn):
        kt, kh = r[dn[:, 0]].astype(np.int64), r[dn[:, 1]].astype(np.int64)
        assert np.all(kh < kt)
        key = kh * (1 << 32) + kt
        assert np.all(np.diff(key) > 0)


def oracle_round_counts(o):
    return [(r["alive_before"], r["n_sources"], r["n_affected"], r["n_selected"],
             r["n_targets"], r["n_pruned"], r["n_shortcuts"], r["overlay_arcs"])
            for r in o.round_stats()]


def gpu_round_counts(ch):
    return [(r["alive_before"], r["n_sources"], r["n_affected"], r["n_selected"],
             r["n_targets"], r["n_pruned"], r["n_shortcuts"], r["overlay_arcs"])
            for r in ch.round_stats()]


UINT64_MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


def reference_distances(off, dst, w, s, t):
    """Plain Dijkstra (oracle) for each distinct source."""
    out = np.empty(len(s), np.uint64)
    cache = {}
    for i, (a, b) in enumerate(zip(s.tolist(), t.tolist())):
        if a not in cache:
            cache[a] = oracle.dijkstra(off, dst, w, a)
        out[i] = cache[a][b]
    return out


def closure_sizes(o, s, t):
    """|vertices reachable from s over upward arcs| + |vertices that reach t
    over downward arcs|, from the oracle's finished CH (plain reachability)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import breadth_first_order

    n = o.n
    up, dn = o.up(), o.down()
    U = csr_matrix((np.ones(len(up["tail"])), (up["tail"], up["head"])), shape=(n, n))
    D = csr_matrix((np.ones(len(dn["tail"])), (dn["head"], dn["tail"])), shape=(n, n))
    out = np.empty(len(s), np.int64)
    for i, (a, b) in enumerate(zip(s, t)):
        out[i] = (len(breadth_first_order(U, int(a), return_predecessors=False))
                  + len(breadth_first_order(D, int(b), return_predecessors=False)))
    return out

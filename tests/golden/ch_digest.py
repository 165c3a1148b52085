"""Order-independent digest of a finished contraction hierarchy.

Used to store the oracle's result for a graph too large to keep in the
repository (the 24M-vertex clustered road-like graph) and to compare a GPU
build with it: one SHA-256 per array of the canonical form -- level, score
at contraction and rank per vertex (vertex order), upward and downward arcs
as (tail, head, weight, middle vertex) rows sorted lexicographically -- plus
the per-round counts.  Pure numpy and hashlib; it computes nothing of the
construction itself.
"""
import hashlib

import numpy as np

ROUND_FIELDS = ("alive_before", "n_sources", "n_affected", "n_selected", "n_targets",
                "n_pruned", "n_shortcuts", "overlay_arcs")


def _sha(a):
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.view(np.uint8).reshape(-1)).hexdigest()


def canon_arcs(tail, head, w, mid):
    """Rows (tail, head, w, mid) as uint32, sorted lexicographically."""
    rows = np.stack([np.asarray(x, np.uint32) for x in (tail, head, w, mid)], 1)
    if len(rows) == 0:
        return rows.reshape(0, 4)
    key = (rows[:, 0].astype(np.uint64) << np.uint64(32)) | rows[:, 1].astype(np.uint64)
    # (tail, head) pairs are distinct in a CH (one arc per ordered pair)
    return rows[np.argsort(key, kind="stable")]


def digest(level, score, rank, up, down, rounds):
    """up / down: (tail, head, w, mid) tuples of arrays; rounds: list of dicts
    with ROUND_FIELDS."""
    cu, cd = canon_arcs(*up), canon_arcs(*down)
    return {
        "n": int(len(level)),
        "up_arcs": int(len(cu)),
        "down_arcs": int(len(cd)),
        "rounds": len(rounds),
        "level": _sha(np.asarray(level, np.uint32)),
        "score": _sha(np.asarray(score, np.int32)),
        "rank": _sha(np.asarray(rank, np.uint32)),
        "up": _sha(cu),
        "down": _sha(cd),
        "round_counts": [[int(r[f]) for f in ROUND_FIELDS] for r in rounds],
    }

"""Seeded synthetic graphs, labels and query pairs.

These stand in for the road, mesh and chain graphs of the paper's
experiments (its OpenStreetMap, DIMACS and k-NN data are not available):

* ``grid``            64x64-style 4-neighbour grid, independent uniform
                      integer weight per arc (a 2-D mesh with random
                      weights, like the paper's BUB/TRCE inputs);
* ``road_like``       uniform random points, edges to the 3 nearest
                      neighbours, symmetrised, weight = round(1e4 * length)
                      + 1, a fraction of edges one-way;
* ``clustered_road``  the same construction over Gaussian "city" clusters
                      with travel-time weights (length / speed class);
* ``chain``           a path with weights 1..32 (the paper's chain family);
* ``knn_graph``       arcs from every point to its k nearest neighbours with
                      weights 1..32 (the paper's k-NN family);
* ``fan``             a path plus a hub with arcs to all of it (a vertex
                      whose upward search space is the whole graph);
* ``random_digraph``  small random digraphs with self-loops, parallel arcs
                      and zero weights, for input-hygiene tests.

This module only makes inputs.  It contains none of the construction's
arithmetic and is shared by the oracle-side and the GPU-side tests.
Every graph is returned as CSR: ``off`` (uint64, n+1), ``dst`` (uint32, m),
``w`` (uint32, m), arcs of a vertex in generation order.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def to_csr(n, src, dst, w):
    """Group arcs by source (stable), returning (off, dst, w)."""
    src = np.asarray(src, dtype=np.int64)
    order = np.argsort(src, kind="stable")
    cnt = np.bincount(src, minlength=n) if len(src) else np.zeros(n, np.int64)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum(cnt, dtype=np.uint64)
    return (off, np.asarray(dst, dtype=np.uint32)[order].copy(),
            np.asarray(w, dtype=np.uint32)[order].copy())


def arcs_of(off, dst, w):
    """Inverse of to_csr: arrays (src, dst, w)."""
    n = len(off) - 1
    deg = np.diff(off.astype(np.int64))
    src = np.repeat(np.arange(n, dtype=np.uint32), deg)
    return src, np.asarray(dst, np.uint32), np.asarray(w, np.uint32)


def grid(rows, cols, seed=0, wmin=1, wmax=1000):
    """4-neighbour grid, arcs in both directions, each arc an independent
    uniform integer weight in [wmin, wmax]."""
    rng = _rng(seed)
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    pairs = []
    pairs.append((idx[:, :-1].ravel(), idx[:, 1:].ravel()))   # east
    pairs.append((idx[:, 1:].ravel(), idx[:, :-1].ravel()))   # west
    pairs.append((idx[:-1, :].ravel(), idx[1:, :].ravel()))   # south
    pairs.append((idx[1:, :].ravel(), idx[:-1, :].ravel()))   # north
    src = np.concatenate([p[0] for p in pairs])
    dst = np.concatenate([p[1] for p in pairs])
    w = rng.integers(wmin, wmax + 1, size=len(src), dtype=np.int64)
    return to_csr(rows * cols, src, dst, w)


def fan(k, w_hub=1000):
    """A bidirectional unit-weight path 0..k-1 and a hub k with one-way arcs
    of weight w_hub to every path vertex.  The hub has no in-arcs, so it is
    contracted first and its upward search space holds the whole path."""
    i = np.arange(k - 1)
    src = np.concatenate([i, i + 1, np.full(k, k)])
    dst = np.concatenate([i + 1, i, np.arange(k)])
    w = np.concatenate([np.ones(2 * (k - 1), np.int64), np.full(k, w_hub, np.int64)])
    return to_csr(k + 1, src, dst, w)


def _knn_edges(pts, k):
    from scipy.spatial import cKDTree

    tree = cKDTree(pts)
    _, nb = tree.query(pts, k=k + 1, workers=-1)
    n = len(pts)
    i = np.repeat(np.arange(n, dtype=np.int64), k)
    j = nb[:, 1:].reshape(-1).astype(np.int64)
    a = np.minimum(i, j)
    b = np.maximum(i, j)
    key = np.unique(a * n + b)
    return key // n, key % n


def _orient(n, a, b, w, oneway_frac, rng):
    """Both directions for most undirected edges; `oneway_frac` of them keep
    one random direction."""
    ow = rng.random(len(a)) < oneway_frac
    flip = rng.random(len(a)) < 0.5
    two = ~ow
    src = np.concatenate([a[two], b[two], np.where(flip[ow], b[ow], a[ow])])
    dst = np.concatenate([b[two], a[two], np.where(flip[ow], a[ow], b[ow])])
    ww = np.concatenate([w[two], w[two], w[ow]])
    return to_csr(n, src, dst, ww)


def road_like(n, seed=0, k=3, oneway_frac=0.1, scale=1e4):
    """Uniform points in the unit square; undirected edge {i, j} if j is one
    of the k nearest neighbours of i or vice versa; integer weight
    round(scale * Euclidean length) + 1; `oneway_frac` of the edges one-way."""
    rng = _rng(seed)
    pts = rng.random((n, 2))
    a, b = _knn_edges(pts, k)
    ln = np.hypot(*(pts[a] - pts[b]).T)
    w = np.rint(scale * ln).astype(np.int64) + 1
    return _orient(n, a, b, w, oneway_frac, _rng(seed + 2))


def clustered_road(n, seed=0, k=3, oneway_frac=0.1, centres=64, frac_city=0.7,
                   speeds=(30, 50, 80, 110), scale=1.1e6):
    """Road-like graph over clustered points: `centres` Gaussian cities with
    sigma log-uniform in [0.002, 0.03] holding `frac_city` of the points, the
    rest uniform.  Weight = round(scale * length / speed) + 1, the speed class
    chosen by edge-length quartile (longer edges are faster)."""
    rng = _rng(seed)
    nc = int(round(frac_city * n))
    c = rng.random((centres, 2))
    sig = np.exp(rng.uniform(np.log(0.002), np.log(0.03), size=centres))
    which = rng.integers(0, centres, size=nc)
    city = c[which] + rng.standard_normal((nc, 2)) * sig[which, None]
    pts = np.concatenate([city, rng.random((n - nc, 2))])
    pts = pts[rng.permutation(n)]
    a, b = _knn_edges(pts, k)
    ln = np.hypot(*(pts[a] - pts[b]).T)
    q = np.quantile(ln, [0.25, 0.5, 0.75])
    sp = np.asarray(speeds, dtype=np.float64)[np.searchsorted(q, ln)]
    w = np.rint(scale * ln / sp).astype(np.int64) + 1
    return _orient(n, a, b, w, oneway_frac, _rng(seed + 2))


def knn_graph(n, k, seed=0, wmin=1, wmax=32):
    """k-NN graph over n uniform points in the unit square: each vertex has
    arcs to its k nearest other points (m = k n), each with an independent
    uniform integer weight in [wmin, wmax] (the paper's k-NN family: k
    out-going edges per vertex, random weights 1..32)."""
    from scipy.spatial import cKDTree

    rng = _rng(seed)
    pts = rng.random((n, 2))
    _, nb = cKDTree(pts).query(pts, k=k + 1, workers=-1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = nb[:, 1:].reshape(-1).astype(np.int64)
    w = _rng(seed + 1).integers(wmin, wmax + 1, size=len(src), dtype=np.int64)
    return to_csr(n, src, dst, w)


def chain(n, seed=0, directed=True, wmin=1, wmax=32):
    """Path 0 - 1 - ... - n-1 with uniform integer weights; `directed` keeps
    only the forward arcs, else both directions with independent weights."""
    rng = _rng(seed)
    a = np.arange(n - 1, dtype=np.int64)
    if directed:
        src, dst = a, a + 1
    else:
        src, dst = np.concatenate([a, a + 1]), np.concatenate([a + 1, a])
    w = rng.integers(wmin, wmax + 1, size=len(src), dtype=np.int64)
    return to_csr(n, src, dst, w)


def star(d, weights=None, seed=0):
    """Bidirectional star: centre 0, leaves 1..d."""
    rng = _rng(seed)
    leaves = np.arange(1, d + 1, dtype=np.int64)
    w = rng.integers(1, 100, size=d) if weights is None else np.asarray(weights)
    src = np.concatenate([np.zeros(d, np.int64), leaves])
    dst = np.concatenate([leaves, np.zeros(d, np.int64)])
    return to_csr(d + 1, src, dst, np.concatenate([w, w]))


def random_digraph(n, m, seed=0, wmax=20, zero_frac=0.0, loops=False):
    """Uniform random arcs (parallel arcs possible); optional self-loops and
    a fraction of zero weights."""
    rng = _rng(seed)
    src = rng.integers(0, n, size=m)
    dst = rng.integers(0, n, size=m)
    if not loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    w = rng.integers(1, wmax + 1, size=len(src))
    if zero_frac > 0:
        w[rng.random(len(src)) < zero_frac] = 0
    return to_csr(n, src, dst, w)


def random_geometric_small(n, seed=0, k=3, oneway_frac=0.1):
    """Small road-like graph with weights round(1e2 * length) + 1 (many ties)."""
    return road_like(n, seed=seed, k=k, oneway_frac=oneway_frac, scale=1e2)


def labels(n, seed=0):
    """Distinct uint32 tie-break labels: a random permutation of 0..n-1."""
    return _rng(seed).permutation(n).astype(np.uint32)


def queries(n, q, seed=1):
    """q (s, t) pairs drawn uniformly with replacement."""
    rng = _rng(seed)
    return (rng.integers(0, n, size=q).astype(np.uint32),
            rng.integers(0, n, size=q).astype(np.uint32))


def permute(off, dst, w, perm):
    """Relabel vertex v as perm[v] (arc order within a row preserved)."""
    n = len(off) - 1
    src, d, ww = arcs_of(off, dst, w)
    perm = np.asarray(perm, np.int64)
    return to_csr(n, perm[src.astype(np.int64)], perm[d.astype(np.int64)], ww)


# Named workloads.
def config_grid64(seed=0):
    return grid(64, 64, seed=seed)


def config_road1m(seed=0):
    return road_like(1_000_000, seed=seed)


def config_road24m(seed=0):
    return clustered_road(24_000_000, seed=seed)


def batch512_sizes(seed=512, k=512, lo=1e4, hi=5e5):
    """Vertex counts of the batched-construction workload: k sizes
    log-uniform in [lo, hi] (floor), from PCG64(seed)."""
    rng = _rng(seed)
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=k))).astype(np.int64)


def config_batch512(k=512):
    """k road-like graphs (the road-like 1M recipe) with batch512_sizes()
    vertices, graph i from seed i."""
    return [road_like(int(n), seed=i) for i, n in enumerate(batch512_sizes(k=512)[:k])]

"""Pins of the learned-priority reference (CPU):
* the numpy backward equals central finite differences (fp64);
* GELU through the Pade tanh is within 1e-4 of the erf-form GELU (so it is
  a GELU), and the C oracle's single-precision GELU and MLP priority equal
  the fp64 reference within float rounding, and the quantised priority is
  rint(y * 2^q) of the same output;
* the learned oracle build preserves every pairwise distance (several
  quantisations), and with a constant network Select takes exactly the
  label-local minima."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2412_18008_amd import synth
from test_oracle_pins import graph_closure, small_graphs, INF


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    w = mlp.init(3) + rng.standard_normal(mlp.N_PARAMS) * 0.05
    X = rng.random((32, 8)) * 2 - 0.5
    t = rng.random(32)
    g = mlp.grad(w, X, t)
    idx = np.concatenate([rng.choice(512, 40, replace=False), 512 + np.arange(64),
                          576 + rng.choice(4096, 80, replace=False), 4672 + np.arange(129)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(w)
        e[i] = h
        fd = (mlp.loss(w + e, X, t) - mlp.loss(w - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_pade_gelu_is_gelu():
    x = np.linspace(-8, 8, 20001)
    exact = 0.5 * x * (1 + np.vectorize(math.erf)(x / math.sqrt(2)))
    assert np.max(np.abs(mlp.gelu(x) - exact)) < 1e-3
    # tanh form vs erf form differ by < 5e-4; the Pade tanh adds < 1e-4
    tanh_form = 0.5 * x * (1 + np.tanh(mlp.K * (x + mlp.C3 * x ** 3)))
    assert np.max(np.abs(mlp.gelu(x) - tanh_form)) < 1e-4 * (1 + np.max(np.abs(x)))


def test_c_single_precision_matches_reference():
    rng = np.random.default_rng(1)
    for x in np.concatenate([np.linspace(-7, 7, 301), rng.standard_normal(100)]):
        assert abs(oracle.gelu(x) - mlp.gelu(np.float32(x))) <= 2e-6 * (1 + abs(x))
    w = mlp.init(5).astype(np.float32)
    X = rng.random((50, 8)).astype(np.float32)
    y_ref, _ = mlp.forward(w.astype(np.float64), X.astype(np.float64))
    for i in range(50):
        p, y = oracle.mlp_priority(w, X[i])
        assert abs(y - y_ref[i]) <= 1e-4 * (1 + abs(y_ref[i]))
        assert p == int(np.clip(np.rint(np.float32(y) * np.float32(65536)), -2**31, 2**31 - 1))
        for q in (1, 3, 8, 24):  # quantised output: rint(y * 2^q), the same y
            pq, yq = oracle.mlp_priority(w, X[i], q)
            assert yq == y
            assert pq == int(np.clip(np.rint(np.float64(y) * 2.0 ** q), -2**31, 2**31 - 1))


def test_learned_build_preserves_distances(oracle_lib):
    w = mlp.init(11).astype(np.float32)
    for (name, (off, dst, w_)), q in zip(small_graphs()[:10], (0, 2, 0, 4, 0, 1, 0, 8, 0, 2)):
        n = len(off) - 1
        D = graph_closure(off, dst, w_)
        o = oracle.OracleCH(off, dst, w_, labels=synth.labels(n, 1), mlp=w, record=True,
                            mlp_qbits=q).run()
        s = np.repeat(np.arange(n, dtype=np.uint32), n)
        t = np.tile(np.arange(n, dtype=np.uint32), n)
        d, _ = o.query_batch(s, t)
        exp = np.where(D >= INF, np.uint64(0xFFFFFFFFFFFFFFFF), D.astype(np.uint64)).ravel()
        assert np.array_equal(d, exp), name
        f = o.features()
        assert np.all(np.isfinite(f)) and np.all(np.abs(f) < 1.0)


def test_quantised_priority_ties_follow_labels(oracle_lib):
    # a network whose output is 0.3 for every input: with 1 fractional bit
    # every priority is rint(0.6) = 1, so Select takes the local minima of the
    # labels alone; with 16 bits too (all equal); the round-0 selection must
    # then be exactly the vertices whose label is below every neighbour's
    w = np.zeros(4801, np.float32)
    w[4800] = np.float32(0.3)
    off, dst, w_ = synth.grid(6, 7, seed=4)
    n = len(off) - 1
    lab = synth.labels(n, 2)
    nb = [set() for _ in range(n)]
    for u in range(n):
        for e in range(off[u], off[u + 1]):
            if dst[e] != u:
                nb[u].add(int(dst[e]))
                nb[int(dst[e])].add(u)
    expect = sum(1 for u in range(n) if all(lab[u] < lab[v] for v in nb[u]))
    for q in (1, 16):
        o = oracle.OracleCH(off, dst, w_, labels=lab, mlp=w, mlp_qbits=q)
        o.round()
        assert o.round_stats()[0]["n_selected"] == expect, q
    with pytest.raises(oracle.OracleError):
        oracle.OracleCH(off, dst, w_, mlp=w, mlp_qbits=25)


def test_priority_rounding_and_saturation(oracle_lib):
    # The priority is the output scaled by 2^qbits, rounded to nearest (ties
    # to even) and saturated to int32; a NaN output saturates high.  With
    # every weight zero but the output bias b3, the output is b3 exactly.
    w = np.zeros(4801, np.float32)
    x = np.zeros(8, np.float32)
    cases = [
        (0.5, 16, 32768),              # exact
        (2.5 / 65536, 16, 2),          # 2.5 rounds to even 2
        (3.5 / 65536, 16, 4),          # 3.5 rounds to even 4
        (-2.5 / 65536, 16, -2),
        (0.375, 3, 3),                 # 3 fractional bits: 0.375 * 8 = 3
        (0.4375, 3, 4),                # 3.5 -> 4
        (32767.0, 16, 2**31 - 2**16),  # in range: exact
        (32768.0, 16, 2**31 - 1),      # 2^31 does not fit: saturates high
        (1e6, 16, 2**31 - 1),
        (-32768.0, 16, -2**31),        # -2^31 fits exactly
        (-1e6, 16, -2**31),            # saturates low
        (float("nan"), 16, 2**31 - 1),
    ]
    for b3, q, exp in cases:
        w[4800] = b3
        p, y = oracle.mlp_priority(w, x, qbits=q)
        if b3 == b3:
            assert y == np.float32(b3)
        assert p == exp, (b3, q, p, exp)

"""Pins of the learned-priority reference (CPU):
* the numpy backward equals central finite differences (fp64);
* GELU through the Pade tanh is within 1e-4 of the erf-form GELU (so it is
  a GELU), and the C oracle's single-precision GELU and MLP priority equal
  the fp64 reference within float rounding;
* the learned oracle build preserves every pairwise distance."""
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


def test_learned_build_preserves_distances(oracle_lib):
    w = mlp.init(11).astype(np.float32)
    for name, (off, dst, w_) in small_graphs()[:10]:
        n = len(off) - 1
        D = graph_closure(off, dst, w_)
        o = oracle.OracleCH(off, dst, w_, labels=synth.labels(n, 1), mlp=w, record=True).run()
        s = np.repeat(np.arange(n, dtype=np.uint32), n)
        t = np.tile(np.arange(n, dtype=np.uint32), n)
        d, _ = o.query_batch(s, t)
        exp = np.where(D >= INF, np.uint64(0xFFFFFFFFFFFFFFFF), D.astype(np.uint64)).ravel()
        assert np.array_equal(d, exp), name
        f = o.features()
        assert np.all(np.isfinite(f)) and np.all(np.abs(f) < 1.0)

"""Learned priority: training data from plain builds, training on the GPU.

The network (an MLP 8 -> 64 -> 64 -> 1 with GELU, see ``include/spoch.h``)
maps the features of a rescored vertex to its priority.  It is trained to
predict when the plain method (edge difference) contracts a vertex: for
every vertex of a training graph the features it had at contraction are the
input, and its level divided by the graph's last level is the target (MSE).
Used as a priority, it orders contraction like the plain method but from a
smoother signal; Select and everything else are unchanged, so distances
stay exact whatever the weights.  Training runs in the library's own GPU
kernels (``ch_mlp_train``).
"""
from __future__ import annotations

import numpy as np

from . import binding, synth

N_PARAMS = binding.CH_MLP_PARAMS


def init_weights(seed=0):
    """He-style initial weights (PCG64), float32, in the library's layout."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.standard_normal((64, 8)) * np.sqrt(2.0 / 8)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    W3 = rng.standard_normal(64) * np.sqrt(1.0 / 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3,
                           [0.0]]).astype(np.float32)


def training_graphs(count, seed0=1000, nmin=10_000, nmax=100_000):
    """Road-like graphs (3-NN, weight round(1e4 length)+1, 10% one-way) with
    n log-uniform in [nmin, nmax], seeds seed0 .. seed0+count-1."""
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        n = int(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        yield synth.road_like(n, seed=seed0 + i)


def record(graphs):
    """(X, t): features at contraction and normalised contraction level of
    every vertex of every graph, from plain builds on the GPU."""
    xs, ts = [], []
    for off, dst, w in graphs:
        ch = binding.build(off, dst, w, record=True)
        x = ch.features()
        lvl = ch.export()["level"].astype(np.float64)
        last = max(lvl.max(), 1.0) if len(lvl) else 1.0
        xs.append(x)
        ts.append((lvl / last).astype(np.float32))
        ch.free()
    return np.concatenate(xs), np.concatenate(ts)


def train(X, t, steps=2000, batch=4096, lr=2e-3, seed=0, init_seed=0):
    """Trained weights and the per-step batch losses."""
    return binding.mlp_train(X, t, init_weights(init_seed), batch=batch, steps=steps, lr=lr,
                             seed=seed)


def main():
    import argparse
    import json
    import time

    ap = argparse.ArgumentParser(description="train the learned priority on the GPU")
    ap.add_argument("--graphs", type=int, default=200)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", required=True, help="output .npy file of 4801 float32 weights")
    args = ap.parse_args()
    t0 = time.time()
    xs, ts = [], []
    for i, g in enumerate(training_graphs(args.graphs)):
        x, y = record([g])
        xs.append(x)
        ts.append(y)
        if (i + 1) % 20 == 0:
            print(f"[learned] recorded {i + 1}/{args.graphs} graphs", flush=True)
    X, t = np.concatenate(xs), np.concatenate(ts)
    t1 = time.time()
    w, losses = train(X, t, steps=args.steps, batch=args.batch, lr=args.lr)
    t2 = time.time()
    np.save(args.out, w)
    print(json.dumps(dict(samples=int(len(X)), graphs=args.graphs, record_s=t1 - t0,
                          train_s=t2 - t1, loss_first=float(losses[:50].mean()),
                          loss_last=float(losses[-50:].mean()), steps=args.steps,
                          batch=args.batch, lr=args.lr)))


if __name__ == "__main__":
    main()

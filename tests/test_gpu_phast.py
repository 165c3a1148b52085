"""One-to-all and many-to-many distances on the built CH (the paper's SSSP
on a CH: an upward search from the source, then a downward pass over the
levels from the top; PHAST's level grouping) against plain Dijkstra on the
input graph, which is exact: every row must equal Dijkstra's distances bit
for bit, unreachable vertices included."""
import numpy as np
import pytest

import oracle
from paper_2412_18008_amd import synth
from parity_util import progress

pytestmark = pytest.mark.gpu

INF = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18008_amd import binding

    binding.lib()
    return binding


def _rows(off, dst, w, srcs):
    return np.stack([oracle.dijkstra(off, dst, w, int(s)) for s in srcs])


def test_one_to_all_small_and_grid(gpu):
    cases = [("digraph", synth.random_digraph(300, 700, seed=3, wmax=9, zero_frac=0.1)),
             ("grid64", synth.config_grid64(seed=0)),
             ("fan", synth.fan(3000)),
             ("knn5", synth.knn_graph(5000, 5, seed=5)),
             ("chain", synth.chain(2000, seed=1, directed=True))]
    for name, (off, dst, w) in cases:
        n = len(off) - 1
        ch = gpu.build(off, dst, w, labels=synth.labels(n, 2))
        rng = np.random.Generator(np.random.PCG64(7))
        # 1, 3, 17 and 70 sources: passes of 1, 4, 64 lanes, and two passes
        for k in (1, 3, 17, 70):
            srcs = rng.integers(0, n, size=k).astype(np.uint32)
            got = ch.one_to_all(srcs)
            assert got.shape == (k, n)
            assert np.array_equal(got, _rows(off, dst, w, srcs)), (name, k)
        progress(f"one_to_all {name}: equal to Dijkstra")
    # unreachable vertices are UINT64_MAX
    assert np.any(got == INF) or name != "chain"


def test_many_to_many_and_device(gpu):
    import torch

    off, dst, w = synth.road_like(30_000, seed=4)
    n = len(off) - 1
    ch = gpu.build(off, dst, w)
    rng = np.random.Generator(np.random.PCG64(9))
    srcs = rng.integers(0, n, size=20).astype(np.uint32)
    tgts = rng.integers(0, n, size=50).astype(np.uint32)
    ref = _rows(off, dst, w, srcs)
    assert np.array_equal(ch.one_to_all(srcs, tgts), ref[:, tgts])
    dev = torch.device("cuda:0")
    ds = torch.from_numpy(srcs.view(np.int32)).to(dev)
    dt = torch.from_numpy(tgts.view(np.int32)).to(dev)
    got = ch.one_to_all(ds, dt).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref[:, tgts])
    got = ch.one_to_all(ds[:5]).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, ref[:5])
    # a source id out of range is an error, no sweep runs
    with pytest.raises(gpu.ChError) as e:
        ch.one_to_all(np.array([n], np.uint32))
    assert e.value.code == gpu.CH_E_INVALID
    with pytest.raises(gpu.ChError) as e:
        ch.one_to_all(srcs[:2], np.array([0, n + 5], np.uint32))
    assert e.value.code == gpu.CH_E_INVALID

"""ch_query_batch_noalloc -- the query batch that allocates nothing (every
scratch array in one fixed device array per GPU) -- against
ch_query_batch_stats, through the C ABI: two calls in a row, the second
with fewer queries, on CHs whose queries use every query tier.  The fixed
array keeps the previous call's contents, so the second call also checks
that everything that must start cleared is cleared."""
import ctypes as C

import numpy as np
import pytest

from paper_2412_18008_amd import synth
from parity_util import progress

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_18008_amd import binding

    binding.lib()
    return binding


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to("cuda:0")


def _stats_on_device(gpu, ch, s, t):
    """ch_query_batch_stats with device arrays (the existing entry point)."""
    import torch

    q = s.numel()
    dist = torch.empty(q, dtype=torch.int64, device=s.device)
    vis = torch.empty(q, dtype=torch.int32, device=s.device)
    st = torch.cuda.current_stream().cuda_stream
    rc = gpu.lib().ch_query_batch_stats(ch.h, s.data_ptr(), t.data_ptr(), q, dist.data_ptr(),
                                        vis.data_ptr(), gpu.CH_Q_ON_DEVICE, st)
    assert rc == gpu.CH_OK, gpu.lib().ch_last_error()
    return dist.cpu().numpy(), vis.cpu().numpy()


def _cases():
    # road-like (first two tiers), fans whose hub queries need the
    # 16384-slot global tier (k = 13000) and the last tier (k = 60000)
    out = [("road30k", synth.road_like(30_000, seed=4), None)]
    for k in (13000, 60000):
        out.append((f"fan{k}", synth.fan(k), k))
    return out


def test_noalloc_equals_query_batch(gpu):
    for name, (off, dst, w), hub in _cases():
        n = len(off) - 1
        ch = gpu.build(off, dst, w, labels=synth.labels(n, 7))
        s, t = synth.queries(n, 5000, seed=11)
        if hub is not None:  # hub queries reach the upper tiers (one at a time
            s[:6] = hub       # in the fixed array's single last-tier table)
        ds, dt = _dev(s), _dev(t)
        ref_d, ref_v = _stats_on_device(gpu, ch, ds, dt)
        progress(f"noalloc {name}: n={n}, reference done")
        # two calls in a row, the second with a smaller input
        for q in (len(s), 1234):
            d, v = ch.query_noalloc(ds[:q], dt[:q])
            assert np.array_equal(d.cpu().numpy(), ref_d[:q]), (name, q)
            assert np.array_equal(v.cpu().numpy(), ref_v[:q]), (name, q)
            d, _ = ch.query_noalloc(ds[:q], dt[:q], visited=False, window=1)
            assert np.array_equal(d.cpu().numpy(), ref_d[:q]), (name, q, "window 1")
        progress(f"noalloc {name}: equal")


def test_noalloc_errors(gpu):
    off, dst, w = synth.grid(20, 20, seed=1)
    n = len(off) - 1
    ch = gpu.build(off, dst, w)
    s, t = synth.queries(n, 100, seed=2)
    L = gpu.lib()
    dist = np.empty(100, np.uint64)
    # host arrays are refused (the call would have to stage them)
    rc = L.ch_query_batch_noalloc(ch.h, s.ctypes.data, t.ctypes.data, 100, dist.ctypes.data,
                                  None, 0, None)
    assert rc == gpu.CH_E_INVALID and "CH_Q_ON_DEVICE" in L.ch_last_error().decode()
    # an id >= n
    bad = s.copy()
    bad[5] = n
    with pytest.raises(RuntimeError):
        ch.query_noalloc(_dev(bad), _dev(t))
    # nothing to do
    assert L.ch_query_batch_noalloc(ch.h, None, None, 0, None, None, gpu.CH_Q_ON_DEVICE,
                                    None) == gpu.CH_OK


def test_noalloc_limit(gpu):
    # a CH of more than 524,287 vertices whose hub query has an upward search
    # space of a million vertices: past the fixed array's largest table, so
    # the call fails with CH_E_LIMIT; ch_query_batch answers it
    k = 1_000_000
    off, dst, w = synth.fan(k)
    n = len(off) - 1
    ch = gpu.build(off, dst, w)
    progress("noalloc limit: fan of 1M built")
    s = np.array([k, 5, 77], np.uint32)
    t = np.array([3, k - 1, 12], np.uint32)
    # the path queries by ch_query_batch (the hub query's answer, 1000, is the
    # weight of its arc to 3; its search space would take that call long)
    ref = ch.query(s[1:], t[1:])
    assert ref[1] == 65  # 77 -> 12 on the unit-weight path
    progress("noalloc limit: reference queries done")
    with pytest.raises(gpu.ChError) as e:
        ch.query_noalloc(_dev(s), _dev(t))
    assert e.value.code == gpu.CH_E_LIMIT
    # the next call on the same array works
    d, _ = ch.query_noalloc(_dev(s[1:]), _dev(t[1:]))
    assert np.array_equal(d.cpu().numpy().view(np.uint64), ref)

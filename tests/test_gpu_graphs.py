"""Recorded (HIP graph) construction and query batches: every replay equals
the eager result, with eager work and synchronisations between replays."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def _eager(pts, qs, ds, curve, refine):
    idx = sfc.Index(dev(pts), curve, refine=refine)
    off, ids = idx.query(dev(qs), dev(ds))
    return idx, off.clone(), ids.clone()


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_query_graph_replays_equal_eager(curve, refine):
    wl = workload.clustered_loguniform(n=200_000, m=20_000, curve=curve, seed=21)
    idx, off, ids = _eager(wl.points, wl.queries, wl.delta, curve, refine)
    q, d = dev(wl.queries), dev(wl.delta)
    rows = (idx.last_stats()["candidates"] // 64) + 20_000 * 8
    g = sfc.Graph.query(idx, q, d, max_rows=int(rows * 2), ids_cap=ids.numel() + 16)
    for rep in range(4):
        g.launch()
        goff, gids = g.result()
        assert torch.equal(goff, off) and torch.equal(gids, ids), rep
        # eager work between replays
        e_off, e_ids = idx.query(q, d)
        assert torch.equal(e_off, off)
    g.close()


def test_build_graph_rebuilds_in_place():
    wl = workload.batched_uneven(n_sets=30, log2_n=(6, 13), log2_m=(3, 8), seed=22)
    pts = dev(wl.points)
    idx = sfc.Index(pts, MORTON, set_off=wl.set_off)
    k0, i0, x0 = idx.sorted_arrays()
    gb = sfc.Graph.build(idx, pts)
    qset = dev(wl.qset, torch.int32)
    want = idx.query_sets(dev(wl.queries), dev(wl.delta), qset)
    for rep in range(3):
        gb.launch()
        gb.wait()
        k, i, x = idx.sorted_arrays()
        assert torch.equal(k, k0) and torch.equal(i, i0) and torch.equal(x, x0)
        got = idx.query_sets(dev(wl.queries), dev(wl.delta), qset)
        assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1])
    gb.close()


def test_build_graph_follows_new_data():
    rng = np.random.default_rng(23)
    a = rng.random((50_000, 2))
    b = rng.random((50_000, 2))
    buf = dev(a)
    idx = sfc.Index(buf, HILBERT)
    gb = sfc.Graph.build(idx, buf)
    buf.copy_(dev(b))
    gb.launch()
    gb.wait()
    k, i, x = idx.sorted_arrays()
    ok, oi, ox = oracle.build(b, HILBERT)
    assert np.array_equal(sfc.u64(k), ok) and np.array_equal(x.cpu().numpy(), ox)
    gb.close()


def test_sets_query_graph_and_overflow():
    wl = workload.batched_uneven(n_sets=40, log2_n=(6, 14), log2_m=(3, 9), seed=24)
    idx = sfc.Index(dev(wl.points), MORTON, set_off=wl.set_off)
    q, d, qs = dev(wl.queries), dev(wl.delta), dev(wl.qset, torch.int32)
    want = idx.query_sets(q, d, qs)
    rows = idx.last_stats()["candidates"] // 64 + 8 * len(wl.queries)
    g = sfc.Graph.query(idx, q, d, max_rows=int(rows * 2), ids_cap=want[1].numel() + 1, qset=qs)
    for _ in range(3):
        g.launch()
        off, ids = g.result()
        assert torch.equal(off, want[0]) and torch.equal(ids, want[1])
    g.close()
    small = sfc.Graph.query(idx, q, d, max_rows=64, ids_cap=want[1].numel() + 1, qset=qs)
    small.launch()
    with pytest.raises(sfc.CapacityError):
        small.wait()
    small.close()


@pytest.mark.parametrize("chunk", [1, 3, 64])
def test_multi_chunk_compaction(chunk):
    """Compaction in many small chunks (eager: exact count; graph: capacity
    larger than the count, read on the device) equals the oracle."""
    wl = workload.clustered_loguniform(n=120_000, m=6_000, curve=HILBERT, seed=23)
    ref = oracle.query(oracle.build(wl.points, HILBERT), wl.queries, wl.delta, HILBERT,
                       nthreads=4)
    q, d = dev(wl.queries), dev(wl.delta)
    try:
        sfc.debug_chunk_tiles(chunk)
        idx = sfc.Index(dev(wl.points), HILBERT, refine=True)
        off, ids = idx.query(q, d)
        assert np.array_equal(off.cpu().numpy().view(np.uint64), ref[0])
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])
        rows = idx.last_stats()["rows"]
        assert rows > 4 * 64 * chunk            # several chunks
        g = sfc.Graph.query(idx, q, d, max_rows=rows + 5 * 64 * chunk + 17,
                            ids_cap=ids.numel() + 1)
        for rep in range(3):
            g.launch()
            goff, gids = g.result()
            assert torch.equal(goff, off) and torch.equal(gids, ids), rep
        g.close()
        tight = sfc.Graph.query(idx, q, d, max_rows=rows, ids_cap=ids.numel())
        tight.launch()
        goff, gids = tight.result()
        assert torch.equal(goff, off) and torch.equal(gids, ids)
        tight.close()
        short = sfc.Graph.query(idx, q, d, max_rows=rows - 1, ids_cap=ids.numel())
        short.launch()
        with pytest.raises(sfc.CapacityError):
            short.wait()
        short.close()
    finally:
        sfc.debug_chunk_tiles(0)

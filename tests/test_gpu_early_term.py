"""Early termination (occupancy bits of the quadtree nodes down to depth 12):
the bitmap against its definition over the oracle's keys, and query results
unchanged with cells skipped."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import sfc, workload
from snapshots import Model

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
DEPTH = 12


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def expected_bitmap(keys):
    """Bit (4^k - 1)/3 + p set for every prefix p of k = 0..12 key digits."""
    words = np.zeros(((4 ** (DEPTH + 1) - 1) // 3 + 31) // 32, np.uint32)
    keys = np.asarray(keys, np.uint64)
    for k in range(DEPTH + 1):
        if len(keys) == 0:
            break
        pre = np.zeros(1, np.uint64) if k == 0 else np.unique(keys >> np.uint64(64 - 2 * k))
        node = (4 ** k - 1) // 3 + pre.astype(np.int64)
        np.bitwise_or.at(words, node >> 5, (np.uint32(1) << (node & 31).astype(np.uint32)))
    return words


def _sparse_queries(n, m, seed):
    """Clustered points, uniform queries with about 0.2 expected reports at
    the background density: most queries are empty."""
    wl = workload.clustered_uniform_queries(n=n, m=m, curve=MORTON, seed=seed, expected=1.0)
    return wl.points, wl.queries, wl.delta


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_bitmap_matches_definition(curve):
    pts, _, _ = _sparse_queries(80_000, 10, 51)
    idx = sfc.Index(dev(pts), curve, early_term=True)
    got = idx.occupancy().cpu().numpy().view(np.uint32)
    keys = oracle.build(pts, curve)[0]
    assert np.array_equal(got, expected_bitmap(keys))


@pytest.mark.parametrize("search", [sfc.BINARY, sfc.LEARNED])
@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_results_unchanged_and_cells_pruned(curve, refine, search):
    pts, qs, ds = _sparse_queries(200_000, 20_000, 52)
    qs[:4] = [[0.5, 0.5], [-1.0, 0.5], [0.3, 0.3], [0.9, 0.1]]
    ds[:4] = [2.0, 0.1, 0.0, 0.3]
    ref = oracle.query(oracle.build(pts, curve), qs, ds, curve, nthreads=4)
    idx = sfc.Index(dev(pts), curve, refine=refine, search=search, early_term=True)
    off, ids = idx.query(dev(qs), dev(ds))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])
    st = idx.last_stats()
    plain = sfc.Index(dev(pts), curve, refine=refine, search=search)
    plain.query(dev(qs), dev(ds))
    assert st["pruned"] > 0 and plain.last_stats()["pruned"] == 0
    assert st["candidates"] <= plain.last_stats()["candidates"]


def test_bitmap_follows_updates_and_graph_rebuilds():
    pts, qs, ds = _sparse_queries(60_000, 5_000, 53)
    idx = sfc.Index(dev(pts), HILBERT, refine=True, early_term=True)
    model = Model(pts)
    more = workload.uniform_points(8000, 5353)
    idx.insert(dev(more))
    model.insert(more)
    keys = idx.sorted_arrays()[0].cpu().numpy().view(np.uint64)
    assert np.array_equal(idx.occupancy().cpu().numpy().view(np.uint32), expected_bitmap(keys))
    rng = np.random.default_rng(54)
    gone = rng.choice(len(model.xy), 9000, replace=False)
    idx.erase(dev(gone, torch.int32))
    model.erase(gone)
    ref = model.reference(qs, ds, np.full(len(qs), model.epoch), HILBERT)
    off, ids = idx.query(dev(qs), dev(ds))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])
    keys = idx.sorted_arrays()[0].cpu().numpy().view(np.uint64)   # compacted: live keys only
    assert idx.update_info()["compactions"] == 1
    assert np.array_equal(idx.occupancy().cpu().numpy().view(np.uint32), expected_bitmap(keys))
    # A recorded build rebuilds the bitmap with the arrays.
    fresh = sfc.Index(dev(pts), MORTON, early_term=True)
    other = workload.uniform_points(len(pts), 5454)
    g = sfc.Graph.build(fresh, dev(other))
    g.launch()
    g.wait()
    want = expected_bitmap(oracle.build(other, MORTON)[0])
    assert np.array_equal(fresh.occupancy().cpu().numpy().view(np.uint32), want)
    g.close()


@pytest.mark.parametrize("refine", [False, True])
def test_graph_replays_with_early_term(refine):
    """Recorded query batches over the dense (query, cell) work list: every
    replay equals the oracle, with eager batches between replays (the list's
    order across blocks varies from run to run; the results may not)."""
    pts, qs, ds = _sparse_queries(150_000, 12_000, 55)
    ref = oracle.query(oracle.build(pts, MORTON), qs, ds, MORTON, nthreads=4)
    idx = sfc.Index(dev(pts), MORTON, refine=refine, early_term=True)
    q, d = dev(qs), dev(ds)
    off, ids = idx.query(q, d)
    rows = idx.last_stats()["candidates"] // 64 + 8 * len(qs)
    g = sfc.Graph.query(idx, q, d, max_rows=int(rows * 2), ids_cap=ids.numel() + 16)
    for rep in range(4):
        g.launch()
        goff, gids = g.result()
        assert np.array_equal(goff.cpu().numpy().view(np.uint64), ref[0]), rep
        assert np.array_equal(gids.cpu().numpy().view(np.uint32), ref[1]), rep
        e_off, e_ids = idx.query(q, d)
        assert torch.equal(e_off, off) and torch.equal(e_ids, ids)
    g.close()


def test_sets_refuse_early_term():
    """An index of several point sets keeps no occupancy bits (the bits would
    have to be per set): asking for them is refused, not ignored."""
    wl = workload.batched_uneven(n_sets=5, log2_n=(6, 9), log2_m=(3, 5), seed=56)
    with pytest.raises(sfc.SfcError) as ei:
        sfc.Index(dev(wl.points), HILBERT, set_off=wl.set_off, early_term=True)
    assert ei.value.status == sfc.SFC_ERR_UNSUPPORTED


@pytest.mark.parametrize("bad", [(0.5, 0.5, -1.0), (float("nan"), 0.5, 0.1)])
def test_invalid_query_with_early_term(bad):
    pts, qs, ds = _sparse_queries(20_000, 500, 57)
    qs[123], ds[123] = bad[:2], bad[2]
    idx = sfc.Index(dev(pts), MORTON, refine=True, early_term=True)
    with pytest.raises(sfc.SfcError) as ei:
        idx.query(dev(qs), dev(ds))
    assert ei.value.status == sfc.SFC_ERR_INVALID
    off, ids = idx.query(torch.empty((0, 2), dtype=torch.float64, device=DEV),
                         torch.empty(0, dtype=torch.float64, device=DEV))
    assert off.cpu().tolist() == [0] and ids.numel() == 0

"""Square-window (L-infinity) queries through the C ABI against the oracle's
window test: plain, refined, learned, with early termination, with point
sets, after updates, recorded in a graph, and the metric switch."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, LINF, MORTON
from paper_2508_19891_amd import sfc, workload
from snapshots import Model
from test_oracle import _window_adversarial

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def check(idx, pts, qs, ds, curve):
    ref = oracle.query(oracle.build(pts, curve), qs, ds, curve, nthreads=4, metric=LINF)
    off, ids = idx.query(dev(qs), dev(ds))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])
    return ref


@pytest.mark.parametrize("early_term", [False, True])
@pytest.mark.parametrize("search", [sfc.BINARY, sfc.LEARNED])
@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_windows_match_oracle(curve, refine, search, early_term):
    wl = workload.square_windows(n=150_000, m=15_000, side=4e-3, curve=curve, seed=61,
                                 points="clustered")
    ds = wl.delta * workload.loguniform(np.random.default_rng(62), 0.05, 20.0, len(wl.delta))
    idx = sfc.Index(dev(wl.points), curve, refine=refine, search=search, early_term=early_term,
                    metric=sfc.LINF)
    ref = check(idx, wl.points, wl.queries, ds, curve)
    assert ref[1].size > 100_000


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_windows_adversarial_edges(curve):
    rng = np.random.default_rng(63 + curve)
    pts, qs, ds = _window_adversarial(rng)
    for refine in (False, True):
        idx = sfc.Index(dev(pts), curve, refine=refine, metric=sfc.LINF)
        check(idx, pts, qs, ds, curve)


def test_windows_grid_boundaries():
    """Dyadic grid points on the window's edges and corners are reported."""
    g = 256
    ii, jj = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    pts = np.stack([ii.ravel() / g, jj.ravel() / g], 1)
    rng = np.random.default_rng(64)
    a = rng.integers(0, g, (2000, 2))
    k = rng.integers(0, 9, 2000)
    qs = a / g
    ds = k / g
    idx = sfc.Index(dev(pts), HILBERT, refine=True, metric=sfc.LINF)
    ref = check(idx, pts, qs, ds, HILBERT)
    lo = np.clip(a - k[:, None], 0, g - 1)
    hi = np.clip(a + k[:, None], 0, g - 1)
    want = (hi[:, 0] - lo[:, 0] + 1) * (hi[:, 1] - lo[:, 1] + 1)
    assert np.array_equal(np.diff(ref[0].astype(np.int64)), want)


def test_metric_switch_and_graph_keeps_its_metric():
    wl = workload.square_windows(n=100_000, m=8_000, side=1e-2, curve=MORTON, seed=65)
    idx = sfc.Index(dev(wl.points), MORTON, refine=True)
    q, d = dev(wl.queries), dev(wl.delta)
    l2 = oracle.query(oracle.build(wl.points, MORTON), wl.queries, wl.delta, MORTON, nthreads=4)
    off, ids = idx.query(q, d)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), l2[1])
    idx.set_metric(sfc.LINF)
    ref = check(idx, wl.points, wl.queries, wl.delta, MORTON)
    rows = idx.last_stats()["candidates"] // 64 + 8 * len(wl.queries)
    g = sfc.Graph.query(idx, q, d, max_rows=int(rows * 2), ids_cap=int(ref[0][-1]) + 16)
    idx.set_metric(sfc.L2)
    for rep in range(3):
        g.launch()
        goff, gids = g.result()
        assert np.array_equal(gids.cpu().numpy().view(np.uint32), ref[1]), rep
        e_off, e_ids = idx.query(q, d)                      # eager: the Euclidean test now
        assert np.array_equal(e_ids.cpu().numpy().view(np.uint32), l2[1])
    g.close()
    with pytest.raises(sfc.SfcError) as ei:
        idx.set_metric(7)
    assert ei.value.status == sfc.SFC_ERR_INVALID


def test_windows_with_sets_and_updates():
    wl = workload.batched_uneven(n_sets=20, log2_n=(6, 13), log2_m=(3, 9), seed=66)
    idx = sfc.Index(dev(wl.points), HILBERT, set_off=wl.set_off, metric=sfc.LINF)
    off, ids = idx.query_sets(dev(wl.queries), dev(wl.delta), dev(wl.qset, torch.int32))
    off = off.cpu().numpy().view(np.uint64)
    ids = ids.cpu().numpy().view(np.uint32)
    for s in range(20):
        a, b = int(wl.set_off[s]), int(wl.set_off[s + 1])
        sel = np.nonzero(wl.qset == s)[0]
        if len(sel) == 0:
            continue
        r = oracle.brute(wl.points[a:b], wl.queries[sel], wl.delta[sel], metric=LINF)
        for t, j in enumerate(sel):
            got = np.sort(ids[off[j]:off[j + 1]].astype(np.int64) - a)
            assert np.array_equal(got, r[1][r[0][t]:r[0][t + 1]]), (s, j)
    # dynamic index: inserts and erases, answered at the current epoch
    pts = workload.uniform_points(40_000, 67)
    dyn = sfc.Index(dev(pts), MORTON, refine=True, metric=sfc.LINF)
    model = Model(pts)
    more = workload.uniform_points(6_000, 68)
    dyn.insert(dev(more))
    model.insert(more)
    gone = np.random.default_rng(69).choice(len(model.xy), 3_000, replace=False)
    dyn.erase(dev(gone, torch.int32))
    model.erase(gone)
    qs = workload.uniform_points(3_000, 70)
    ds = np.full(3_000, 0.01)
    want = model.reference(qs, ds, np.full(3_000, model.epoch), MORTON, metric=LINF)
    off, ids = dyn.query(dev(qs), dev(ds))
    assert np.array_equal(off.cpu().numpy().view(np.uint64), want[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1])

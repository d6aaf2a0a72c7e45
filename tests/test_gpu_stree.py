"""The static search tree (a third search) through the C ABI: its index
ranges equal the oracle's lower/upper bounds, at sizes on and around the
tree's layer boundaries and with runs of equal keys longer than a block;
query results equal the oracle with every other option; the tree follows
inserts, compactions and recorded builds."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, LINF, MORTON
from paper_2508_19891_amd import sfc, workload
from snapshots import Model

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def _points(n, seed):
    """Uniform points with a third of them on 7 spots (runs of equal keys of
    about n/21, longer than 16 and 256 for the larger n)."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    k = n // 3
    if k:
        spots = rng.random((7, 2))
        pts[:k] = spots[rng.integers(0, 7, k)]
        pts = pts[rng.permutation(n)]
    return pts, rng


@pytest.mark.parametrize("n", [1, 15, 16, 17, 255, 256, 257, 4095, 4096, 4097, 65537, 300_000])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_stree_index_ranges(curve, n):
    pts, rng = _points(n, 81 + n)
    m = 600
    qs = rng.random((m, 2))
    ds = 10 ** rng.uniform(-6, -0.5, m)
    qs[:7] = pts[:7]                   # on points (duplicated spots among them)
    ds[:7] = 1e-9
    qs[7], ds[7] = (0.5, 0.5), 2.0     # the whole domain: upper key 2^64 - 1
    qs[8], ds[8] = (0.0, 0.0), 0.0
    idx = sfc.Index(dev(pts), curve, search=sfc.STREE)
    klo, khi, b, e, nr = idx.query_ranges(dev(qs), dev(ds))
    sk = oracle.build(pts, curve)[0]
    b, e, nr = b.cpu().numpy(), e.cpu().numpy(), nr.cpu().numpy()
    for j in range(m):
        ir = oracle.index_ranges(sk, qs[j, 0], qs[j, 1], ds[j], curve)
        assert nr[j] == len(ir), j
        for r, (bb, ee) in enumerate(ir):
            assert (int(b[j, r]), int(e[j, r])) == (bb, ee), (j, r)
    off, ids = idx.query(dev(qs), dev(ds))
    ref = oracle.query(oracle.build(pts, curve), qs, ds, curve)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])


@pytest.mark.parametrize("early_term", [False, True])
@pytest.mark.parametrize("metric", [sfc.L2, sfc.LINF])
@pytest.mark.parametrize("refine", [False, True])
def test_stree_queries_match_oracle(refine, metric, early_term):
    wl = workload.clustered_loguniform(n=250_000, m=20_000, curve=HILBERT, seed=82)
    idx = sfc.Index(dev(wl.points), HILBERT, search=sfc.STREE, refine=refine, metric=metric,
                    early_term=early_term)
    off, ids = idx.query(dev(wl.queries), dev(wl.delta))
    ref = oracle.query(oracle.build(wl.points, HILBERT), wl.queries, wl.delta, HILBERT,
                       nthreads=4, metric=LINF if metric == sfc.LINF else oracle.L2)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])


def test_stree_switch_updates_and_graphs():
    pts = workload.uniform_points(60_000, 83)
    qs = workload.uniform_points(4_000, 84)
    ds = np.full(4_000, 0.008)
    idx = sfc.Index(dev(pts), MORTON, refine=True)
    model = Model(pts)
    want = model.reference(qs, ds, np.zeros(4_000, np.int64), MORTON)
    for search in (sfc.STREE, sfc.LEARNED, sfc.STREE, sfc.BINARY):
        idx.set_search(search)
        off, ids = idx.query(dev(qs), dev(ds))
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1]), search
    idx.set_search(sfc.STREE)
    # inserts grow the tree (past a layer boundary), erases then a compaction rebuild it
    for k, seed in ((20_000, 85), (200_000, 86)):
        more = workload.uniform_points(k, seed)
        idx.insert(dev(more))
        model.insert(more)
        want = model.reference(qs, ds, np.full(4_000, model.epoch), MORTON)
        off, ids = idx.query(dev(qs), dev(ds))
        assert np.array_equal(off.cpu().numpy().view(np.uint64), want[0])
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1])
    gone = np.random.default_rng(87).choice(len(model.xy), 60_000, replace=False)
    idx.erase(dev(gone, torch.int32))
    model.erase(gone)
    assert idx.update_info()["compactions"] >= 1
    want = model.reference(qs, ds, np.full(4_000, model.epoch), MORTON)
    off, ids = idx.query(dev(qs), dev(ds))
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1])
    # a recorded build rebuilds the tree over the new keys
    fresh = sfc.Index(dev(pts), HILBERT, search=sfc.STREE)
    other = workload.uniform_points(len(pts), 88)
    g = sfc.Graph.build(fresh, dev(other))
    for _ in range(2):
        g.launch()
        g.wait()
        off, ids = fresh.query(dev(qs), dev(ds))
        ref = oracle.query(oracle.build(other, HILBERT), qs, ds, HILBERT)
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])
    g.close()
    # and a recorded query batch
    q, d = dev(qs), dev(ds)
    off, ids = fresh.query(q, d)
    rows = fresh.last_stats()["candidates"] // 64 + 8 * len(qs)
    gq = sfc.Graph.query(fresh, q, d, max_rows=int(rows * 2), ids_cap=ids.numel() + 16)
    for _ in range(3):
        gq.launch()
        goff, gids = gq.result()
        assert torch.equal(goff, off) and torch.equal(gids, ids)
    gq.close()


def test_sets_refuse_stree():
    wl = workload.batched_uneven(n_sets=4, log2_n=(6, 9), log2_m=(3, 5), seed=89)
    with pytest.raises(sfc.SfcError) as ei:
        sfc.Index(dev(wl.points), MORTON, set_off=wl.set_off, search=sfc.STREE)
    assert ei.value.status == sfc.SFC_ERR_UNSUPPORTED
    idx = sfc.Index(dev(wl.points), MORTON, set_off=wl.set_off)
    with pytest.raises(sfc.SfcError) as ei:
        idx.set_search(sfc.STREE)
    assert ei.value.status == sfc.SFC_ERR_UNSUPPORTED

"""Host-side logic without a GPU: the seeded workload generators (shapes,
invariants of the serving trace) and the snapshot model the update and
serving tests judge the GPU against (checked here against brute force)."""
import math

import numpy as np
import pytest

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import workload
from snapshots import LIVE, Model


def test_serving_trace_invariants():
    tr = workload.serving_trace(n0=5000, requests=300, seed=11, log2_size=(4, 8))
    R = len(tr.kind)
    assert R == 300 and set(np.unique(tr.kind)) <= {0, 1, 2}
    # the mix is roughly 40/40/20
    frac = np.bincount(tr.kind, minlength=3) / R
    assert abs(frac[0] - 0.4) < 0.1 and abs(frac[1] - 0.4) < 0.1 and abs(frac[2] - 0.2) < 0.1
    assert (tr.gaps > 0).all()
    # payload slices tile each pool exactly, in stream order
    for kind, pool in ((0, len(tr.queries)), (1, len(tr.inserts)), (2, len(tr.erase_ids))):
        sel = np.nonzero(tr.kind == kind)[0]
        starts, sizes = tr.start[sel], tr.size[sel]
        assert starts[0] == 0 and np.array_equal(starts[1:], np.cumsum(sizes)[:-1])
        assert starts[-1] + sizes[-1] == pool
    # every erased id is live when its request runs (simulated independently)
    live = set(range(5000))
    nxt = 5000
    for r in range(R):
        a, k = int(tr.start[r]), int(tr.size[r])
        if tr.kind[r] == 1:
            live.update(range(nxt, nxt + k))
            nxt += k
        elif tr.kind[r] == 2:
            ids = tr.erase_ids[a:a + k].tolist()
            assert len(set(ids)) == k and set(ids) <= live
            live.difference_update(ids)
    assert (tr.delta > 0).all() and np.isfinite(tr.delta).all()
    assert ((tr.inserts >= 0) & (tr.inserts < 1)).all()


def test_serving_trace_is_seeded():
    a = workload.serving_trace(n0=1000, requests=50, seed=3, log2_size=(3, 6))
    b = workload.serving_trace(n0=1000, requests=50, seed=3, log2_size=(3, 6))
    c = workload.serving_trace(n0=1000, requests=50, seed=4, log2_size=(3, 6))
    assert np.array_equal(a.erase_ids, b.erase_ids) and np.array_equal(a.queries, b.queries)
    assert not np.array_equal(a.initial, c.initial)


def test_batched_uneven_shapes():
    wl = workload.batched_uneven(n_sets=12, log2_n=(4, 8), log2_m=(2, 5), seed=2)
    assert len(wl.set_off) == 13 and wl.set_off[0] == 0
    assert int(wl.set_off[-1]) == len(wl.points)
    assert np.all(np.diff(wl.set_off.astype(np.int64)) >= 1)
    assert np.all(np.diff(wl.qset.astype(np.int64)) >= 0) and wl.qset.max() < 12
    assert len(wl.queries) == len(wl.delta) == len(wl.qset)


def _brute(xy, ids, q, d):
    """Brute force with the paper's test order (closed ball)."""
    out = []
    for (qx, qy), dd in zip(q, d):
        dx = xy[:, 0] - qx
        dy = xy[:, 1] - qy
        s = dx * dx + dy * dy
        out.append(np.sort(ids[s <= dd * dd]))
    return out


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_snapshot_model_against_brute_force(curve):
    """The model's per-epoch answers (the oracle over the snapshot, ids
    mapped back) equal brute force over the points visible at that epoch."""
    rng = np.random.default_rng(5)
    m = Model(rng.random((400, 2)), hold=True)
    m.insert(rng.random((150, 2)))                       # epoch 1
    m.erase(rng.choice(550, 120, replace=False))         # epoch 2
    m.insert(rng.random((60, 2)))                        # epoch 3
    m.erase(np.array([3, 3, 999, 560, 561]))             # epoch 4 (dup, unknown)
    qs = rng.random((40, 2))
    ds = rng.uniform(0.01, 0.3, 40)
    for e in range(5):
        off, ids = m.reference(qs, ds, np.full(40, e), curve)
        vis = m.visible(e)
        want = _brute(m.xy[vis], vis.astype(np.uint32), qs, ds)
        for j in range(40):
            got = np.sort(ids[off[j]:off[j + 1]])
            assert np.array_equal(got, want[j]), (e, j)
    # visibility rules: inserted at epoch 3 invisible before it, erased at 2 invisible after
    assert 560 not in m.visible(2) and 560 in m.visible(3) and 560 not in m.visible(4)


def test_snapshot_model_compaction_policy():
    rng = np.random.default_rng(6)
    m = Model(rng.random((1000, 2)))
    m.erase(np.arange(50))            # 5 %: kept as tombstones
    assert m.compactions == 0 and m.stored.sum() == 1000
    m.erase(np.arange(50, 100))       # 10 % droppable: compacted
    assert m.compactions == 1 and m.stored.sum() == 900
    h = Model(rng.random((1000, 2)), hold=True)
    h.erase(np.arange(200))           # held epochs: nothing droppable
    assert h.compactions == 0
    h.retire(1)
    assert h.compactions == 1 and h.stored.sum() == 800

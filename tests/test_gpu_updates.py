"""Inserts, erases, epochs and compaction on the GPU, checked per query
against the oracle built over the snapshot the query's epoch sees."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import sfc, workload
from snapshots import LIVE, Model

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def check(got, want):
    off, ids = got
    assert np.array_equal(off.cpu().numpy().view(np.uint64), want[0])
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1])


def check_stored(idx, model, curve):
    keys, ids, xy = idx.sorted_arrays()
    st = np.nonzero(model.stored)[0]
    sk, si = oracle.build(model.xy[st], curve)[:2]
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), sk)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), st[si].astype(np.uint32))
    assert np.array_equal(xy.cpu().numpy(), model.xy[st[si]])


def _mix(n, seed):
    wl = workload.clustered_loguniform(n=n, m=2000, curve=MORTON, seed=seed)
    return wl


@pytest.mark.parametrize("learned", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_insert_erase_sequence_matches_oracle(curve, learned):
    rng = np.random.default_rng(40 + curve)
    wl = _mix(40_000, 41)
    pts0 = wl.points
    idx = sfc.Index(dev(pts0), curve, search=sfc.LEARNED if learned else sfc.BINARY,
                    refine=True)
    model = Model(pts0)
    qs, ds = wl.queries, wl.delta
    more = workload.clustered_points(60_000, 4242, workload.make_mixture(41))
    used = 0
    for step in range(8):
        if step % 3 != 2:
            k = [3000, 7000, 1, 5000, 2500, 6000, 4000, 3000][step]
            new = more[used:used + k]
            used += k
            got_ids = idx.insert(dev(new))
            want_ids = model.insert(new)
            assert np.array_equal(got_ids.cpu().numpy(), want_ids)
        else:
            cand = np.nonzero(model.stored)[0]
            dele = rng.choice(cand, size=min(6000, len(cand)), replace=False)
            # unknown, repeated and already erased ids are skipped
            dele = np.concatenate([dele, dele[:50], [len(model.xy) + 5, 0x7FFFFFFF]])
            got = idx.erase(dev(dele, torch.int32))
            assert got == model.erase(dele)
        info = idx.update_info()
        assert info["epoch"] == model.epoch and info["stored"] == model.stored.sum()
        assert info["compactions"] == model.compactions
        check(idx.query(dev(qs), dev(ds)),
              model.reference(qs, ds, np.full(len(qs), model.epoch), curve))
        if learned:
            assert idx.learned_info()["fallbacks_last"] == 0
    check_stored(idx, model, curve)
    assert model.compactions >= 1


def test_held_epochs_and_retire():
    wl = _mix(30_000, 43)
    pts0 = wl.points
    idx = sfc.Index(dev(pts0), HILBERT, refine=True)
    idx.hold_epochs(True)
    model = Model(pts0, hold=True)
    rng = np.random.default_rng(44)
    more = workload.uniform_points(20_000, 4343)
    for step in range(6):
        if step % 2 == 0:
            new = more[step * 3000:(step + 1) * 3000]
            idx.insert(dev(new))
            model.insert(new)
        else:
            dele = rng.choice(np.nonzero(model.stored & (model.era == LIVE))[0], 5000,
                              replace=False)
            assert idx.erase(dev(dele, torch.int32)) == model.erase(dele)
    info = idx.update_info()
    assert info["oldest"] == 0 and info["compactions"] == 0 and info["dead"] > 0
    qs, ds = wl.queries, wl.delta
    epochs = rng.integers(0, model.epoch + 1, len(qs))
    check(idx.query_epochs(dev(qs), dev(ds), dev(epochs, torch.int32)),
          model.reference(qs, ds, epochs, HILBERT))
    with pytest.raises(sfc.SfcError):
        idx.query_epochs(dev(qs), dev(ds), dev(np.full(len(qs), model.epoch + 1), torch.int32))
    idx.retire(4)
    model.retire(4)
    info = idx.update_info()
    assert info["oldest"] == 4 and info["compactions"] == model.compactions == 1
    epochs = rng.integers(4, model.epoch + 1, len(qs))
    check(idx.query_epochs(dev(qs), dev(ds), dev(epochs, torch.int32)),
          model.reference(qs, ds, epochs, HILBERT))
    with pytest.raises(sfc.SfcError):
        idx.query_epochs(dev(qs), dev(ds), dev(np.full(len(qs), 3), torch.int32))
    idx.hold_epochs(False)
    model.hold = False
    model.oldest = model.epoch
    model._maybe_compact()
    check_stored(idx, model, HILBERT)
    check(idx.query(dev(qs), dev(ds)), model.reference(qs, ds, np.full(len(qs), model.epoch),
                                                      HILBERT))


def test_empty_index_grows_and_shrinks_to_empty():
    idx = sfc.Index(dev(np.zeros((0, 2))), MORTON)
    model = Model(np.zeros((0, 2)))
    pts = workload.uniform_points(5000, 4545)
    qs = workload.uniform_points(500, 4546)
    ds = np.full(500, 0.02)
    ids = idx.insert(dev(pts))
    model.insert(pts)
    check(idx.query(dev(qs), dev(ds)), model.reference(qs, ds, np.full(500, model.epoch), MORTON))
    assert idx.erase(ids) == 5000
    model.erase(np.arange(5000))
    assert idx.size() == 0 and idx.update_info()["live"] == 0
    off, got = idx.query(dev(qs), dev(ds))
    assert got.numel() == 0 and int(off[-1]) == 0
    idx.insert(dev(pts[:10]))
    model.insert(pts[:10])
    check(idx.query(dev(qs), dev(ds)), model.reference(qs, ds, np.full(500, model.epoch), MORTON))


def test_insert_outside_domain_leaves_index_unchanged():
    pts = workload.uniform_points(2000, 4747)
    idx = sfc.Index(dev(pts), MORTON)
    bad = workload.uniform_points(100, 4748)
    bad[17, 0] = 1.0
    with pytest.raises(sfc.DomainError):
        idx.insert(dev(bad))
    info = idx.update_info()
    assert info["epoch"] == 0 and info["stored"] == 2000 and info["next_id"] == 2000
    ids = idx.insert(dev(bad[:17]))
    assert ids.cpu().tolist() == list(range(2000, 2017))


def test_graphs_go_stale_after_an_update():
    wl = _mix(20_000, 49)
    idx = sfc.Index(dev(wl.points), MORTON)
    q, d = dev(wl.queries), dev(wl.delta)
    want = idx.query(q, d)
    g = sfc.Graph.query(idx, q, d, max_rows=idx.last_stats()["rows"] + 64,
                        ids_cap=want[1].numel() + 1)
    g.launch()
    off, ids = g.result()
    assert torch.equal(off, want[0]) and torch.equal(ids, want[1])
    idx.insert(dev(wl.points[:10]))
    with pytest.raises(sfc.SfcError):
        g.launch()
    g.close()
    with pytest.raises(sfc.SfcError):
        sfc.Graph.build(idx, dev(wl.points))

"""sfc_insert_runs: consecutive batches inserted with one sort and one merge
give exactly what one sfc_insert per batch gives: the same stored entries
(keys, ids, points), the same ids returned, and the same answer at every
epoch they create, with erases before and after, the learned index and the
static search tree kept up, and an empty run advancing the epoch."""
import numpy as np
import pytest
import torch

from oracle import HILBERT, MORTON
from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def state(idx):
    k, i, xy = idx.sorted_arrays()
    return k.cpu().numpy(), i.cpu().numpy(), xy.cpu().numpy()


@pytest.mark.parametrize("search", [sfc.BINARY, sfc.LEARNED, sfc.STREE])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_runs_equal_one_insert_per_batch(curve, search):
    rng = np.random.default_rng(3 + curve + 4 * search)
    mix = workload.make_mixture(8, k=6, sigma=0.02)
    base = workload.clustered_points(120_000, 9, mix)
    sizes = [1500, 1, 4000, 777, 2048]
    batches = [workload.clustered_points(s, 10 + t, mix) for t, s in enumerate(sizes)]
    batches[1][0] = batches[0][5]                       # a duplicate across runs
    qs = workload.clustered_points(3000, 20, mix)
    ds = np.full(3000, 0.01)
    a = sfc.Index(dev(base), curve, search=search, refine=True)
    b = sfc.Index(dev(base), curve, search=search, refine=True)
    for x in (a, b):
        x.hold_epochs(True)
        x.erase(dev(np.arange(0, 3000, 7), torch.int32))
    e0 = a.update_info()["epoch"]
    ids_a = [a.insert(dev(p)).cpu().numpy() for p in batches]
    off = np.concatenate([[0], np.cumsum(sizes)])
    ids_b = b.insert_runs(dev(np.concatenate(batches)), off).cpu().numpy()
    assert np.array_equal(np.concatenate(ids_a), ids_b)
    assert a.update_info()["epoch"] == b.update_info()["epoch"] == e0 + len(sizes)
    for x in (a, b):
        x.erase(dev(np.concatenate([ids_b[::13], np.arange(5, 2000, 11)]), torch.int32))
    sa, sb = state(a), state(b)
    for u, v in zip(sa, sb):
        assert np.array_equal(u, v)
    for e in range(e0, e0 + len(sizes) + 2):
        qe = dev(np.full(3000, e), torch.int32)
        oa, ia = a.query_epochs(dev(qs), dev(ds), qe)
        ob, ib = b.query_epochs(dev(qs), dev(ds), qe)
        assert torch.equal(oa, ob) and torch.equal(ia, ib)


def test_empty_run_advances_the_epoch():
    rng = np.random.default_rng(5)
    idx = sfc.Index(dev(rng.random((5000, 2))), MORTON)
    e0 = idx.update_info()["epoch"]
    pts = rng.random((300, 2))
    ids = idx.insert_runs(dev(pts), [0, 100, 100, 300]).cpu().numpy()
    assert idx.update_info()["epoch"] == e0 + 3
    assert np.array_equal(ids, np.arange(5000, 5300))


def test_rejects_bad_offsets():
    idx = sfc.Index(dev(np.random.default_rng(1).random((100, 2))), MORTON)
    with pytest.raises(ValueError):
        idx.insert_runs(dev(np.random.default_rng(2).random((10, 2))), [0, 5, 9])
    with pytest.raises(sfc.SfcError):
        idx.insert_runs(dev(np.random.default_rng(2).random((10, 2))), [0, 6, 5, 10])

"""Device allocations that fail: the index's allocator hook (sfc_options
alloc) returns NULL at one allocation of an operation, for every allocation
that operation makes in turn.  Each such call returns SFC_ERR_NOMEM and
leaves the index as it was (sorted keys, ids and points, the update
counters, and its answers); the same call succeeds once memory is back, and
the answers then equal the oracle over the snapshot of the current epoch.
A construction that fails leaves nothing allocated."""
import numpy as np
import pytest
import torch

from oracle import MORTON
from paper_2508_19891_amd import sfc, workload
from snapshots import Model

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


class FailingAllocator:
    """Device memory from torch's caching allocator; the fail_at-th
    allocation after arm() returns NULL."""

    def __init__(self):
        self.blocks = {}
        self.count = 0
        self.fail_at = None

    def arm(self, k):
        self.count, self.fail_at = 0, k

    def disarm(self):
        self.fail_at = None

    def alloc(self, nbytes):
        self.count += 1
        if self.fail_at is not None and self.count == self.fail_at:
            return 0
        t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=DEV)
        self.blocks[t.data_ptr()] = t
        return t.data_ptr()

    def release(self, ptr):
        self.blocks.pop(ptr, None)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def state(idx):
    keys, ids, xy = idx.sorted_arrays()
    info = idx.update_info()
    return keys.clone(), ids.clone(), xy.clone(), {k: info[k] for k in
                                                   ("epoch", "next_id", "stored", "live", "dead")}


def same_state(a, b):
    return all(torch.equal(x, y) for x, y in zip(a[:3], b[:3])) and a[3] == b[3]


def under_failures(alloc, idx, op, what):
    """Runs op with the k-th allocation failing, k = 1, 2, ..., until it
    succeeds; every failed attempt must leave the index unchanged."""
    for k in range(1, 200):
        before = state(idx)
        alloc.arm(k)
        try:
            out = op()
            alloc.disarm()
            return k, out
        except sfc.SfcError as err:
            alloc.disarm()
            assert err.status == sfc.SFC_ERR_NOMEM, (what, k, err)
        assert same_state(before, state(idx)), (what, k)
    raise AssertionError(f"{what}: still failing after 200 allocations")


def test_build_that_fails_allocates_nothing():
    wl = workload.uniform_fixed_radius(n=20_000, m=10, curve=MORTON)
    alloc = FailingAllocator()
    pts = dev(wl.points)
    for k in range(1, 100):
        alloc.arm(k)
        try:
            idx = sfc.Index(pts, MORTON, search=sfc.LEARNED, refine=True, allocator=alloc)
        except sfc.SfcError as err:
            assert err.status == sfc.SFC_ERR_NOMEM
            assert not alloc.blocks, (k, len(alloc.blocks))
            continue
        alloc.disarm()
        assert k > 1
        idx.close()
        assert not alloc.blocks
        return
    raise AssertionError("construction never succeeded")


@pytest.mark.parametrize("search", [sfc.LEARNED, sfc.STREE, sfc.BINARY])
def test_updates_and_queries_under_failing_allocations(search):
    trace = workload.serving_trace(n0=30_000, requests=8, seed=11, log2_size=(8, 11))
    alloc = FailingAllocator()
    idx = sfc.Index(dev(trace.initial), MORTON, search=search, refine=True, allocator=alloc)
    model = Model(trace.initial)
    rng = np.random.default_rng(5)
    qs = trace.queries[:500]
    ds = trace.delta[:500]
    steps = 0
    for r in range(len(trace.kind)):
        a, k = int(trace.start[r]), int(trace.size[r])
        if trace.kind[r] == workload.INSERT:
            pts = dev(trace.inserts[a:a + k])
            n_try, _ = under_failures(alloc, idx, lambda: idx.insert(pts, want_ids=False),
                                      f"insert {r}")
            model.insert(trace.inserts[a:a + k])
        elif trace.kind[r] == workload.ERASE:
            ids = dev(trace.erase_ids[a:a + k].view(np.int32), torch.int32)
            n_try, cnt = under_failures(alloc, idx, lambda: idx.erase(ids), f"erase {r}")
            assert cnt == model.erase(trace.erase_ids[a:a + k])
        else:
            continue
        steps += 1
        print(f"search={search} request {r}: succeeded at allocation {n_try}", flush=True)
        # a batch under failures, then against the oracle at the current epoch
        sel = rng.choice(len(qs), 200, replace=False)
        q, d = dev(qs[sel]), dev(ds[sel])
        _, (off, got) = under_failures(alloc, idx, lambda: idx.query(q, d), f"query {r}")
        want = model.reference(qs[sel], ds[sel], np.full(200, model.epoch), MORTON)
        assert np.array_equal(off.cpu().numpy().view(np.uint64), want[0])
        assert np.array_equal(got.cpu().numpy().view(np.uint32), want[1])
    assert steps >= 3
    idx.close()
    assert not alloc.blocks

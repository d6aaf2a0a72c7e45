"""The continuous-batching loop: every query request, answered in a batch
with others (in the mix) or in a tick of its own (alone), equals the oracle
over the snapshot of the epoch it was admitted at."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import serving, sfc, workload
from snapshots import Model

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("curve,search", [(MORTON, sfc.LEARNED), (HILBERT, sfc.BINARY)])
def test_batched_and_alone_equal_snapshot_oracle(curve, search):
    trace = workload.serving_trace(n0=20_000, requests=90, seed=7, curve=curve,
                                   log2_size=(6, 11))
    pools = serving.Pools.upload(trace, DEV)
    init = torch.as_tensor(trace.initial).to(DEV)
    runs = []
    for max_tick, slots in ((16, 0), (1, 0), (16, 3)):
        idx = sfc.Index(init, curve, search=search, refine=True)
        runs.append((idx, serving.serve(idx, trace, pools, max_tick=max_tick, record=True,
                                        slots=slots, slot_queries=1 << 14, slot_ids=1 << 20,
                                        slot_rows=1 << 16)))
    mixed, alone, queued = runs[0][1], runs[1][1], runs[2][1]
    assert mixed.ticks < alone.ticks == len(trace.kind)

    model = Model(trace.initial, hold=True)    # never retires: keeps every snapshot
    expect_epoch = {}
    for r in range(len(trace.kind)):
        a, k = int(trace.start[r]), int(trace.size[r])
        if trace.kind[r] == workload.INSERT:
            model.insert(trace.inserts[a:a + k])
        elif trace.kind[r] == workload.ERASE:
            assert model.erase(trace.erase_ids[a:a + k]) == k
        else:
            expect_epoch[r] = model.epoch
    for r, e in expect_epoch.items():
        assert mixed.admitted[r] == e and alone.admitted[r] == e and queued.admitted[r] == e
        a, k = int(trace.start[r]), int(trace.size[r])
        want = model.reference(trace.queries[a:a + k], trace.delta[a:a + k], np.full(k, e), curve)
        for run in (mixed, alone, queued):
            off, ids = run.outputs[r]
            assert np.array_equal(off.view(np.uint64), want[0]), r
            assert np.array_equal(ids.view(np.uint32), want[1]), r

    # After the stream: compaction leaves exactly the live entries, sorted.
    for idx, _ in runs:
        idx.compact()
        live = model.visible(model.epoch)
        keys, ids, _ = idx.sorted_arrays()
        sk, si = oracle.build(model.xy[live], curve)[:2]
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), sk)
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), live[si].astype(np.uint32))
        info = idx.update_info()
        assert info["dead"] == 0 and info["stored"] == len(live)


def test_poisson_arrivals_complete_after_arrival():
    trace = workload.serving_trace(n0=30_000, requests=60, seed=8, log2_size=(6, 10))
    pools = serving.Pools.upload(trace, DEV)
    idx = sfc.Index(torch.as_tensor(trace.initial).to(DEV), MORTON, refine=True)
    run = serving.serve(idx, trace, pools, rate=2000.0)
    lat = run.latency()
    assert (lat > 0).all() and np.all(np.diff(run.arrival) >= 0)
    s = serving.summarize(trace, run)
    assert s["p99_ms"] >= s["p50_ms"] > 0 and s["requests"] == 60


def test_queued_batches_that_outgrow_their_slot_are_answered_again():
    trace = workload.serving_trace(n0=20_000, requests=40, seed=9, log2_size=(6, 10))
    pools = serving.Pools.upload(trace, DEV)
    init = torch.as_tensor(trace.initial).to(DEV)
    ref_idx = sfc.Index(init, MORTON, refine=True)
    ref = serving.serve(ref_idx, trace, pools, record=True)
    idx = sfc.Index(init, MORTON, refine=True)
    run = serving.serve(idx, trace, pools, record=True, slots=2, slot_queries=300,
                        slot_ids=500, slot_rows=128)
    for r, (off, ids) in ref.outputs.items():
        assert np.array_equal(run.outputs[r][0], off) and np.array_equal(run.outputs[r][1], ids)
    assert (run.latency() > 0).all()


class _FailSome:
    """uint8 device buffers; the calls numbered in `fail` raise the device's
    out-of-memory error instead."""

    def __init__(self, fail):
        self.fail, self.calls = set(fail), 0

    def __call__(self, nbytes):
        self.calls += 1
        if self.calls in self.fail:
            raise torch.cuda.OutOfMemoryError("injected")
        return torch.empty(nbytes, dtype=torch.uint8, device=DEV)


@pytest.mark.parametrize("curve,search,keep", [(MORTON, sfc.LEARNED, False),
                                               (HILBERT, sfc.STREE, False),
                                               (MORTON, sfc.BINARY, True),
                                               (HILBERT, sfc.LEARNED, True)])
def test_side_by_side_batches_equal_snapshot_oracle(curve, search, keep):
    """Query batches on three streams at once, admitted by memory, with
    some of their allocations failing (put back and admitted again): every
    request equals the oracle over the snapshot of its epoch.  With kept
    buffers the streams allocate only for their first batches and for
    larger ones, so the failures are placed among the first allocations:
    the out buffer of each of the first three allocating batches (one
    failure apart, so that two never come in a row with nothing in
    flight)."""
    trace = workload.serving_trace(n0=20_000, requests=90, seed=7, curve=curve,
                                   log2_size=(6, 11))
    pools = serving.Pools.upload(trace, DEV)
    init = torch.as_tensor(trace.initial).to(DEV)
    idx = sfc.Index(init, curve, search=search, refine=True)
    per_query = 8 * 48 + 8 + 4 * 1200 + 28 + 300     # scratch estimate + outputs + inputs
    budget = 3 * 600 * per_query + (4 << 20)
    alloc = _FailSome({2, 6, 10} if keep else {4, 11, 23, 40})
    run = serving.serve(idx, trace, pools, record=True, streams=3, budget_bytes=budget,
                        slot_queries=600, alloc=alloc, keep_buffers=keep)
    assert run.max_batches >= 2          # batches were on the device together
    assert run.requeued >= 3             # and the failed allocations were admitted again
    assert run.max_in_flight <= budget
    model = Model(trace.initial, hold=True)
    expect_epoch = {}
    for r in range(len(trace.kind)):
        a, k = int(trace.start[r]), int(trace.size[r])
        if trace.kind[r] == workload.INSERT:
            model.insert(trace.inserts[a:a + k])
        elif trace.kind[r] == workload.ERASE:
            model.erase(trace.erase_ids[a:a + k])
        else:
            expect_epoch[r] = model.epoch
    for r, e in expect_epoch.items():
        assert run.admitted[r] == e
        a, k = int(trace.start[r]), int(trace.size[r])
        want = model.reference(trace.queries[a:a + k], trace.delta[a:a + k], np.full(k, e), curve)
        off, ids = run.outputs[r]
        assert np.array_equal(off.view(np.uint64), want[0]), r
        assert np.array_equal(ids.view(np.uint32), want[1]), r
    idx.close()


def test_side_by_side_budget_limits_batches_in_flight():
    """A budget below the memory of any batch: each batch is admitted alone
    (never two in flight), with the same answers as the synchronous loop."""
    trace = workload.serving_trace(n0=20_000, requests=40, seed=9, log2_size=(6, 10))
    pools = serving.Pools.upload(trace, DEV)
    init = torch.as_tensor(trace.initial).to(DEV)
    ref_idx = sfc.Index(init, MORTON, refine=True)
    ref = serving.serve(ref_idx, trace, pools, record=True)
    idx = sfc.Index(init, MORTON, refine=True)
    m = 64                                   # the smallest request of the trace
    one = idx.query_scratch_bytes(m, 48 * m + 1024) + 8 * (m + 1) + 4 * 1200 * m - 1
    run = serving.serve(idx, trace, pools, record=True, streams=4, budget_bytes=one,
                        slot_queries=300)
    assert run.max_batches == 1
    for r, (off, ids) in ref.outputs.items():
        assert np.array_equal(run.outputs[r][0], off) and np.array_equal(run.outputs[r][1], ids)

"""Continuous batching of query, insert and erase requests over one index.

Requests arrive in stream order at their arrival times.  Each tick takes
the requests that have arrived (at most ``max_tick`` of them), applies the
inserts and erases in stream order (consecutive inserts together, as one
sort and one merge that gives each its own epoch), and answers the queries of
all of them in one batch, each query at the epoch it was admitted at (the
epoch after the updates that arrived before it), so that batching never
changes an answer.  Epochs older than every query still running are
retired, which lets the index drop the tombstones no query can see any
more.  All GPU work runs in the library; this loop only slices the request
pools and keeps the clock.

Three modes:
  * ``slots = 0, streams = 0``: each tick's query batch is answered before
    the next tick starts (sfc_query_epochs).
  * ``slots = k > 0``: query batches are queued without waiting
    (sfc_query_async) into k preallocated output slots on the index's own
    stream; while they run, the loop admits the next arrivals and queues
    their work behind them, and a batch's requests complete when its slot's
    event has passed.  A tick with queries waits only for a free slot.
  * ``streams = k > 0``: query batches run side by side on k streams
    (sfc_query_async_on), each with its own scratch and outputs: a stream
    keeps them for its next batch and allocates larger ones only when a
    batch needs more.  Admission is by memory: a batch is admitted while the
    memory the loop holds (the streams' buffers and the batches' inputs)
    plus what the batch adds stays within ``budget_bytes`` and a stream is
    free; idle streams first give their buffers back, then the loop waits
    for the oldest batch.  An allocation that fails (the device, or the
    library reporting SFC_ERR_NOMEM) puts the batch back at the head of the
    queue until a batch in flight has finished.  A batch's queries and radii
    are views of the request pools (consecutive query requests take
    consecutive slices).  Updates run on the index's stream; the library
    makes them wait, on the device, for the batches still reading the
    index.
A batch that outgrew its output (rows or ids) is answered again
synchronously into larger buffers.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import sfc
from .workload import ERASE, INSERT, QUERY, ServingTrace


@dataclasses.dataclass
class Pools:
    """The trace's payloads in device memory."""
    queries: torch.Tensor
    delta: torch.Tensor
    inserts: torch.Tensor
    erase_ids: torch.Tensor

    @classmethod
    def upload(cls, trace: ServingTrace, device="cuda:0") -> "Pools":
        def f64(a):
            return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(device)
        return cls(f64(trace.queries).reshape(-1, 2), f64(trace.delta),
                   f64(trace.inserts).reshape(-1, 2),
                   torch.as_tensor(trace.erase_ids.view(np.int32)).to(device))


@dataclasses.dataclass
class Slot:
    """Preallocated outputs of one queued query batch."""
    offsets: torch.Tensor
    ids: torch.Tensor
    flags: torch.Tensor
    event: torch.cuda.Event
    max_rows: int
    busy: bool = False
    members: list = dataclasses.field(default_factory=list)   # (request, epoch, size)
    batch: tuple = ()                                           # (q, delta, epochs)


def make_slots(k: int, device, max_queries: int, max_ids: int, max_rows: int) -> list:
    return [Slot(torch.empty(max_queries + 1, dtype=torch.int64, device=device),
                 torch.empty(max_ids, dtype=torch.int32, device=device),
                 torch.zeros(1, dtype=torch.int32, device=device),
                 torch.cuda.Event(enable_timing=True), max_rows) for _ in range(k)]


@dataclasses.dataclass
class Run:
    arrival: np.ndarray       # seconds from the start
    done: np.ndarray          # completion, seconds from the start
    admitted: np.ndarray      # epoch each query request was answered at (-1 otherwise)
    ticks: int
    seconds: float
    outputs: dict             # request -> (offsets, ids) on the host, if recorded
    max_in_flight: int = 0    # side-by-side mode: most batch memory held at once (bytes)
    max_batches: int = 0      # side-by-side mode: most batches in flight at once
    requeued: int = 0         # side-by-side mode: batches put back for want of memory

    def latency(self) -> np.ndarray:
        return self.done - self.arrival


def _batch_inputs(trace, pools, members, dev):
    """Queries, radii and query epochs of a batch's requests (r, epoch, k) in
    order: consecutive query requests take consecutive slices of the pools,
    so the batch is one view of each; one fill when they share an epoch."""
    starts = [int(trace.start[r]) for r, _, _ in members]
    sizes = [k for _, _, k in members]
    m = sum(sizes)
    if all(starts[t + 1] == starts[t] + sizes[t] for t in range(len(members) - 1)):
        q = pools.queries[starts[0]:starts[0] + m]
        d = pools.delta[starts[0]:starts[0] + m]
    else:
        q = torch.cat([pools.queries[a:a + k] for a, k in zip(starts, sizes)])
        d = torch.cat([pools.delta[a:a + k] for a, k in zip(starts, sizes)])
    eps = [e for _, e, _ in members]
    if all(x == eps[0] for x in eps):
        e = torch.full((m,), eps[0], dtype=torch.int32, device=dev)
    else:
        e = torch.cat([torch.full((k,), x, dtype=torch.int32, device=dev)
                       for x, k in zip(eps, sizes)])
    return q, d, e


class _Inserts:
    """Insert requests of a tick not yet applied: consecutive ones (their
    points are consecutive slices of the insert pool) go to the index as one
    sfc_insert_runs call, one sort and one merge, with the epochs and ids
    they would get one by one.  Applied before an erase and before the
    tick's queries are answered."""

    def __init__(self, index, pools):
        self.index, self.pools, self.reqs = index, pools, []

    def add(self, r: int, a: int, k: int):
        if self.reqs and self.reqs[-1][1] + self.reqs[-1][2] != a:
            raise ValueError("insert requests must take consecutive pool slices")
        self.reqs.append((r, a, k))

    def flush(self) -> list:
        if not self.reqs:
            return []
        a0 = self.reqs[0][1]
        off = [0]
        for _, _, k in self.reqs:
            off.append(off[-1] + k)
        self.index.insert_runs(self.pools.inserts[a0:a0 + off[-1]], off, want_ids=False)
        done = [r for r, _, _ in self.reqs]
        self.reqs = []
        return done


def serve(index: sfc.Index, trace: ServingTrace, pools: Pools, rate: float = float("inf"),
          max_tick: int = 16, record: bool = False, out_ids: torch.Tensor | None = None,
          slots: int = 0, slot_queries: int = 1 << 20, slot_ids: int = 1 << 26,
          slot_rows: int = 1 << 24, streams: int = 0, budget_bytes: int = 2 << 30,
          rows_per_query: int = 48, ids_per_query: int = 1200, alloc=None,
          keep_buffers: bool = True) -> Run:
    """Runs the trace with Poisson arrivals at ``rate`` requests/s (inf: all
    at time 0) and returns arrival and completion times per request.

    streams > 0: batches of at most slot_queries queries run side by side,
    each sized for rows_per_query candidate rows and ids_per_query ids per
    query, admitted against budget_bytes; alloc(nbytes) -> uint8 device
    tensor (default torch.empty) provides their memory.  With keep_buffers
    each stream keeps its scratch and output buffers for its next batch
    (allocating only when a batch needs more) and the kept bytes count
    against the budget; idle streams give theirs back when a batch needs
    the room.  Without it every batch allocates and frees its own."""
    if streams > 0:
        return _serve_overlap(index, trace, pools, rate, max_tick, record, streams, budget_bytes,
                              slot_queries, rows_per_query, ids_per_query, alloc, keep_buffers)
    if slots > 0:
        return _serve_async(index, trace, pools, rate, max_tick, record, slots, slot_queries,
                            slot_ids, slot_rows)
    R = len(trace.kind)
    arrival = np.zeros(R) if not np.isfinite(rate) else np.cumsum(trace.gaps) / rate
    done = np.zeros(R)
    admitted = np.full(R, -1, np.int64)
    outputs = {}
    index.hold_epochs(True)
    epoch = index.update_info()["epoch"]
    dev = pools.queries.device
    if out_ids is None:
        out_ids = torch.empty(1 << 24, dtype=torch.int32, device=dev)
    ticks = 0
    i = 0
    t0 = time.perf_counter()
    while i < R:
        now = time.perf_counter() - t0
        if arrival[i] > now:
            wait = arrival[i] - now
            if wait > 2e-3:
                time.sleep(wait - 1e-3)
            while time.perf_counter() - t0 < arrival[i]:
                pass
            now = time.perf_counter() - t0
        j = int(np.searchsorted(arrival, now, side="right"))
        j = min(max(j, i + 1), i + max_tick)
        pending = []
        inserts = _Inserts(index, pools)
        for r in range(i, j):
            a, k = int(trace.start[r]), int(trace.size[r])
            if trace.kind[r] == QUERY:
                pending.append((r, epoch))
            elif trace.kind[r] == INSERT:
                inserts.add(r, a, k)
                epoch += 1
            else:
                for ri in inserts.flush():
                    done[ri] = time.perf_counter() - t0
                index.erase(pools.erase_ids[a:a + k])
                epoch += 1
                done[r] = time.perf_counter() - t0
        for ri in inserts.flush():
            done[ri] = time.perf_counter() - t0
        if pending:
            q, d, e = _batch_inputs(trace, pools,
                                    [(r, e, int(trace.size[r])) for r, e in pending], dev)
            try:
                off, ids = index.query_epochs(q, d, e, out_ids=out_ids)
            except sfc.CapacityError as err:
                out_ids = torch.empty(2 * err.total, dtype=torch.int32, device=dev)
                off, ids = index.query_epochs(q, d, e, out_ids=out_ids)
            t = time.perf_counter() - t0
            base = 0
            if record:
                off_h = off.cpu().numpy()
                ids_h = ids.cpu().numpy()
            for r, e_r in pending:
                done[r] = t
                admitted[r] = e_r
                k = int(trace.size[r])
                if record:
                    o = off_h[base:base + k + 1]
                    outputs[r] = (o - o[0], ids_h[o[0]:o[-1]].copy())
                base += k
        index.retire(epoch)
        ticks += 1
        i = j
    seconds = time.perf_counter() - t0
    return Run(arrival, done, admitted, ticks, seconds, outputs)


def _serve_async(index, trace, pools, rate, max_tick, record, nslots, slot_queries, slot_ids,
                 slot_rows) -> Run:
    R = len(trace.kind)
    arrival = np.zeros(R) if not np.isfinite(rate) else np.cumsum(trace.gaps) / rate
    done = np.zeros(R)
    admitted = np.full(R, -1, np.int64)
    outputs = {}
    index.hold_epochs(True)
    epoch = index.update_info()["epoch"]
    dev = pools.queries.device
    pool = make_slots(nslots, dev, slot_queries, slot_ids, slot_rows)
    busy = []                      # slots in launch order
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()

    def finish(slot: Slot):
        """The slot's batch has run: check it, record its requests."""
        slot.event.synchronize()
        t_done = start.elapsed_time(slot.event) * 1e-3
        m = sum(k for _, _, k in slot.members)
        flags = int(slot.flags.item())
        total = int(slot.offsets[m].item()) if flags == 0 else -1
        if flags != 0 or total > slot.ids.numel():
            if flags & ~16:
                raise sfc.SfcError(sfc.SFC_ERR_INVALID, f"query batch flags {flags}")
            q, d, e = slot.batch          # outgrew the slot: answer it again, synchronously
            off, ids = index.query_epochs(q, d, e)
            t_done = time.perf_counter() - t0
        else:
            off, ids = slot.offsets[:m + 1], slot.ids[:total]
        base = 0
        if record:
            off_h = off.cpu().numpy()
            ids_h = ids.cpu().numpy()
        for r, e_r, k in slot.members:
            done[r] = t_done
            admitted[r] = e_r
            if record:
                o = off_h[base:base + k + 1]
                outputs[r] = (o - o[0], ids_h[o[0]:o[-1]].copy())
            base += k
        slot.busy = False
        slot.members = []
        slot.batch = ()

    def reap(block: bool):
        """Completes finished slots in launch order (the oldest first)."""
        while busy and (block or busy[0].event.query()):
            finish(busy.pop(0))
            block = False

    ticks = 0
    i = 0
    while i < R:
        reap(False)
        now = time.perf_counter() - t0
        if arrival[i] > now and busy:
            reap(True)                 # nothing arrived yet: wait for the oldest batch
            continue
        if arrival[i] > now:
            wait = arrival[i] - now
            if wait > 2e-3:
                time.sleep(wait - 1e-3)
            while time.perf_counter() - t0 < arrival[i]:
                pass
            now = time.perf_counter() - t0
        j = int(np.searchsorted(arrival, now, side="right"))
        j = min(max(j, i + 1), i + max_tick)
        pending = []
        inserts = _Inserts(index, pools)
        for r in range(i, j):
            a, k = int(trace.start[r]), int(trace.size[r])
            if trace.kind[r] == QUERY:
                pending.append((r, epoch, k))
            elif trace.kind[r] == INSERT:
                inserts.add(r, a, k)
                epoch += 1
            else:
                for ri in inserts.flush():
                    done[ri] = time.perf_counter() - t0
                index.erase(pools.erase_ids[a:a + k])
                epoch += 1
                done[r] = time.perf_counter() - t0
        for ri in inserts.flush():
            done[ri] = time.perf_counter() - t0
        # an update waits for all queued work, so slots may have finished
        reap(False)
        while pending:
            if len(busy) == nslots:
                reap(True)             # admission: wait until a slot frees up
            slot = next(sl for sl in pool if not sl.busy)
            take, m = [], 0
            while pending and m + pending[0][2] <= slot_queries:
                take.append(pending.pop(0))
                m += take[-1][2]
            if not take:               # a single request larger than a slot
                take.append(pending.pop(0))
                m = take[0][2]
            q, d, e = _batch_inputs(trace, pools, take, dev)
            slot.members = take
            slot.batch = (q, d, e)
            slot.busy = True
            if m <= slot_queries:
                index.query_async(q, d, e, slot.max_rows, slot.offsets, slot.ids, slot.flags)
            else:
                slot.flags.fill_(16)   # answered synchronously when reaped
            slot.event.record()
            busy.append(slot)
        # retire what no queued or running query can see
        oldest = min([e for sl in busy for _, e, _ in sl.members], default=epoch)
        index.retire(oldest)
        ticks += 1
        i = j
    while busy:
        reap(True)
    index.retire(epoch)
    seconds = time.perf_counter() - t0
    return Run(arrival, done, admitted, ticks, seconds, outputs)


class _Batch:
    """One admitted query batch of the side-by-side mode: its requests, its
    stream, and the memory it holds until it completes."""

    def __init__(self, members, q, d, e, stream, nbytes):
        self.members, self.q, self.d, self.e = members, q, d, e
        self.stream, self.nbytes = stream, nbytes
        self.event = torch.cuda.Event(enable_timing=True)
        self.scratch = self.offsets = self.ids = self.flags = None
        self.max_rows = 0


def _serve_overlap(index, trace, pools, rate, max_tick, record, nstreams, budget, max_batch,
                   rows_per_query, ids_per_query, alloc, keep_buffers) -> Run:
    R = len(trace.kind)
    arrival = np.zeros(R) if not np.isfinite(rate) else np.cumsum(trace.gaps) / rate
    done = np.zeros(R)
    admitted = np.full(R, -1, np.int64)
    outputs = {}
    index.hold_epochs(True)
    epoch = index.update_info()["epoch"]
    dev = pools.queries.device
    if alloc is None:
        def alloc(nbytes):
            return torch.empty(nbytes, dtype=torch.uint8, device=dev)
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    free = list(streams)
    busy = []                      # batches in launch order
    # Each stream's scratch and output buffers, kept between its batches
    # (keep_buffers) and replaced by larger ones when a batch needs more.
    # held: bytes of those buffers plus the query epochs of the batches in
    # flight; admission keeps it within the budget.
    kept = {}
    held = [0]
    stats = {"max_in_flight": 0, "max_batches": 0, "requeued": 0}
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()

    def kept_bytes(st) -> int:
        k = kept.get(st)
        return 0 if k is None else k[0].numel() + k[1].numel()

    def drop(st):
        held[0] -= kept_bytes(st)
        kept.pop(st, None)

    def finish(b: _Batch):
        b.event.synchronize()
        t_done = start.elapsed_time(b.event) * 1e-3
        m = sum(k for _, _, k in b.members)
        flags = int(b.flags[0].item())
        total = int(b.offsets[m].item()) if flags == 0 else -1
        if flags != 0 or total > b.ids.numel():
            if flags & ~16:
                raise sfc.SfcError(sfc.SFC_ERR_INVALID, f"query batch flags {flags}")
            off, ids = index.query_epochs(b.q, b.d, b.e)   # outgrew its outputs
            t_done = time.perf_counter() - t0
        else:
            off, ids = b.offsets[:m + 1], b.ids[:total]
        base = 0
        if record:
            off_h = off.cpu().numpy()
            ids_h = ids.cpu().numpy()
        for r, e_r, k in b.members:
            done[r] = t_done
            admitted[r] = e_r
            if record:
                o = off_h[base:base + k + 1]
                outputs[r] = (o - o[0], ids_h[o[0]:o[-1]].copy())
            base += k
        held[0] -= b.nbytes
        b.offsets = b.ids = b.flags = b.scratch = None
        if not keep_buffers:
            drop(b.stream)
        free.append(b.stream)

    def reap(block: bool):
        while busy and (block or busy[0].event.query()):
            finish(busy.pop(0))
            block = False

    def launch(take) -> bool:
        """Admits one batch: False when its memory could not be had (the
        caller waits for a batch in flight and tries again)."""
        m = sum(k for _, _, k in take)
        max_rows = rows_per_query * m + 1024
        ids_cap = ids_per_query * m
        scratch_bytes = index.query_scratch_bytes(m, max_rows)
        out_bytes = 256 + 8 * (m + 1) + 4 * ids_cap
        in_bytes = 4 * m               # the query epochs (queries and radii are pool views)

        def fits_kept(st) -> bool:
            k = kept.get(st)
            return k is not None and k[0].numel() >= scratch_bytes and k[1].numel() >= out_bytes

        def adds(st) -> int:           # bytes held more once the batch runs on st
            if fits_kept(st):
                return in_bytes
            return scratch_bytes + out_bytes + in_bytes - kept_bytes(st)

        while True:                    # admission by memory and streams
            if free:
                if held[0] + adds(free[0]) <= budget:
                    break
                for st in free[1:]:    # idle streams give their buffers back first
                    drop(st)
                if held[0] + adds(free[0]) <= budget:
                    break
            if not busy:               # alone: admitted whatever it needs
                break
            reap(True)
        st = free[0]
        try:
            q, d, e = _batch_inputs(trace, pools, take, dev)
            if not fits_kept(st):
                drop(st)
                scratch = alloc(scratch_bytes)
                if scratch is None or scratch.numel() < scratch_bytes:
                    return False       # the caller's allocator had no memory
                out = alloc(out_bytes)
                if out is None or out.numel() < out_bytes:
                    return False
                kept[st] = (scratch, out)
                held[0] += scratch.numel() + out.numel()
            scratch, out = kept[st]
            b = _Batch(take, q, d, e, st, in_bytes)
            b.max_rows = max_rows
            b.scratch = scratch
            b.flags = out[:256].view(torch.int32)
            b.offsets = out[256:256 + 8 * (m + 1)].view(torch.int64)
            b.ids = out[256 + 8 * (m + 1):256 + 8 * (m + 1) + 4 * ids_cap].view(torch.int32)
            b.flags.zero_()
        except torch.cuda.OutOfMemoryError:
            return False
        b.stream.wait_stream(torch.cuda.current_stream())
        try:
            index.query_async_on(b.stream, b.scratch, q, d, e, max_rows, b.offsets, b.ids,
                                 b.flags)
        except sfc.SfcError as err:
            if err.status != sfc.SFC_ERR_NOMEM:
                raise
            return False
        b.event.record(b.stream)
        free.pop(0)
        busy.append(b)
        held[0] += in_bytes
        stats["max_in_flight"] = max(stats["max_in_flight"], held[0])
        stats["max_batches"] = max(stats["max_batches"], len(busy))
        return True

    ticks = 0
    i = 0
    alone_failures = 0
    while i < R:
        reap(False)
        now = time.perf_counter() - t0
        if arrival[i] > now and busy:
            reap(True)                 # nothing arrived yet: wait for the oldest batch
            continue
        if arrival[i] > now:
            wait = arrival[i] - now
            if wait > 2e-3:
                time.sleep(wait - 1e-3)
            while time.perf_counter() - t0 < arrival[i]:
                pass
            now = time.perf_counter() - t0
        j = int(np.searchsorted(arrival, now, side="right"))
        j = min(max(j, i + 1), i + max_tick)
        pending = []
        inserts = _Inserts(index, pools)
        for r in range(i, j):
            a, k = int(trace.start[r]), int(trace.size[r])
            if trace.kind[r] == QUERY:
                pending.append((r, epoch, k))
            elif trace.kind[r] == INSERT:
                inserts.add(r, a, k)
                epoch += 1
            else:
                for ri in inserts.flush():
                    done[ri] = time.perf_counter() - t0
                index.erase(pools.erase_ids[a:a + k])
                epoch += 1
                done[r] = time.perf_counter() - t0
        for ri in inserts.flush():
            done[ri] = time.perf_counter() - t0
        reap(False)
        while pending:
            take, m = [], 0
            while pending and (not take or m + pending[0][2] <= max_batch):
                take.append(pending.pop(0))
                m += take[-1][2]
            if launch(take):
                alone_failures = 0
                continue
            # requeue: after a batch in flight frees its memory, or, with none
            # in flight, once more after the device is idle
            pending[:0] = take
            stats["requeued"] += 1
            if busy:
                reap(True)
            else:
                alone_failures += 1
                if alone_failures > 1:
                    raise sfc.SfcError(sfc.SFC_ERR_NOMEM, "a query batch found no memory "
                                       "with nothing in flight")
                for st in list(kept):  # nothing runs: every stream's buffers go back
                    drop(st)
                torch.cuda.synchronize()
        oldest = min([e for b in busy for _, e, _ in b.members], default=epoch)
        index.retire(oldest)
        ticks += 1
        i = j
    while busy:
        reap(True)
    index.retire(epoch)
    seconds = time.perf_counter() - t0
    return Run(arrival, done, admitted, ticks, seconds, outputs, **stats)


def summarize(trace: ServingTrace, run: Run) -> dict:
    lat = run.latency() * 1e3
    out = {"requests": len(lat), "ticks": run.ticks, "seconds": run.seconds,
           "requests_per_s": len(lat) / run.seconds,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}
    for name, kd in (("query", QUERY), ("insert", INSERT), ("erase", ERASE)):
        sel = trace.kind == kd
        if sel.any():
            out[f"{name}_p50_ms"] = float(np.percentile(lat[sel], 50))
            out[f"{name}_p99_ms"] = float(np.percentile(lat[sel], 99))
    out["queries_per_s"] = float(trace.size[trace.kind == QUERY].sum() / run.seconds)
    out["inserts_per_s"] = float(trace.size[trace.kind == INSERT].sum() / run.seconds)
    out["erases_per_s"] = float(trace.size[trace.kind == ERASE].sum() / run.seconds)
    return out

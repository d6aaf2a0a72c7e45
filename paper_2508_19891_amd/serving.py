"""Continuous batching of query, insert and erase requests over one index.

Requests arrive in stream order at their arrival times.  Each tick takes
the requests that have arrived (at most ``max_tick`` of them), applies the
inserts and erases one by one in stream order, and answers the queries of
all of them in one batch, each query at the epoch it was admitted at (the
epoch after the updates that arrived before it), so that batching never
changes an answer.  After the batch every older epoch is retired, which
lets the index drop the tombstones no query can see any more.  All GPU work
runs in the library; this loop only slices the request pools and keeps the
clock.
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
class Run:
    arrival: np.ndarray       # seconds from the start
    done: np.ndarray          # completion, seconds from the start
    admitted: np.ndarray      # epoch each query request was answered at (-1 otherwise)
    ticks: int
    seconds: float
    outputs: dict             # request -> (offsets, ids) on the host, if recorded

    def latency(self) -> np.ndarray:
        return self.done - self.arrival


def serve(index: sfc.Index, trace: ServingTrace, pools: Pools, rate: float = float("inf"),
          max_tick: int = 16, record: bool = False, out_ids: torch.Tensor | None = None) -> Run:
    """Runs the trace with Poisson arrivals at ``rate`` requests/s (inf: all
    at time 0) and returns arrival and completion times per request."""
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
        for r in range(i, j):
            a, k = int(trace.start[r]), int(trace.size[r])
            if trace.kind[r] == QUERY:
                pending.append((r, epoch))
            elif trace.kind[r] == INSERT:
                index.insert(pools.inserts[a:a + k], want_ids=False)
                epoch += 1
                done[r] = time.perf_counter() - t0
            else:
                index.erase(pools.erase_ids[a:a + k])
                epoch += 1
                done[r] = time.perf_counter() - t0
        if pending:
            qs, ds, es = [], [], []
            for r, e in pending:
                a, k = int(trace.start[r]), int(trace.size[r])
                qs.append(pools.queries[a:a + k])
                ds.append(pools.delta[a:a + k])
                es.append(torch.full((k,), e, dtype=torch.int32, device=dev))
            q = qs[0] if len(qs) == 1 else torch.cat(qs)
            d = ds[0] if len(ds) == 1 else torch.cat(ds)
            e = es[0] if len(es) == 1 else torch.cat(es)
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

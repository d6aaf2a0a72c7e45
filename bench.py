"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input that
is already resident in device memory: construction of the index over n points
(curve keys, radix sort of (key, id), gather of the points) followed by one
batch of m distance queries (ranges, searches, exact test, compaction into
CSR).  Prints one JSON line on stdout; progress goes to stderr.

Workload: n = 2^24 points, 80% from 16 isotropic Gaussians (sigma 0.01,
uniform centres) and 20% uniform, clamped to [0,1)^2; Hilbert keys; 2^20
queries drawn from the same mixture, each with a radius aimed at an expected
output log-uniform in [1, 1000] points.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(name: str) -> str:
    path = os.path.join(ROOT, "paper_2508_19891_amd", "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


# Kernels whose algorithmic bytes the bench states (candidates for the
# roofline's dominant kernel).
ROOFLINE_KERNELS = ("keygen_tiles", "tile_hist", "scatter_pass", "chunk_sort", "ranges_search",
                    "compact_test", "query_filters", "compact_write")


def timed_calls(fn, steps: int):
    """(ms per call of fn, timed without events, {kernel: (launches, ms)} of
    the same number of calls repeated with HIP events around every launch,
    which add gaps between kernels)."""
    import torch

    from paper_2508_19891_amd import sfc

    torch.cuda.synchronize()
    sfc.profile_reset()
    sfc.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    sfc.profile_enable(False)
    kern = sfc.profile_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, kern


def load_traffic(kernel: str, source: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (its 'traffic: kernel bytes source hash' lines), or None if the
    kernel's source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_clustered_n2p24_m2p20_refined.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) == 5 and parts[0] == "traffic:" and parts[1] == kernel:
            if parts[3] == source and parts[4] == kernel_source_hash(source):
                return float(parts[2])
    return None


def cpu_baseline(wl, curve: int, m_sample: int):
    """The oracle timed on the host: full construction (single thread) and
    the first m_sample queries (by default the whole batch; contiguous slices
    over the host threads), the query time scaled to the full batch when the
    sample is smaller; the single-thread rate on an eighth of the sample."""
    import oracle
    # every core this process may run on: the machine's CPU share as its harness
    # states it (OMP_NUM_THREADS), else the affinity mask
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    idx = oracle.build(wl.points, curve)
    t_build = time.perf_counter() - t0
    qs = wl.queries[:m_sample]
    ds = wl.delta[:m_sample]
    t0 = time.perf_counter()
    off, _ = oracle.query(idx, qs, ds, curve, nthreads=threads)
    t_query = time.perf_counter() - t0
    m1 = max(1, m_sample // 8)   # one thread: an eighth of the sample
    t0 = time.perf_counter()
    oracle.query(idx, qs[:m1], ds[:m1], curve, nthreads=1)
    t_query1 = time.perf_counter() - t0
    m = wl.queries.shape[0]
    t_step = t_build + t_query * (m / m_sample)
    return {
        "value": m / t_step,
        "unit": "queries/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle build of all {wl.points.shape[0]} points on 1 thread "
                   f"({t_build:.2f} s) + " +
                   (f"all {m} queries" if m_sample == m else f"the first {m_sample} of {m} queries")
                   + f" on {threads} threads ({t_query:.2f} s"
                   + (")" if m_sample == m else f", scaled x{m / m_sample:g})")),
        "reported_sample": int(off[-1]),
        "queries_per_s_1_thread": m1 / t_query1,
        "queries_per_s_all_threads": m_sample / t_query,
    }


def batched_sets_bench(args, sfc, workload, torch):
    """256 independent point sets (sizes 2^U[10,20], uniform or clustered by
    coin) with 2^U[8,16] queries each: all sets built in one pass sequence and
    all queries in one batch, recorded as two graphs, against the same work
    done set by set with separate calls."""
    dev = torch.device("cuda:0")
    wl = workload.batched_uneven(n_sets=256, curve=sfc.MORTON)
    pts = torch.as_tensor(wl.points).to(dev)
    q = torch.as_tensor(wl.queries).to(dev)
    d = torch.as_tensor(wl.delta).to(dev)
    qs = torch.as_tensor(wl.qset.astype("int32")).to(dev)
    n, m = pts.shape[0], q.shape[0]
    log(f"batched sets: {n} points, {m} queries")
    tune_b, tune_b_ms = sfc.autotune_build(pts, sfc.MORTON, wl.set_off)
    idx = sfc.Index(pts, sfc.MORTON, refine=True, set_off=wl.set_off)
    off, ids = idx.query_sets(q, d, qs)
    st = idx.last_stats()
    rep, rows = int(ids.numel()), st["rows"]
    tune_q, tune_q_ms = sfc.autotune_query(idx, q, d, qs, ids_cap=rep + 1)
    gb = sfc.Graph.build(idx, pts)
    gq = sfc.Graph.query(idx, q, d, max_rows=rows + 64, ids_cap=rep + 1, qset=qs)

    def timed(fn, steps):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    def graph_step():
        gb.launch()
        gq.launch()
        assert gq.wait() == rep

    def eager_step():
        ix = sfc.Index(pts, sfc.MORTON, refine=True, set_off=wl.set_off)
        ix.query_sets(q, d, qs)
        ix.close()

    so, qoff = wl.set_off, np.searchsorted(wl.qset, np.arange(257))

    def separate_step():
        for s in range(256):
            a, b = int(so[s]), int(so[s + 1])
            ix = sfc.Index(pts[a:b], sfc.MORTON, refine=True)
            if qoff[s + 1] > qoff[s]:
                ix.query(q[qoff[s]:qoff[s + 1]], d[qoff[s]:qoff[s + 1]])
            ix.close()

    ms_graph = timed(graph_step, args.steps)
    ms_eager = timed(eager_step, args.steps)
    ms_sep = timed(separate_step, max(1, args.steps // 5))
    gb.close()
    gq.close()
    idx.close()
    return {"workload": wl.name, "sets": 256, "points": n, "queries": m, "reported": rep,
            "ms_per_step_graph": ms_graph, "ms_per_step_batched_eager": ms_eager,
            "ms_per_step_separate_calls": ms_sep,
            "queries_per_s_graph": m / (ms_graph * 1e-3),
            "speedup_vs_separate": ms_sep / ms_graph,
            "autotune": {"sort_items": tune_b, "sort_items_ms": tune_b_ms,
                         "test_shape": tune_q, "test_shape_ms": tune_q_ms}}


def learned_large_bench(args, sfc, workload, torch):
    """The learned-index shape: 2^26 clustered points, Morton keys, 2^22
    uniform queries with delta = sqrt(10 / (pi n)) (about 10 reports each at
    unit density); query batches over one built index, binary vs learned
    search (and the static search tree), the learned fit timed once.  A
    secondary batch draws the queries from the points' mixture (same delta,
    a few hundred reports each)."""
    dev = torch.device("cuda:0")
    wl = workload.clustered_uniform_queries(n=1 << 26, m=1 << 22, curve=sfc.MORTON)
    n, m = wl.points.shape[0], wl.queries.shape[0]
    log(f"learned at scale: n={n} m={m}")
    pts = torch.as_tensor(wl.points).to(dev)
    q = torch.as_tensor(wl.queries).to(dev)
    d = torch.as_tensor(wl.delta).to(dev)
    qm = torch.as_tensor(workload.clustered_points(m, 4003, workload.make_mixture(503))).to(dev)
    offsets = torch.empty(m + 1, dtype=torch.int64, device=dev)
    out = {"workload": wl.name + "_morton", "n": n, "m": m}
    reps, reps_m = [], []
    for name, search in (("bsearch", sfc.BINARY), ("learned", sfc.LEARNED),
                         ("stree", sfc.STREE)):
        torch.cuda.synchronize()
        sfc.profile_reset()
        sfc.profile_enable(True)
        idx = sfc.Index(pts, sfc.MORTON, search=search)
        torch.cuda.synchronize()
        sfc.profile_enable(False)
        build = {k: v[1] for k, v in sfc.profile_read().items()}
        _, ids0 = idx.query(q, d)
        out_ids = torch.empty(ids0.numel() + 1024, dtype=torch.int32, device=dev)
        reps.append(int(ids0.numel()))
        del ids0
        for _ in range(max(1, args.warmup)):
            idx.query(q, d, out_ids=out_ids, out_offsets=offsets)
        ms, kern = timed_calls(lambda: idx.query(q, d, out_ids=out_ids, out_offsets=offsets),
                               args.steps)
        kern = {k: v[1] / args.steps for k, v in kern.items()}
        out[name] = {"ms_per_batch": ms, "queries_per_s": m / (ms * 1e-3),
                     "search_ms": kern.get({sfc.BINARY: "ranges_search", sfc.LEARNED:
                                            "ranges_learned", sfc.STREE: "ranges_stree"}[search]),
                     "kernels_ms_per_batch": kern,
                     "build_ms": sum(v for k, v in build.items()
                                     if not k.startswith("learned_") and k != "stree_fill"),
                     "fit_ms": sum(v for k, v in build.items()
                                   if k.startswith("learned_") or k == "stree_fill")}
        if search == sfc.LEARNED:
            info = idx.learned_info()
            out[name]["model"] = {k: info[k] for k in ("leaves_nonempty", "max_leaf", "pieces",
                                                       "mean_window", "max_window", "search_steps",
                                                       "fallbacks_last")}
        del out_ids
        # Secondary: queries from the mixture.
        _, ids0 = idx.query(qm, d)
        out_ids = torch.empty(ids0.numel() + 1024, dtype=torch.int32, device=dev)
        reps_m.append(int(ids0.numel()))
        del ids0
        idx.query(qm, d, out_ids=out_ids, out_offsets=offsets)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            idx.query(qm, d, out_ids=out_ids, out_offsets=offsets)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t0) / args.steps * 1e3
        out[name]["mixture_q"] = {"ms_per_batch": ms_m, "queries_per_s": m / (ms_m * 1e-3),
                                  "reported_pts_per_s": reps_m[-1] / (ms_m * 1e-3)}
        idx.close()
        del out_ids
    assert reps[0] == reps[1] == reps[2] and reps_m[0] == reps_m[1] == reps_m[2]
    out["reported_per_batch"] = reps[0]
    out["reported_per_batch_mixture_q"] = reps_m[0]
    out["speedup_batch"] = out["bsearch"]["ms_per_batch"] / out["learned"]["ms_per_batch"]
    out["speedup_search"] = out["bsearch"]["search_ms"] / out["learned"]["search_ms"]
    out["speedup_search_stree"] = out["bsearch"]["search_ms"] / out["stree"]["search_ms"]
    del pts, q, d, qm
    torch.cuda.empty_cache()
    return out


def early_term_bench(args, sfc, workload, torch, pts_c2):
    """Sparse queries, where early termination pays: the bench's clustered
    2^24 points (Hilbert) with 2^20 uniform queries aimed at one report per
    query at unit density (most land in the sparse background and report
    nothing); query batches over one built index with and without the
    occupancy bits."""
    dev = torch.device("cuda:0")
    n = pts_c2.shape[0]
    m = 1 << 20
    qh = workload.uniform_points(m, 7007)
    q = torch.as_tensor(qh).to(dev)
    d = torch.full((m,), workload.radius_for_count(1.0, n), dtype=torch.float64, device=dev)
    offsets = torch.empty(m + 1, dtype=torch.int64, device=dev)
    out = {"workload": f"clustered_n{n}_hilbert_uniformq_m{m}_c1"}
    for name, et in (("plain", False), ("early_term", True)):
        idx = sfc.Index(pts_c2, sfc.HILBERT, refine=True, early_term=et)
        _, ids0 = idx.query(q, d)
        out_ids = torch.empty(ids0.numel() + 1024, dtype=torch.int32, device=dev)
        rep = int(ids0.numel())
        for _ in range(max(1, args.warmup)):
            idx.query(q, d, out_ids=out_ids, out_offsets=offsets)
        ms, kern = timed_calls(lambda: idx.query(q, d, out_ids=out_ids, out_offsets=offsets),
                               args.steps)
        st = idx.last_stats()
        out[name] = {"ms_per_batch": ms, "queries_per_s": m / (ms * 1e-3), "reported": rep,
                     "candidates": st["candidates"], "cells_pruned": st["pruned"],
                     "kernels_ms_per_batch": {k: v[1] / args.steps for k, v in kern.items()}}
        idx.close()
    assert out["plain"]["reported"] == out["early_term"]["reported"]
    out["speedup_batch"] = out["plain"]["ms_per_batch"] / out["early_term"]["ms_per_batch"]
    # The paper's own empty and sparse queries: 10^7 normal points, 10^6
    # uniform square windows of small sides, Hilbert, refined ranges.
    nw, mw = 10_000_000, 1_000_000
    wl = workload.square_windows(n=nw, m=mw, side=1e-7, points="normal")
    pw = torch.as_tensor(wl.points).to(dev)
    qw = torch.as_tensor(wl.queries).to(dev)
    offw = torch.empty(mw + 1, dtype=torch.int64, device=dev)
    rows = []
    for side in (1e-7, 1e-5, 1e-4):
        dw = torch.full((mw,), side / 2, dtype=torch.float64, device=dev)
        res = {"side": side}
        for name, et in (("plain", False), ("early_term", True)):
            idx = sfc.Index(pw, sfc.HILBERT, refine=True, early_term=et, metric=sfc.LINF)
            _, ids0 = idx.query(qw, dw)
            ow = torch.empty(ids0.numel() + 1024, dtype=torch.int32, device=dev)
            res["reported"] = int(ids0.numel())
            for _ in range(max(1, args.warmup)):
                idx.query(qw, dw, out_ids=ow, out_offsets=offw)
            ms, _ = timed_calls(lambda: idx.query(qw, dw, out_ids=ow, out_offsets=offw),
                                args.steps)
            res[f"ms_{name}"] = ms
            idx.close()
        res["speedup_batch"] = res["ms_plain"] / res["ms_early_term"]
        rows.append(res)
    out["paper_windows"] = {"workload": f"normal_n{nw}_uniformq_m{mw}_square_windows_hilbert",
                            "sides": rows}
    del pw, qw
    torch.cuda.empty_cache()
    return out


def paper_windows_bench(args, sfc, workload, torch):
    """The paper's query sweep (Sec. 4): 10^7 points from its normal
    distribution (centre 1/2, sigma 1/8), 10^6 uniform query centres, square
    windows of relative side 1e-7 .. 0.02 (half side = side / 2); Morton
    (Curve-Z) and Hilbert (Curve-H) keys, with the method's ranges and with
    refined ranges.  The paper's single-threaded seconds for the same sweep
    (its own CPU, n = 10^7, 10^6 queries) ride along as context."""
    dev = torch.device("cuda:0")
    n, m = 10_000_000, 1_000_000
    sides = [1e-7, 1e-4, 1e-3, 1e-2, 2e-2]
    paper_s = {"morton": [0.114, 0.199, 0.696, 9.849, 34.773],
               "hilbert": [0.323, 0.324, 0.725, 9.765, 34.740]}
    wl = workload.square_windows(n=n, m=m, side=sides[0], points="normal")
    pts = torch.as_tensor(wl.points).to(dev)
    q = torch.as_tensor(wl.queries).to(dev)
    offsets = torch.empty(m + 1, dtype=torch.int64, device=dev)
    out = {"workload": f"normal_n{n}_uniformq_m{m}_square_windows",
           "paper_context": "single-threaded seconds per 10^6 queries, n = 10^7, "
                            "Xeon w5-3435X (the paper's sweep table)"}
    for cname, curve in (("morton", sfc.MORTON), ("hilbert", sfc.HILBERT)):
        for refine in (False, True):
            idx = sfc.Index(pts, curve, refine=refine, metric=sfc.LINF)
            rows = []
            for i, side in enumerate(sides):
                d = torch.full((m,), side / 2, dtype=torch.float64, device=dev)
                try:
                    idx.query(q, d, ids_cap=1, out_offsets=offsets)
                    total = int(offsets[m].item())
                except sfc.CapacityError as e:   # the usual case: only the size is wanted
                    total = int(e.total)
                out_ids = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
                steps = max(2, args.steps // (4 if side >= 1e-2 else 1))
                idx.query(q, d, out_ids=out_ids, out_offsets=offsets)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    idx.query(q, d, out_ids=out_ids, out_offsets=offsets)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / steps * 1e3
                st = idx.last_stats()
                rows.append({"side": side, "ms_per_batch": ms, "queries_per_s": m / (ms * 1e-3),
                             "reported": total, "reported_pts_per_s": total / (ms * 1e-3),
                             "candidates_per_report": st["candidates"] / max(total, 1),
                             "paper_cpu_s": paper_s[cname][i],
                             "paper_cpu_s_over_gpu_s": paper_s[cname][i] / (ms * 1e-3)})
                del out_ids
            out[f"{cname}_{'refined' if refine else 'ranges'}"] = rows
            log(f"windows {cname} refine={refine}: " +
                " ".join(f"{r['ms_per_batch']:.3g}" for r in rows) + " ms")
            idx.close()
    del pts, q
    torch.cuda.empty_cache()
    return out


def three_d_bench(args, sfc, workload, torch):
    """Three dimensions (d = 3 Morton keys): 2^24 clustered points in the
    unit cube, 2^20 queries from the same mixture with radii aimed at
    1..300 reports; one step = build + one query batch; refined cubes with
    binary search and with the static search tree, and the static search
    tree over the unsplit cubes."""
    dev = torch.device("cuda:0")
    wl = workload.clustered3(n=1 << 24, m=1 << 20)
    n, m = wl.points.shape[0], wl.queries.shape[0]
    pts = torch.as_tensor(wl.points).to(dev)
    q = torch.as_tensor(wl.queries).to(dev)
    d = torch.as_tensor(wl.delta).to(dev)
    offsets = torch.empty(m + 1, dtype=torch.int64, device=dev)
    out = {"workload": wl.name, "n": n, "m": m}
    reps = []
    for name, search, refine in (("bsearch", sfc.BINARY, True), ("stree", sfc.STREE, True),
                                 ("stree_unrefined", sfc.STREE, False)):
        idx = sfc.Index(pts, sfc.MORTON3, search=search, refine=refine)
        _, ids0 = idx.query(q, d)
        out_ids = torch.empty(ids0.numel() + 1024, dtype=torch.int32, device=dev)
        reps.append(int(ids0.numel()))
        del ids0
        idx.close()

        def step():
            ix = sfc.Index(pts, sfc.MORTON3, search=search, refine=refine)
            ix.query(q, d, out_ids=out_ids, out_offsets=offsets)
            return ix

        for _ in range(max(1, args.warmup)):
            step().close()
        ms, kern = timed_calls(lambda: step().close(), args.steps)
        kern = {k: v[1] / args.steps for k, v in kern.items()}
        ix = sfc.Index(pts, sfc.MORTON3, search=search, refine=refine)
        ix.query(q, d, out_ids=out_ids, out_offsets=offsets)
        cand = ix.last_stats()["candidates"]
        ix.close()
        out[name] = {"ms_per_step": ms, "queries_per_s": m / (ms * 1e-3),
                     "reported_pts_per_s": reps[-1] / (ms * 1e-3),
                     "candidates_per_report": cand / max(reps[-1], 1),
                     "kernels_ms_per_step": kern}
        del out_ids
        log(f"3-D {name}: {ms:.3f} ms per step (build + batch)")
    assert reps[0] == reps[1] == reps[2]
    out["reported_per_batch"] = reps[0]
    del pts, q, d
    torch.cuda.empty_cache()
    return out


def serving_bench(args, sfc, workload, torch):
    """Poisson stream of query / insert / erase batches (40/40/20 unless
    --serving-mix says otherwise, sizes 2^U[10,16]) over 2^25 clustered
    points, Morton keys, learned search:
    first the saturation throughput (every request queued at time 0), then
    arrivals at fractions of it; p50/p99 from arrival to completion.  Loops:
    sync (each tick's batch answered before the next tick), queued (batches
    queued on the index's stream into three output slots), overlap (batches
    side by side on three streams, each keeping its scratch and outputs for
    400 ids per query, admitted against a 2 GiB budget)."""
    from paper_2508_19891_amd import serving
    dev = torch.device("cuda:0")
    mix = tuple(float(x) for x in args.serving_mix.split(","))
    trace = workload.serving_trace(n0=1 << args.serving_n_log2, requests=args.serving_requests,
                                   mix=mix)
    log(f"serving: n0={len(trace.initial)}, {len(trace.kind)} requests")
    pools = serving.Pools.upload(trace, dev)
    init = torch.as_tensor(trace.initial).to(dev)
    out_ids = torch.empty(1 << 26, dtype=torch.int32, device=dev)
    out = {"workload": trace.name, "curve": "morton", "search": "learned",
           "mix": (f"{100 * mix[0]:.0f}% query, {100 * mix[1]:.0f}% insert, "
                   f"{100 * mix[2]:.0f}% erase batches of 2^U[10,16]")}
    kw = {"sync": {}, "queued": {"slots": 3, "slot_queries": 1 << 20, "slot_ids": 1 << 27,
                                 "slot_rows": 1 << 24},
          "overlap": {"streams": 3, "budget_bytes": 2 << 30, "ids_per_query": 400,
                      "slot_queries": 1 << args.serving_batch_log2}}

    def one(rate, mode):
        idx = sfc.Index(init, sfc.MORTON, search=sfc.LEARNED, refine=True)
        torch.cuda.synchronize()
        run = serving.serve(idx, trace, pools, rate=rate, out_ids=out_ids, **kw[mode])
        s = serving.summarize(trace, run)
        s["compactions"] = idx.update_info()["compactions"]
        if mode == "overlap":
            s["max_batches_in_flight"] = run.max_batches
            s["max_bytes_in_flight"] = run.max_in_flight
            s["requeued"] = run.requeued
        idx.close()
        return s

    for mode in args.serving_modes.split(","):
        sat = one(float("inf"), mode)
        res = {"saturation": sat}
        log(f"serving ({mode}) saturation: {sat['requests_per_s']:.0f} requests/s")
        for f in (float(x) for x in args.serving_loads.split(",") if x):
            rate = f * sat["requests_per_s"]
            s = one(rate, mode)
            s["offered_requests_per_s"] = rate
            res[f"load_{f}"] = s
            log(f"serving ({mode}) at {f} of saturation: p50 {s['p50_ms']:.2f} ms, "
                f"p99 {s['p99_ms']:.2f} ms")
        out[mode] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--m-log2", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=20)
    ap.add_argument("--only-refined", action="store_true",
                    help="time only the refined range mode (for profiler runs)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched point-set measurement")
    ap.add_argument("--no-learned-large", action="store_true",
                    help="skip the learned-index measurement at n=2^26")
    ap.add_argument("--no-early-term", action="store_true",
                    help="skip the early-termination measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the three-dimensional leg")
    ap.add_argument("--no-windows", action="store_true",
                    help="skip the paper's square-window sweep")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the insert/erase/query serving measurement")
    ap.add_argument("--serving-requests", type=int, default=10_000)
    ap.add_argument("--serving-modes", default="sync,overlap",
                    help="serving loops to time: sync (each tick answered before the next), "
                         "queued (batches queued on the index's stream), overlap (batches side "
                         "by side on their own streams, admitted by memory)")
    ap.add_argument("--serving-loads", default="0.5,0.8,0.95",
                    help="offered loads, as fractions of the saturation rate")
    ap.add_argument("--serving-batch-log2", type=int, default=17,
                    help="overlap loop: most queries in one batch (log2)")
    ap.add_argument("--serving-profile", action="store_true",
                    help="run the serving leg even with --only-refined (for kernel traces)")
    ap.add_argument("--serving-n-log2", type=int, default=25)
    ap.add_argument("--serving-mix", default="0.4,0.4,0.2",
                    help="fractions of query, insert and erase requests in the serving trace")
    ap.add_argument("--detail-out", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="file that receives every leg's figures (empty: none)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device three times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2508_19891_amd import sfc, workload

    if args.copy_probe:
        # Counter calibration: kernels of known traffic per launch, three
        # launches each -- a write-only fill of 2^30 bytes, a read-only sum
        # over 2^30 bytes (one scalar written), and a copy of 2^30 bytes.
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            a.fill_(1.0)
        for _ in range(3):
            s = a.sum()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b, s
        log("counter probe: 3 x fill, sum and copy of 2^30 B")

    # The attainable HBM rate: a plain device-to-device copy of 2^30 bytes
    # (2^31 bytes moved per copy), timed over 10 copies.
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    # And of a plain read-only stream: a sum over the same 2^30 bytes.
    s = a.sum()
    e0.record()
    for _ in range(10):
        s = a.sum()
    e1.record()
    torch.cuda.synchronize()
    read_gbs = 10 * (1 << 30) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b, s
    log(f"device copy: {copy_gbs:.0f} GB/s, read-only sum: {read_gbs:.0f} GB/s")

    n, m = 1 << args.n_log2, 1 << args.m_log2
    curve = sfc.HILBERT
    log(f"generating workload n={n} m={m}")
    wl = workload.clustered_loguniform(n=n, m=m, curve=curve)
    dev = torch.device("cuda:0")
    pts = torch.as_tensor(wl.points).to(dev)
    q = torch.as_tensor(wl.queries).to(dev)
    d = torch.as_tensor(wl.delta).to(dev)
    offsets = torch.empty(m + 1, dtype=torch.int64, device=dev)

    def run_mode(refine: bool, search: int = sfc.BINARY):
        # Size the output once (capacity errors in the timed region would be a bug).
        idx = sfc.Index(pts, curve, refine=refine, search=search)
        _, ids0 = idx.query(q, d)
        total = int(ids0.numel())
        stats = idx.last_stats()
        linfo = idx.learned_info() if search == sfc.LEARNED else None
        idx.close()
        out_ids = torch.empty(total + 1024, dtype=torch.int32, device=dev)
        del ids0
        log(f"refine={refine} search={search}: reports per batch {total}, "
            f"candidates {stats['candidates']}")

        def step():
            ix = sfc.Index(pts, curve, refine=refine, search=search)
            ix.query(q, d, out_ids=out_ids, out_offsets=offsets)
            ix.close()

        for i in range(args.warmup):
            step()
        # Per-kernel breakdown: the same steps with HIP events around every
        # launch (the events add gaps between kernels, so these steps are
        # not the timed ones).
        torch.cuda.synchronize()
        sfc.profile_reset()
        sfc.profile_enable(True)
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        sfc.profile_enable(False)
        kern = sfc.profile_read()
        dom = max((k for k in ROOFLINE_KERNELS if k in kern), key=lambda k: kern[k][1])
        # Timed steps: events only around the dominant kernel's launches.
        sfc.profile_reset()
        sfc.profile_only(dom)
        sfc.profile_enable(True)
        # one event pair per step on the library's stream (torch's current
        # stream): the median step beside the whole timed region's mean
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for i in range(args.steps):
            step()
            ev[i + 1].record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sfc.profile_enable(False)
        sfc.profile_only(None)
        kern_dom = sfc.profile_read()
        per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
        log(f"timed {args.steps} steps in {dt:.3f} s")
        if linfo is not None:
            stats = dict(stats, learned=linfo)
        return (dt / args.steps * 1e3, kern, stats, total, (dom, kern_dom.get(dom)),
                float(np.median(per_step)))

    if args.only_refined:
        ms_paper, kern_paper, stats_paper = float("nan"), {}, {"candidates": None}
    else:
        ms_paper, kern_paper, stats_paper, _, _, _ = run_mode(False)
    ms_step, kern, stats, total, (dom_timed, dom_kern), ms_median = run_mode(True)
    def query_only(search: int, cells: bool = True):
        """One index (built and, for the learned search, fitted once); the
        timed steps are query batches only.  cells=False: every candidate
        takes the exact test (no decisions from grid cells)."""
        torch.cuda.synchronize()
        sfc.profile_reset()
        sfc.profile_enable(True)
        idx = sfc.Index(pts, curve, refine=True, search=search)
        idx.set_cell_filter(cells)
        torch.cuda.synchronize()
        sfc.profile_enable(False)
        fit = {k: v[1] for k, v in sfc.profile_read().items() if k.startswith("learned_")}
        _, ids0 = idx.query(q, d)
        out_ids = torch.empty(ids0.numel() + 1024, dtype=torch.int32, device=dev)
        del ids0
        for _ in range(max(1, args.warmup)):
            idx.query(q, d, out_ids=out_ids, out_offsets=offsets)
        dt, kern_q = timed_calls(lambda: idx.query(q, d, out_ids=out_ids, out_offsets=offsets),
                                 args.steps)
        kern_q = {k: v[1] / args.steps for k, v in kern_q.items()}
        info = idx.learned_info() if search == sfc.LEARNED else None
        rep_q = idx.last_stats()["reported"]
        idx.close()
        log(f"query-only search={search}: {dt:.3f} ms per batch")
        return dt, kern_q, fit, info, rep_q

    if args.only_refined:
        lvb = None
    else:
        ms_qb, kern_qb, _, _, rep_qb = query_only(sfc.BINARY)
        ms_ql, kern_ql, fit_l, info_l, rep_ql = query_only(sfc.LEARNED)
        ms_qs, kern_qs, _, _, rep_qs = query_only(sfc.STREE)
        ms_qx, kern_qx, _, _, rep_qx = query_only(sfc.BINARY, cells=False)
        assert rep_qb == rep_ql == rep_qs == rep_qx == total
        lvb = {
            "step": "one query batch over a built index (refined ranges); the learned index is "
                    "fitted once beforehand",
            "queries_per_s_learned": m / (ms_ql * 1e-3),
            "queries_per_s_bsearch": m / (ms_qb * 1e-3),
            "reported_pts_per_s_learned": rep_ql / (ms_ql * 1e-3),
            "reported_pts_per_s_bsearch": rep_qb / (ms_qb * 1e-3),
            "ms_per_batch_learned": ms_ql,
            "ms_per_batch_bsearch": ms_qb,
            "speedup_batch": ms_qb / ms_ql,
            "search_ms_learned": kern_ql.get("ranges_learned", float("nan")),
            "search_ms_bsearch": kern_qb.get("ranges_search", float("nan")),
            "speedup_search": kern_qb.get("ranges_search", float("nan"))
            / kern_ql.get("ranges_learned", float("nan")),
            "fit_ms_once": fit_l,
            "kernels_ms_per_batch_learned": kern_ql,
            "kernels_ms_per_batch_bsearch": kern_qb,
            "model": {k: info_l.get(k) for k in
                      ("steps", "loss_init", "loss_final", "leaves_nonempty", "max_leaf", "pieces",
                       "mean_window", "max_window", "search_steps", "endpoints_last",
                       "fallbacks_last")},
            # the third search: the static search tree over the keys
            "queries_per_s_stree": m / (ms_qs * 1e-3),
            "ms_per_batch_stree": ms_qs,
            "search_ms_stree": kern_qs.get("ranges_stree", float("nan")),
            "kernels_ms_per_batch_stree": kern_qs,
        }
        # The same batch (binary search) with every candidate taking the exact
        # test: the test kernel then reads 16 B per candidate.
        cand_q = stats["candidates"]
        ct_x = kern_qx.get("compact_test", float("nan"))
        exact_bytes = 16 * cand_q + 24 * m + 12 * 8 * m + cand_q // 8 + 4 * math.ceil(cand_q / 4096)
        cell_filter = {
            "step": "one query batch over a built index (refined ranges, binary search)",
            "ms_per_batch_cells": ms_qb, "ms_per_batch_exact": ms_qx,
            "compact_test_ms_cells": kern_qb.get("compact_test", float("nan")),
            "compact_test_ms_exact": ct_x,
            "exact_compact_test_gbs": exact_bytes / (ct_x * 1e-3) / 1e9,
            "exact_compact_test_frac": exact_bytes / (ct_x * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }

    # Algorithmic bytes per step of each kernel (what the method must move).
    cand, rep = stats["candidates"], total
    passes = round(kern["scatter_pass"][0] / args.steps)   # radix passes per build
    tiles = math.ceil(cand / 4096)
    slots = 8 * m   # refined layout: eight slots (begin u32, count u32, offset u64) per query
    algo = {
        "keygen_tiles": 16 * n + 8 * n + 16 * n,            # points in, keys and input-order copy out
        "tile_hist": (passes - 1) * 8 * n,                  # passes 2.. read the keys
        "scatter_pass": passes * 24 * n,                    # (key+id) in and out per pass
        "ranges_search": 24 * m + 8 * slots,                # queries in; begin+count per slot
        # default: each candidate's 8-byte grid cell, the 32-byte filter record
        # of its query per row (the rare undecided candidates read 16 B more)
        "compact_test": 8 * cand + 32 * m + 12 * slots + cand // 8 + 4 * tiles,
        "query_filters": 24 * m + 32 * m,
        "compact_write": cand // 8 + 8 * tiles + 4 * rep + 4 * rep + 8 * (m + 1) + 12 * slots,
    }
    if "chunk_sort" in kern:
        # Chunks of equal top key bits: (key+id) in and out, the grid cell out.
        algo["chunk_sort"] = 12 * n + 12 * n + 8 * n
    else:
        # The last radix pass also writes each point's 8-byte grid cell.
        algo["scatter_pass"] += 8 * n
    kern_gbs = {}
    for k, b in algo.items():
        if k in kern:
            kern_gbs[k] = b / (kern[k][1] / args.steps * 1e-3) / 1e9
    # The dominant kernel (by time in the profiled steps) and its launches
    # timed by HIP events inside the timed steps.
    dom = dom_timed
    d_launch, d_ms = dom_kern if dom_kern else kern[dom]
    launches_per_step = d_launch / args.steps
    bytes_per_launch = algo[dom] / launches_per_step
    achieved = bytes_per_launch / (d_ms / d_launch * 1e-3) / 1e9
    traffic = load_traffic(dom, "build.hip" if dom in ("keygen_tiles", "tile_hist", "digit_scan", "scatter_pass",
                                                       "chunk_sort")
                           else "query.hip")

    detail = {
        "config": {"workload": wl.name + "_hilbert", "n": n, "m": m, "curve": "hilbert",
                   "search": "binary", "ranges": "refined", "step": "build + one query batch"},
        "ms_per_step": ms_step,
        "ms_per_step_median": ms_median,
        "learned_vs_bsearch": lvb,
        "cell_filter": None if args.only_refined else cell_filter,
        "paper_ranges": {"queries_per_s": m / (ms_paper * 1e-3), "ms_per_step": ms_paper,
                         "candidates_per_step": stats_paper["candidates"],
                         "kernels_ms_per_step": {k: v[1] / args.steps
                                                 for k, v in kern_paper.items()}},
        "reported_pts_per_s": rep / (ms_step * 1e-3),
        "reported_per_step": rep,
        "candidates_per_step": cand,
        "candidates_per_report": cand / max(rep, 1),
        "build_ms_per_step": sum(kern[k][1] for k in ("keygen_tiles", "tile_hist", "digit_scan",
                                                      "scatter_pass", "chunk_firsts", "chunk_sort")
                                 if k in kern) / args.steps,
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in kern.items()},
        "kernels_algorithmic_bytes_per_step": algo,
        "kernels_algorithmic_gbs": kern_gbs,
        "copy_gbs": copy_gbs,
        "read_gbs": read_gbs,
    }
    # The dominant kernel's roofline on its own design's bytes, and on the
    # scan bytes the method's description gives (16 B per candidate for the
    # test pass plus 12 B per query: the coordinates of every candidate), for
    # comparison; the latter can exceed 1 because the kernel decides most
    # candidates from their 8-byte grid cell and never reads those bytes.
    # Beside them, the kernel's counted bytes over the same time (when the
    # counters match its current source) and the rates of a plain read-only
    # stream and a plain copy measured in this run.
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_gbs": (traffic / (d_ms / d_launch * 1e-3) / 1e9) if traffic else None,
                "bytes_per_launch": bytes_per_launch, "read_gbs": read_gbs, "copy_gbs": copy_gbs}
    if dom == "compact_test":
        survey_bytes = (16 * cand + 12 * m) / launches_per_step
        roofline["frac_16B_per_candidate"] = (survey_bytes / (d_ms / d_launch * 1e-3) / 1e9
                                              / HBM_PEAK_GBS)
    detail["roofline"] = roofline
    if dom != "compact_test" and "compact_test" in kern:
        # Another kernel dominates: the scan's test pass, the main stream
        # over the candidates, is reported beside it (timed by the HIP events
        # of the profiled steps).
        c_launch, c_ms = kern["compact_test"]
        c_bytes = algo["compact_test"] / (c_launch / args.steps)
        c_gbs = c_bytes / (c_ms / c_launch * 1e-3) / 1e9
        detail["roofline_scan"] = {"kernel": "compact_test", "bound": "hbm", "achieved": c_gbs,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": c_gbs / HBM_PEAK_GBS,
                                   "traffic": load_traffic("compact_test", "query.hip")}
    if not args.no_batched and not args.only_refined:
        detail["batched_sets"] = batched_sets_bench(args, sfc, workload, torch)
    if not args.no_early_term and not args.only_refined:
        detail["early_termination"] = early_term_bench(args, sfc, workload, torch, pts)
    if not args.no_windows and not args.only_refined:
        detail["paper_windows"] = paper_windows_bench(args, sfc, workload, torch)
    if not args.no_3d and not args.only_refined:
        detail["three_d"] = three_d_bench(args, sfc, workload, torch)
    if not args.no_learned_large and not args.only_refined:
        detail["learned_large"] = learned_large_bench(args, sfc, workload, torch)
    if (not args.no_serving and not args.only_refined) or args.serving_profile:
        detail["serving"] = serving_bench(args, sfc, workload, torch)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        detail["cpu_baseline"] = cpu_baseline(wl, curve, min(m, 1 << args.cpu_sample_log2))

    line = headline(args, detail, n, m, ms_step, ms_median)
    if args.detail_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail_out)), exist_ok=True)
        with open(args.detail_out, "w") as f:
            json.dump(detail, f, indent=1)
        line["detail"] = os.path.relpath(os.path.abspath(args.detail_out), ROOT)
    print(json.dumps(line, separators=(",", ":")), flush=True)


def _r(v, digits: int = 4):
    """A float rounded to `digits` significant digits (None stays None)."""
    if v is None or not isinstance(v, float) or not math.isfinite(v):
        return v
    return float(f"{v:.{digits}g}")


def headline(args, detail: dict, n: int, m: int, ms_step: float, ms_median: float) -> dict:
    """The one JSON line the bench prints last: the metric, its workload,
    the dominant kernel's roofline, the oracle's rate on the host, and short
    summaries of the learned-versus-binary and early-termination legs (the
    full figures go to the detail file)."""
    rl = detail["roofline"]
    out = {
        "metric": "queries/s + reported pts/s at n=2^24, learned vs bsearch index, % HBM peak",
        "value": _r(m / (ms_step * 1e-3), 6),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": _r(ms_step, 5),
        "ms_per_step_median": _r(ms_median, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": detail["config"],
        "reported_pts_per_s": _r(detail["reported_pts_per_s"]),
        "candidates_per_report": _r(detail["candidates_per_report"]),
        "build_ms": _r(detail["build_ms_per_step"]),
        "roofline": {k: _r(v) for k, v in rl.items()},
    }
    if "roofline_scan" in detail:
        rs = detail["roofline_scan"]
        out["roofline_scan"] = {k: _r(rs[k]) for k in ("kernel", "achieved", "frac", "traffic")}
    lvb = detail.get("learned_vs_bsearch")
    if lvb:
        s = {"n": n, "search_ms_learned": _r(lvb["search_ms_learned"]),
             "search_ms_bsearch": _r(lvb["search_ms_bsearch"]),
             "search_ms_stree": _r(lvb["search_ms_stree"]),
             "ms_per_batch_learned": _r(lvb["ms_per_batch_learned"]),
             "ms_per_batch_bsearch": _r(lvb["ms_per_batch_bsearch"]),
             "fallbacks": lvb["model"].get("fallbacks_last")}
        ll = detail.get("learned_large")
        if ll:
            s["large"] = {"n": ll["n"], "m": ll["m"],
                          "search_ms_learned": _r(ll["learned"]["search_ms"]),
                          "search_ms_bsearch": _r(ll["bsearch"]["search_ms"]),
                          "ms_per_batch_learned": _r(ll["learned"]["ms_per_batch"]),
                          "ms_per_batch_bsearch": _r(ll["bsearch"]["ms_per_batch"])}
        out["learned_vs_bsearch"] = s
    et = detail.get("early_termination")
    if et:
        out["early_termination"] = {"speedup_batch": _r(et["speedup_batch"]),
                                    "ms_plain": _r(et["plain"]["ms_per_batch"]),
                                    "ms_early_term": _r(et["early_term"]["ms_per_batch"])}
        if "paper_windows" in et:
            out["early_termination"]["speedup_windows"] = {
                f"{r['side']:g}": _r(r["speedup_batch"], 3) for r in et["paper_windows"]["sides"]}
    sv = detail.get("serving")
    mode = next((k for k in ("overlap", "queued", "sync") if sv and k in sv), None)
    if mode:
        q = sv[mode]
        out["serving"] = {"mode": mode, "requests": q["saturation"]["requests"],
                          "requests_per_s": _r(q["saturation"]["requests_per_s"])}
        if "load_0.95" in q:
            out["serving"]["p50_ms_0.95"] = _r(q["load_0.95"]["p50_ms"])
            out["serving"]["p99_ms_0.95"] = _r(q["load_0.95"]["p99_ms"])
    cb = detail.get("cpu_baseline")
    if cb:
        out["cpu_baseline"] = {"value": _r(cb["value"]), "unit": cb["unit"],
                               "cores": cb["cores"], "kind": cb["kind"], "sample": cb["sample"]}
    return out


if __name__ == "__main__":
    main()

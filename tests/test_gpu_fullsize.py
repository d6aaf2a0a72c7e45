"""Parity at every workload's full shape: the whole CSR output (offsets, and
every id in curve order) compared with the oracle element by element.

  * clustered 2^24 points, 2^20 queries with radii aimed at 1..1000 reports
    (Hilbert): binary search, learned index and static search tree over the
    refined cells, the method's own cells (Alg. 1), early termination with
    sparse uniform queries, and square windows;
  * three dimensions, 2^24 points and 2^20 queries (d = 3 Morton keys);
  * the learned-index shape: 2^26 clustered points, Morton keys, 2^22
    uniform queries with delta = sqrt(10 / (pi n)), every search;
  * 256 uneven point sets (sizes 2^U[10,20], 2^U[8,16] queries each), built
    and queried through recorded graphs, against the oracle run set by set;
  * serving from 2^25 clustered points: query requests of a mixed stream of
    queries, inserts and erases against the oracle over the snapshot of the
    epoch each was admitted at.

The oracle answers each batch on every host core this process may use."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, L2, LINF, MORTON
from paper_2508_19891_amd import serving, sfc, workload
from snapshots import Model

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N, M = 1 << 24, 1 << 20
THREADS = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))


def host_csr(off, ids):
    return off.cpu().numpy().view(np.uint64), ids.cpu().numpy().view(np.uint32)


def assert_csr_equal(got, want, what):
    off, ids = got
    ref_off, ref_ids = want
    assert off.shape == ref_off.shape, what
    if not np.array_equal(off, ref_off):
        j = int(np.nonzero(off != ref_off)[0][0])
        pytest.fail(f"{what}: offsets differ first at query {j}: {off[j]} vs {ref_off[j]}")
    assert ids.shape == ref_ids.shape, what
    if not np.array_equal(ids, ref_ids):
        p = int(np.nonzero(ids != ref_ids)[0][0])
        j = int(np.searchsorted(ref_off, p, side="right")) - 1
        pytest.fail(f"{what}: ids differ first at output {p} (query {j})")


@pytest.fixture(scope="module")
def clustered():
    wl = workload.clustered_loguniform(n=N, m=M, curve=HILBERT)
    uq = workload.uniform_points(M, 7007)     # the early-termination leg's queries
    ud = np.full(M, workload.radius_for_count(1.0, N))
    print("oracle: building 2^24 points", flush=True)
    ref_index = oracle.build(wl.points, HILBERT)
    return {"wl": wl, "pts": torch.as_tensor(wl.points).to(DEV), "uq": uq, "ud": ud,
            "index": ref_index, "answers": {}}


CONFIGS = [
    # (search, refine, metric, early_term, queries)
    (sfc.BINARY, True, L2, False, "clustered"),      # the headline step
    (sfc.LEARNED, True, L2, False, "clustered"),     # learned-index leg
    (sfc.STREE, True, L2, False, "clustered"),       # static search tree
    (sfc.BINARY, False, L2, False, "clustered"),     # the method's ranges, unrefined
    (sfc.LEARNED, False, L2, False, "clustered"),
    (sfc.BINARY, True, L2, True, "uniform"),         # early-termination leg
    (sfc.BINARY, True, LINF, False, "clustered"),    # square windows
]


@pytest.mark.parametrize("search,refine,metric,early_term,queries", CONFIGS)
def test_clustered_full_batch(clustered, search, refine, metric, early_term, queries):
    wl = clustered["wl"]
    qs, ds = (wl.queries, wl.delta) if queries == "clustered" else (clustered["uq"],
                                                                   clustered["ud"])
    what = (f"full size: search={search} refine={refine} metric={metric} "
            f"early_term={early_term} queries={queries}")
    print(what, flush=True)
    key = (queries, metric)
    if key not in clustered["answers"]:
        clustered["answers"][key] = oracle.query(clustered["index"], qs, ds, HILBERT,
                                                 nthreads=THREADS, metric=metric)
    want = clustered["answers"][key]
    idx = sfc.Index(clustered["pts"], HILBERT, search=search, refine=refine,
                    early_term=early_term, metric=metric)
    got = host_csr(*idx.query(torch.as_tensor(qs).to(DEV), torch.as_tensor(ds).to(DEV)))
    if search == sfc.LEARNED:
        assert idx.learned_info()["fallbacks_last"] == 0
    idx.close()
    assert_csr_equal(got, want, what)
    assert int(want[0][-1]) > M // 2


def test_three_d_full_batch():
    """Three dimensions at 2^24 points and 2^20 queries (the 3-D leg's
    shape), static search tree and binary search over refined cubes."""
    wl = workload.clustered3(n=N, m=M)
    print("oracle: 3-D build and batch", flush=True)
    want = oracle.query3(oracle.build3(wl.points), wl.queries, wl.delta, nthreads=THREADS)
    pts = torch.as_tensor(wl.points).to(DEV)
    for search in (sfc.STREE, sfc.BINARY):
        print(f"3-D full size: search={search}", flush=True)
        idx = sfc.Index(pts, sfc.MORTON3, search=search, refine=True)
        got = host_csr(*idx.query(torch.as_tensor(wl.queries).to(DEV),
                                  torch.as_tensor(wl.delta).to(DEV)))
        idx.close()
        assert_csr_equal(got, want, f"3-D search={search}")


def test_learned_shape_full_batch():
    """2^26 clustered points, Morton keys, 2^22 uniform queries with
    delta = sqrt(10 / (pi n)): binary search, the learned index and the
    static search tree give the oracle's whole output."""
    wl = workload.clustered_uniform_queries(n=1 << 26, m=1 << 22, curve=MORTON)
    print("oracle: building 2^26 points", flush=True)
    want = oracle.query(oracle.build(wl.points, MORTON), wl.queries, wl.delta, MORTON,
                        nthreads=THREADS)
    pts = torch.as_tensor(wl.points).to(DEV)
    q = torch.as_tensor(wl.queries).to(DEV)
    d = torch.as_tensor(wl.delta).to(DEV)
    for search in (sfc.BINARY, sfc.LEARNED, sfc.STREE):
        print(f"2^26 full size: search={search}", flush=True)
        idx = sfc.Index(pts, MORTON, search=search)
        got = host_csr(*idx.query(q, d))
        if search == sfc.LEARNED:
            info = idx.learned_info()
            assert info["fallbacks_last"] == 0 and info["leaves_nonempty"] > 1000
        idx.close()
        assert_csr_equal(got, want, f"2^26 search={search}")
    del pts, q, d
    torch.cuda.empty_cache()


def oracle_sets(wl, curve):
    """The oracle run set by set (each set's ids shifted to input
    positions), in the batch's query order; sets in parallel threads."""
    nsets = len(wl.set_off) - 1
    qoff = np.searchsorted(wl.qset, np.arange(nsets + 1))

    def one(s):
        a, b = int(wl.set_off[s]), int(wl.set_off[s + 1])
        qa, qb = int(qoff[s]), int(qoff[s + 1])
        if qa == qb:
            return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
        if a == b:
            return np.zeros(qb - qa, np.uint64), np.zeros(0, np.uint32)
        off, ids = oracle.query(oracle.build(wl.points[a:b], curve), wl.queries[qa:qb],
                                wl.delta[qa:qb], curve)
        return np.diff(off), ids + np.uint32(a)

    with ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(one, range(nsets)))
    counts = np.concatenate([p[0] for p in parts]).astype(np.uint64)
    offs = np.zeros(len(wl.queries) + 1, np.uint64)
    offs[1:] = np.cumsum(counts)
    return offs, np.concatenate([p[1] for p in parts]).astype(np.uint32)


def test_batched_sets_full_through_graphs():
    """256 uneven sets (the batched workload's shape), built and queried by
    replaying the two recorded graphs, against the per-set oracle; the eager
    batched calls too."""
    wl = workload.batched_uneven(n_sets=256, curve=MORTON)
    assert np.all(np.diff(wl.qset.astype(np.int64)) >= 0)
    print(f"sets: {len(wl.points)} points, {len(wl.queries)} queries", flush=True)
    want = oracle_sets(wl, MORTON)
    pts = torch.as_tensor(wl.points).to(DEV)
    q = torch.as_tensor(wl.queries).to(DEV)
    d = torch.as_tensor(wl.delta).to(DEV)
    qs = torch.as_tensor(wl.qset.astype(np.int32)).to(DEV)
    idx = sfc.Index(pts, MORTON, refine=True, set_off=wl.set_off)
    eager = host_csr(*idx.query_sets(q, d, qs))
    assert_csr_equal(eager, want, "sets, eager")
    rows, rep = idx.last_stats()["rows"], int(want[0][-1])
    gb = sfc.Graph.build(idx, pts)
    gq = sfc.Graph.query(idx, q, d, max_rows=rows + 64, ids_cap=rep + 1, qset=qs)
    for replay in range(2):
        gb.launch()
        gb.wait()
        gq.launch()
        assert gq.wait() == rep
        off, ids = gq.result()
        assert_csr_equal(host_csr(off, ids[:rep]), want, f"sets, graph replay {replay}")
    gb.close()
    gq.close()
    idx.close()


def test_serving_from_2p25_points():
    """A short mixed stream (queries, inserts, erases) over 2^25 clustered
    points, Morton keys, learned search, query batches queued without
    waiting: query requests at several epochs equal the oracle over their
    snapshot."""
    trace = workload.serving_trace(n0=1 << 25, requests=40, seed=5)
    pools = serving.Pools.upload(trace, DEV)
    idx = sfc.Index(torch.as_tensor(trace.initial).to(DEV), MORTON, search=sfc.LEARNED,
                    refine=True)
    run = serving.serve(idx, trace, pools, record=True, slots=3)
    idx.close()
    model = Model(trace.initial, hold=True)
    at = {}
    for r in range(len(trace.kind)):
        a, k = int(trace.start[r]), int(trace.size[r])
        if trace.kind[r] == workload.INSERT:
            model.insert(trace.inserts[a:a + k])
        elif trace.kind[r] == workload.ERASE:
            model.erase(trace.erase_ids[a:a + k])
        else:
            at[r] = model.epoch
    by_epoch = {}
    for r, e in at.items():
        by_epoch.setdefault(e, r)
    epochs = sorted(by_epoch)
    picks = [by_epoch[e] for e in (epochs[0], epochs[len(epochs) // 2], epochs[-1])]
    assert len(set(at.values())) >= 3
    for r in dict.fromkeys(picks):
        e = at[r]
        assert run.admitted[r] == e
        a, k = int(trace.start[r]), int(trace.size[r])
        print(f"serving: request {r} at epoch {e}, {k} queries", flush=True)
        want = model.reference(trace.queries[a:a + k], trace.delta[a:a + k], np.full(k, e),
                               MORTON)
        off, ids = run.outputs[r]
        assert_csr_equal((off.view(np.uint64), ids.view(np.uint32)), want, f"request {r}")

"""Parity at the benchmark's full size: 2^24 clustered points, 2^20 queries
with radii aimed at 1..1000 reports (Hilbert keys), in the configurations
the benchmark times.  The oracle cannot answer the whole batch in seconds,
so: every query's offsets are consistent, every reported id passes the exact
test (checked in numpy, in the test's fixed operation order), a seeded
sample of queries equals brute force over all 2^24 points id for id, and
their ids come in curve order."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, L2, LINF
from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N, M = 1 << 24, 1 << 20
SAMPLE = 48


@pytest.fixture(scope="module")
def full():
    wl = workload.clustered_loguniform(n=N, m=M, curve=HILBERT)
    uq = workload.uniform_points(M, 7007)     # the early-termination leg's queries
    ud = np.full(M, workload.radius_for_count(1.0, N))
    return wl, torch.as_tensor(wl.points).to(DEV), uq, ud


def accepted(pts, q, d, metric):
    dx = pts[:, 0] - q[:, 0]
    dy = pts[:, 1] - q[:, 1]
    if metric == LINF:
        return (np.abs(dx) <= d) & (np.abs(dy) <= d)
    return dx * dx + dy * dy <= d * d


CONFIGS = [
    # (search, refine, metric, early_term, queries)
    (sfc.BINARY, True, L2, False, "clustered"),      # the headline step
    (sfc.LEARNED, True, L2, False, "clustered"),     # learned-index leg
    (sfc.STREE, True, L2, False, "clustered"),       # static search tree
    (sfc.BINARY, False, L2, False, "clustered"),     # the method's ranges, unrefined
    (sfc.BINARY, True, L2, True, "uniform"),         # early-termination leg
    (sfc.BINARY, True, LINF, False, "clustered"),    # square windows
]


@pytest.mark.parametrize("search,refine,metric,early_term,queries", CONFIGS)
def test_full_size(full, search, refine, metric, early_term, queries):
    wl, pts_d, uq, ud = full
    qs, ds = (wl.queries, wl.delta) if queries == "clustered" else (uq, ud)
    print(f"full size: search={search} refine={refine} metric={metric} "
          f"early_term={early_term} queries={queries}", flush=True)
    idx = sfc.Index(pts_d, HILBERT, search=search, refine=refine, early_term=early_term,
                    metric=metric)
    off, ids = idx.query(torch.as_tensor(qs).to(DEV), torch.as_tensor(ds).to(DEV))
    off = off.cpu().numpy().view(np.uint64).astype(np.int64)
    ids = ids.cpu().numpy().view(np.uint32)
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == ids.size
    assert ids.size > M // 2
    # Soundness of every report, in chunks of queries.
    for a in range(0, M, 1 << 16):
        b = min(M, a + (1 << 16))
        sl = slice(off[a], off[b])
        qi = np.repeat(np.arange(a, b), np.diff(off[a:b + 1]))
        assert accepted(wl.points[ids[sl]], qs[qi], ds[qi], metric).all(), a
    # Completeness and order on a sample: brute force over every point.
    rng = np.random.default_rng(71)
    sample = np.sort(rng.choice(M, SAMPLE, replace=False))
    sample[0] = int(np.argmax(np.diff(off)))          # the largest output too
    ref = oracle.brute(wl.points, qs[sample], ds[sample], metric=metric)
    rank = np.empty(N, np.int64)
    rank[idx.sorted_arrays()[1].cpu().numpy().view(np.uint32)] = np.arange(N)
    for t, j in enumerate(sample):
        got = ids[off[j]:off[j + 1]]
        assert np.array_equal(np.sort(got), ref[1][ref[0][t]:ref[0][t + 1]]), j
        assert np.all(np.diff(rank[got]) > 0), j
    idx.close()


def test_full_size_3d():
    """Three dimensions at 2^24 points and 2^20 queries (the 3-D bench leg's
    shape), static search tree, refined cubes: offsets, soundness of every report in the
    3-D test's order, a sample against brute force."""
    wl = workload.clustered3(n=N, m=M)
    qs, ds = wl.queries, wl.delta
    idx = sfc.Index(torch.as_tensor(wl.points).to(DEV), sfc.MORTON3, search=sfc.STREE,
                    refine=True)
    off, ids = idx.query(torch.as_tensor(qs).to(DEV), torch.as_tensor(ds).to(DEV))
    off = off.cpu().numpy().view(np.uint64).astype(np.int64)
    ids = ids.cpu().numpy().view(np.uint32)
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == ids.size
    for a in range(0, M, 1 << 16):
        b = min(M, a + (1 << 16))
        sl = slice(off[a], off[b])
        qi = np.repeat(np.arange(a, b), np.diff(off[a:b + 1]))
        p, q, d = wl.points[ids[sl]], qs[qi], ds[qi]
        dx, dy, dz = p[:, 0] - q[:, 0], p[:, 1] - q[:, 1], p[:, 2] - q[:, 2]
        assert ((dx * dx + dy * dy) + dz * dz <= d * d).all(), a
    rng = np.random.default_rng(72)
    sample = np.sort(rng.choice(M, SAMPLE, replace=False))
    sample[0] = int(np.argmax(np.diff(off)))
    ref = oracle.brute3(wl.points, qs[sample], ds[sample])
    for t, j in enumerate(sample):
        got = np.sort(ids[off[j]:off[j + 1]])
        assert np.array_equal(got, ref[1][ref[0][t]:ref[0][t + 1]]), j
    idx.close()

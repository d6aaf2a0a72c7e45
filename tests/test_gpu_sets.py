"""Batched independent point sets through the C ABI, against the oracle run
set by set (ids are input positions; each query only sees its own set)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def oracle_sets(wl, curve):
    """Per-set oracle CSR in the batch's query order (queries grouped by set)."""
    m = len(wl.queries)
    counts = np.zeros(m, np.int64)
    rows = [None] * m
    for s in range(len(wl.set_off) - 1):
        a, b = int(wl.set_off[s]), int(wl.set_off[s + 1])
        sel = np.nonzero(wl.qset == s)[0]
        if len(sel) == 0:
            continue
        if b == a:
            for j in sel:
                rows[j] = np.zeros(0, np.uint32)
            continue
        off, ids = oracle.query(oracle.build(wl.points[a:b], curve), wl.queries[sel],
                                wl.delta[sel], curve)
        for t, j in enumerate(sel):
            rows[j] = ids[off[t]:off[t + 1]].astype(np.uint64) + a
    for j in range(m):
        counts[j] = len(rows[j])
    offs = np.zeros(m + 1, np.uint64)
    offs[1:] = np.cumsum(counts)
    return offs, (np.concatenate(rows).astype(np.uint32) if m else np.zeros(0, np.uint32))


def check_sets(wl, curve, refine=False):
    idx = sfc.Index(dev(wl.points), curve, refine=refine, set_off=wl.set_off)
    off, ids = idx.query_sets(dev(wl.queries), dev(wl.delta), dev(wl.qset, torch.int32))
    ref_off, ref_ids = oracle_sets(wl, curve)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref_off)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref_ids)
    return idx


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_batched_uneven_sets(curve, refine):
    wl = workload.batched_uneven(n_sets=40, log2_n=(4, 13), log2_m=(2, 9), curve=curve, seed=3)
    check_sets(wl, curve, refine)


def test_sorted_arrays_are_per_set_sorts():
    wl = workload.batched_uneven(n_sets=30, log2_n=(0, 12), log2_m=(1, 3), curve=MORTON, seed=5)
    idx = sfc.Index(dev(wl.points), MORTON, set_off=wl.set_off)
    k, i, xy = idx.sorted_arrays()
    k = sfc.u64(k)
    i = i.cpu().numpy().view(np.uint32)
    for s in range(30):
        a, b = int(wl.set_off[s]), int(wl.set_off[s + 1])
        ok, oi, _ = oracle.build(wl.points[a:b], MORTON)
        assert np.array_equal(k[a:b], ok)
        assert np.array_equal(i[a:b], oi + a)


def test_many_sets_two_set_passes_and_empty_sets():
    rng = np.random.default_rng(9)
    sizes = rng.integers(0, 40, 700)
    sizes[::7] = 0                                   # empty sets
    set_off = np.zeros(701, np.uint64)
    set_off[1:] = np.cumsum(sizes)
    pts = rng.random((int(set_off[-1]), 2))
    m_per = rng.integers(0, 4, 700)
    qset = np.repeat(np.arange(700), m_per).astype(np.uint32)
    qs = rng.random((len(qset), 2))
    ds = 10 ** rng.uniform(-2, -0.3, len(qset))
    wl = workload.BatchedWorkload("many", pts, set_off, qs, ds, qset, HILBERT)
    check_sets(wl, HILBERT)


def test_single_set_equals_plain_build():
    wl = workload.uniform_fixed_radius(n=20_000, m=3000, curve=MORTON)
    idx = sfc.Index(dev(wl.points), MORTON, set_off=[0, 20_000])
    a = idx.query_sets(dev(wl.queries), dev(wl.delta), torch.zeros(3000, dtype=torch.int32,
                                                                   device=DEV))
    plain = sfc.Index(dev(wl.points), MORTON)
    b = plain.query(dev(wl.queries), dev(wl.delta))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_query_sets_invalid_set():
    wl = workload.batched_uneven(n_sets=5, log2_n=(4, 6), log2_m=(1, 2), seed=1)
    idx = sfc.Index(dev(wl.points), MORTON, set_off=wl.set_off)
    qset = wl.qset.copy()
    qset[0] = 5
    with pytest.raises(sfc.SfcError) as ei:
        idx.query_sets(dev(wl.queries), dev(wl.delta), dev(qset, torch.int32))
    assert ei.value.status == sfc.SFC_ERR_INVALID


@pytest.mark.parametrize("items", [8, 16, 24])
def test_sets_at_each_tile_size(items):
    """The set passes of the plain sort at several radix tile sizes (pinned
    for the batch's total size): the same per-set CSR as the oracle."""
    wl = workload.batched_uneven(n_sets=24, log2_n=(6, 15), log2_m=(2, 8), curve=MORTON,
                                 seed=40 + items)
    n = len(wl.points)
    sfc.tune_pin(sfc.TUNE_SORT_ITEMS, n, items)
    try:
        check_sets(wl, MORTON, refine=True).close()
    finally:
        sfc.tune_pin(sfc.TUNE_SORT_ITEMS, n, -1)


@pytest.mark.parametrize("n_sets,log2_m", [(40, (8, 11)), (300, (6, 9))])
def test_large_batches_over_sets(n_sets, log2_m):
    """Batches of 2^14 queries and more over point sets (past 256 sets too:
    two passes over the set index in the build), with radii up to those of
    the smallest sets (compared on coarser cells): the per-set CSR is the
    oracle's."""
    wl = workload.batched_uneven(n_sets=n_sets, log2_n=(4, 12), log2_m=log2_m, curve=HILBERT,
                                 seed=60 + n_sets)
    assert len(wl.queries) >= 1 << 14
    check_sets(wl, HILBERT, refine=True).close()

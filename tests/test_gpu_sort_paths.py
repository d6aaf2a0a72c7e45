"""The construction's two sorts give the oracle's arrays bit for bit.

Builds without point sets first order the keys by their top 32 bits (four
radix passes) and sort each chunk of whole runs of equal top bits in LDS
(by counting within runs of at most 64 keys, else by radix passes over the
chunk); a run too long for a chunk makes the build fall back to the plain
eight-pass radix sort.  Checked here: sizes around the chunk stride (2048)
and capacity (4096), every curve, runs of equal top bits on both sides of
64, up to the length that always fits (2048) and beyond it (the fallback),
duplicates, and the two sorts against each other."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
M3 = sfc.MORTON3


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def expected(pts, curve):
    if curve == M3:
        k, i, s = oracle.build3(pts)
        q = np.floor(s * 2.0 ** 21).astype(np.uint64)
        cells = q[:, 0] | (q[:, 1] << np.uint64(21)) | (q[:, 2] << np.uint64(42))
    else:
        k, i, s = oracle.build(pts, curve)
        ux, uy = oracle.quantize(s)
        cells = ux.astype(np.uint64) | (uy.astype(np.uint64) << np.uint64(32))
    return k, i, cells


def check(pts, curve, fallback=None):
    idx = sfc.Index(dev(pts), curve=curve)
    fell = sfc.debug_sort_path(-1)
    cells = idx.cells().cpu().numpy().view(np.uint64)
    keys, ids, _ = idx.sorted_arrays()
    k, i, c = expected(pts, curve)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), k)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), i)
    assert np.array_equal(cells, c)
    if fallback is not None:
        assert fell == fallback
    idx.close()


def cell_run(rng, count, dim, level=None):
    """count points inside one quadtree (octree) cell of side 2^-level: their
    keys share the top 2 * level (3 * level - 1) bits, at least 32 by
    default."""
    if level is None:
        level = 11 if dim == 3 else 16
    corner = rng.integers(0, 2 ** level, dim) / 2 ** level
    return corner + rng.random((count, dim)) * 2.0 ** -level


@pytest.mark.parametrize("curve", [MORTON, HILBERT, M3])
@pytest.mark.parametrize("n", [1, 2, 3, 2047, 2048, 2049, 4095, 4096, 4097, 12289, 250_001])
def test_sizes(curve, n):
    rng = np.random.default_rng(n * 3 + curve)
    pts = rng.random((n, 3 if curve == M3 else 2))
    check(pts, curve, fallback=0)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_clustered_mixture(curve):
    mix = workload.make_mixture(11, k=8, sigma=0.002, frac=0.9)
    pts = workload.clustered_points(1 << 20, 12, mix)
    check(pts, curve, fallback=0)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
@pytest.mark.parametrize("run", [1, 2, 64, 65, 700, 2048])
def test_runs_that_always_fit(curve, run):
    """Runs of equal top 32 bits no longer than capacity - stride always fit,
    wherever they fall relative to the chunk stride; runs of up to 64 keys
    are ranked by counting, longer ones send their chunk to radix passes."""
    rng = np.random.default_rng(run + 17 * curve)
    parts = [rng.random((30_000, 2))]
    for _ in range(12):
        parts.append(cell_run(rng, run, 2))
    pts = np.concatenate(parts)
    pts = pts[rng.permutation(len(pts))]
    check(pts, curve, fallback=0)


@pytest.mark.parametrize("curve", [MORTON, HILBERT, M3])
def test_long_runs_fall_back(curve):
    """A run of 10^4 equal top bits (a tight cluster, and exact duplicates)
    cannot fit a chunk: the build falls back to the plain sort, same arrays."""
    rng = np.random.default_rng(5 + curve)
    dim = 3 if curve == M3 else 2
    pts = np.concatenate([rng.random((50_000, dim)), cell_run(rng, 10_000, dim),
                          np.tile(rng.random((1, dim)), (9_000, 1))])
    pts = pts[rng.permutation(len(pts))]
    check(pts, curve, fallback=1)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_runs_past_the_guarantee(curve):
    """Runs between 2048 and 4096 keys fit or not depending on where chunks
    start: either way the arrays are the oracle's."""
    rng = np.random.default_rng(99 + curve)
    pts = np.concatenate([rng.random((40_000, 2))] +
                         [cell_run(rng, s, 2) for s in (2100, 3000, 3500, 4000, 4096, 2600)])
    pts = pts[rng.permutation(len(pts))]
    check(pts, curve)


def test_plain_and_chunked_agree():
    rng = np.random.default_rng(3)
    mix = workload.make_mixture(4, k=32, sigma=0.004, frac=0.7)
    pts = dev(workload.clustered_points(700_001, 5, mix))
    out = []
    try:
        for force in (1, 0):
            sfc.debug_sort_path(force)
            idx = sfc.Index(pts, curve=HILBERT)
            keys, ids, xy = idx.sorted_arrays()
            out.append((keys.cpu(), ids.cpu(), xy.cpu(), idx.cells().cpu()))
            idx.close()
    finally:
        sfc.debug_sort_path(0)
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("items", [8, 12, 16, 20, 24])
def test_tile_sizes(items):
    """Every radix tile size (pinned for the build's size, as the autotuner
    records one) gives the oracle's arrays through both sorts; 250 001 points
    leave a ragged last tile at each size (tiles of 256 x items keys)."""
    n = 250_001
    mix = workload.make_mixture(items, k=8, sigma=0.003, frac=0.8)
    pts = workload.clustered_points(n, items + 1, mix)
    sfc.tune_pin(sfc.TUNE_SORT_ITEMS, n, items)
    try:
        for force in (0, 1):
            sfc.debug_sort_path(force)
            check(pts, HILBERT)
    finally:
        sfc.debug_sort_path(0)
        sfc.tune_pin(sfc.TUNE_SORT_ITEMS, n, -1)


def test_tune_pin_rejects_unknown_shapes():
    for what, value in ((sfc.TUNE_SORT_ITEMS, 10), (sfc.TUNE_SORT_ITEMS, 32),
                        (sfc.TUNE_TEST_SHAPE, 5), (7, 0)):
        with pytest.raises(sfc.SfcError):
            sfc.tune_pin(what, 1000, value)


def expected_sets(pts, curve, set_off):
    """The oracle's sorted arrays set by set (ids are input positions)."""
    ks, ids, xs = [], [], []
    for s in range(len(set_off) - 1):
        a, b = int(set_off[s]), int(set_off[s + 1])
        if b == a:
            continue
        k, i, x = oracle.build(pts[a:b], curve)
        ks.append(k)
        ids.append(i.astype(np.uint64) + a)
        xs.append(x)
    return np.concatenate(ks), np.concatenate(ids).astype(np.uint32), np.concatenate(xs)


def sets_with_long_run(seed, n=60_000, run=9_000):
    """n uniform points in three sets, and the same with the first run points
    moved into one cell of side 2^-16 (keys with equal top 32 bits: a run too
    long for a chunk) inside the first set."""
    rng = np.random.default_rng(seed)
    fit = rng.random((n, 2))
    long_run = fit.copy()
    long_run[:run] = cell_run(rng, run, 2)
    return fit, long_run, np.array([0, 20_000, 45_000, n], np.uint64)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_sets_chunked_and_fallback(curve):
    """Point sets take the chunked sort followed by a pass over the set index;
    a run too long for a chunk sends the build to the plain sort with the
    sets.  Both give the oracle's arrays set by set."""
    fit, long_run, set_off = sets_with_long_run(31 + curve)
    for pts, fell in ((fit, 0), (long_run, 1)):
        idx = sfc.Index(dev(pts), curve=curve, set_off=set_off)
        assert sfc.debug_sort_path(-1) == fell
        keys, ids, xy = idx.sorted_arrays()
        k, i, x = expected_sets(pts, curve, set_off)
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), k)
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), i)
        assert np.array_equal(xy.cpu().numpy(), x)
        idx.close()


@pytest.mark.parametrize("sets", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_recorded_build_falls_back_on_the_device(curve, sets):
    """A recorded build holds the chunked sort and, behind it, the plain one,
    whose kernels do nothing unless a run was too long for a chunk.  Replays
    on points that fit and on points that do not, written into the same
    buffer between replays, all give the oracle's arrays."""
    fit, long_run, set_off = sets_with_long_run(41 + curve)
    if not sets:
        set_off = np.array([0, len(fit)], np.uint64)
    pts = dev(fit)
    idx = sfc.Index(pts, curve, set_off=set_off if sets else None)
    gb = sfc.Graph.build(idx, pts)
    for rep, data in enumerate((long_run, fit, long_run, fit)):
        pts.copy_(dev(data))
        gb.launch()
        gb.wait()
        keys, ids, xy = idx.sorted_arrays()
        k, i, x = expected_sets(data, curve, set_off)
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), k), rep
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), i), rep
        assert np.array_equal(xy.cpu().numpy(), x), rep
    gb.close()
    idx.close()

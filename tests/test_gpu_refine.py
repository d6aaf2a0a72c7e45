"""The refined ranges report exactly the method's results.

Crowded cells (more than 64 points) are split two levels down and their
sub-cells kept when they meet the widened box and, for the Euclidean metric,
the disc (with a relative margin of 2^-40 on the squared distance).  Checked
against the oracle with every cell crowded: a dense background plus points
within a few units in the last place of each query's circle (or square), at
radii from a few quanta to a large part of the square, queries on the
domain's edges and corners, and against the unrefined search."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, L2, LINF, MORTON
from paper_2508_19891_amd import sfc
from test_gpu_cells import boundary_points

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def run(pts, qs, ds, curve, metric, refine):
    idx = sfc.Index(dev(pts), curve, refine=refine, metric=metric)
    off, ids = idx.query(dev(qs), dev(ds))
    idx.close()
    return off.cpu().numpy().view(np.uint64), ids.cpu().numpy().view(np.uint32)


def expect(pts, qs, ds, curve, metric):
    index = oracle.build(pts, curve)
    return oracle.query(index, qs, ds, curve, nthreads=8, metric=metric)


@pytest.mark.parametrize("metric", [L2, LINF])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_crowded_cells_boundary_band(curve, metric):
    rng = np.random.default_rng(40 + 2 * curve + metric)
    qs = rng.uniform(0.02, 0.98, (300, 2))
    ds = np.exp(rng.uniform(np.log(2e-4), np.log(3e-2), 300))
    band = boundary_points(rng, qs, ds, per=40, metric=metric)
    pts = np.concatenate([rng.random((250_000, 2)), band])
    pts = pts[rng.permutation(len(pts))]
    want = expect(pts, qs, ds, curve, metric)
    got = run(pts, qs, ds, curve, metric, refine=True)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    plain = run(pts, qs, ds, curve, metric, refine=False)
    assert np.array_equal(plain[0], got[0]) and np.array_equal(plain[1], got[1])


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_edges_corners_and_radii(curve):
    """Queries on the border and corners of the square, radii from a few
    grid quanta (cells of level 1 and 2 split one level) to 0.4, in a cluster
    dense enough that tiny cells are crowded."""
    rng = np.random.default_rng(7 + curve)
    dense = 0.5 + rng.random((60_000, 2)) * 2.0 ** -26   # ~15 points per grid quantum
    corners = np.array([[0.0, 0.0], [0.0, 1 - 2.0 ** -53], [1 - 2.0 ** -53, 0.0],
                        [1 - 2.0 ** -53, 1 - 2.0 ** -53]])
    pts = np.concatenate([rng.random((150_000, 2)), dense, corners,
                          rng.random((20_000, 2)) * [1, 2.0 ** -10]])
    qs = np.concatenate([corners, [[0.5, 0.5]] * 6, rng.uniform(0.5, 0.5 + 2.0 ** -26, (20, 2)),
                         rng.uniform(0, 1, (40, 2)) * [1, 0.0], rng.uniform(0, 1, (40, 2))])
    ds = np.concatenate([[0.01, 0.05, 0.2, 0.4], 2.0 ** -np.arange(30, 24, -1),
                         rng.uniform(1, 6, 20) * 2.0 ** -32, rng.uniform(1e-4, 1e-2, 40),
                         rng.uniform(1e-4, 0.1, 40)])
    want = expect(pts, qs, ds, curve, L2)
    got = run(pts, qs, ds, curve, L2, refine=True)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_tiny_radii_keep_every_sub_cell(curve):
    """Radii around 2^-400 (below it the disc test keeps every sub-cell) with
    duplicates of the query point, so that crowded cells of the lowest levels
    are split."""
    rng = np.random.default_rng(3 + curve)
    q = rng.uniform(0.2, 0.8, (8, 2))
    pts = np.concatenate([np.repeat(q, 100, axis=0), rng.random((50_000, 2))])
    ds = np.array([0.0, 2.0 ** -401, 2.0 ** -400, 2.0 ** -399, 1e-300, 2.0 ** -40, 2.0 ** -33,
                   2.0 ** -31])
    want = expect(pts, q, ds, curve, L2)
    got = run(pts, q, ds, curve, L2, refine=True)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


@pytest.mark.parametrize("metric", [L2, LINF])
def test_three_dimensions_crowded_boundary_band(metric):
    """Crowded cubes split into runs of the children that meet the box:
    points within a few units in the last place of the sphere (or the cube
    window) around each query, in a dense background, refined or not."""
    rng = np.random.default_rng(60 + metric)
    qs = rng.uniform(0.05, 0.95, (200, 3))
    ds = np.exp(rng.uniform(np.log(3e-3), np.log(5e-2), 200))
    band = []
    for q, d in zip(qs, ds):
        for _ in range(30):
            k = rng.integers(-6, 7)
            if metric == L2:
                v = rng.normal(size=3)
                v /= np.linalg.norm(v)
            else:
                v = rng.uniform(-1, 1, 3)
                v[rng.integers(3)] = rng.choice([-1.0, 1.0])
            p = q + d * (1 + k * 2.0 ** -52) * v
            if np.all(p >= 0) and np.all(p < 1):
                band.append(p)
    pts = np.concatenate([rng.random((300_000, 3)), np.array(band)])
    pts = pts[rng.permutation(len(pts))]
    index = oracle.build3(pts)
    want = oracle.query3(index, qs, ds, nthreads=8, metric=metric)
    for refine in (True, False):
        idx = sfc.Index(dev(pts), sfc.MORTON3, refine=refine, metric=metric)
        off, ids = idx.query(dev(qs), dev(ds))
        idx.close()
        assert np.array_equal(off.cpu().numpy().view(np.uint64), want[0])
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1])


TOP = 1 - 2.0 ** -53


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_far_corner_last_cell(curve):
    """Queries at and just past the square's far corner with tiny radii: their
    widened boxes clamp to the single last grid cell (2^32 - 1, 2^32 - 1),
    whose cell loop must stop there; every search, refined or not, with early
    termination and square windows."""
    rng = np.random.default_rng(70 + curve)
    pts = np.concatenate([rng.random((5000, 2)),
                          [[TOP, TOP]] * 3 + [[TOP, 0.5], [0.5, TOP], [TOP, TOP - 2.0 ** -40]]])
    qs = np.array([[1.0, 1.0], [1.0, 1.0], [1.0, 1.0], [1.0 + 2.0 ** -33, 1.0], [1.0, TOP],
                   [TOP, 1.0], [1.5, 1.5], [1.0, 0.5], [0.3, 0.6]])
    ds = np.array([0.0, 2.0 ** -40, 2.0 ** -30, 2.0 ** -35, 2.0 ** -45, 0.0, 0.1, 1e-12, 0.01])
    for metric in (L2, LINF):
        want = expect(pts, qs, ds, curve, metric)
        combos = [dict(refine=rf, early_term=et) for rf in (False, True) for et in (False, True)]
        combos += [dict(refine=True, search=sfc.LEARNED), dict(refine=True, search=sfc.STREE)]
        for kw in combos:
            idx = sfc.Index(dev(pts), curve, metric=metric, **kw)
            off, ids = idx.query(dev(qs), dev(ds))
            idx.close()
            assert np.array_equal(off.cpu().numpy().view(np.uint64), want[0]), kw
            assert np.array_equal(ids.cpu().numpy().view(np.uint32), want[1]), kw

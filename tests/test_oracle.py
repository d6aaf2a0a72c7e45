"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here touches a GPU or the HIP library.  Each test checks the oracle
against something other than itself: values worked by hand from the
definitions, a textbook routine written in a different form, invariants the
definitions imply (Def. 1 contiguity, Def. 3 prefix property, the Observation,
the bound of at most four cells), brute force on small inputs, and a closed
form for the expected output size.
"""
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import workload

M32 = (1 << 32) - 1


# ---- Z-order keys (Alg. 2) ----------------------------------------------------

# Hand-worked from Alg. 2: bit i of x -> key bit 2i, bit i of y -> key bit 2i+1.
MORTON_HAND = [
    ((0, 0), 0x0),
    ((1, 0), 0x1),
    ((0, 1), 0x2),
    ((3, 5), 0x27),              # x=011, y=101 -> y2 x2 y1 x1 y0 x0 = 1 0 0 1 1 1
    ((M32, 0), 0x5555555555555555),
    ((0, M32), 0xAAAAAAAAAAAAAAAA),
    ((M32, M32), 0xFFFFFFFFFFFFFFFF),
    ((1 << 31, 0), 1 << 62),
    ((0, 1 << 31), 1 << 63),
    ((1 << 31, 1 << 31), 3 << 62),
]


@pytest.mark.parametrize("xy,key", MORTON_HAND)
def test_morton_hand_worked(xy, key):
    assert oracle.morton(*xy) == key


def test_morton_each_bit_position():
    # A dropped, shifted or transposed bit fails one of these.
    for i in range(32):
        assert oracle.morton(1 << i, 0) == 1 << (2 * i)
        assert oracle.morton(0, 1 << i) == 1 << (2 * i + 1)
    rng = np.random.default_rng(7)
    for x, y in rng.integers(0, 1 << 32, (200, 2), dtype=np.uint64):
        x, y = int(x), int(y)
        assert oracle.morton(x, y) == oracle.morton(x, 0) | oracle.morton(0, y)


def _golden_corner():
    """The 4x4 corner's labels, worked by hand (tests/golden, with the
    derivation and citations in the file's header)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "corner_4x4_labels.txt")
    tables, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.isalpha():
            cur = tables.setdefault(line, [])
        else:
            cur.append([int(v) for v in line.split()])
    return tables


_CORNER = _golden_corner()
MORTON_4x4 = _CORNER["morton"]
HILBERT_4x4 = _CORNER["hilbert"]


@pytest.mark.parametrize("curve,table", [(MORTON, MORTON_4x4), (HILBERT, HILBERT_4x4)])
def test_corner_4x4(curve, table):
    for row, y in zip(table, (3, 2, 1, 0)):
        for x in range(4):
            assert oracle.key(curve, x, y) == row[x]


# ---- Hilbert keys ------------------------------------------------------------------


def textbook_hilbert(bits: int, x: int, y: int) -> int:
    """Hilbert index by quadrant rotation (the classic textbook xy-to-d
    routine): at each level add the quadrant's rank times the quadrant area,
    then rotate/reflect the coordinates into the quadrant's frame."""
    n = 1 << bits
    d = 0
    s = n >> 1
    while s > 0:
        rx = 1 if x & s else 0
        ry = 1 if y & s else 0
        d += s * s * ((3 * rx) ^ ry)
        if ry == 0:
            if rx == 1:
                x = n - 1 - x
                y = n - 1 - y
            x, y = y, x
        s >>= 1
    return d


def test_hilbert_matches_textbook_exhaustive_corner():
    for x in range(64):
        for y in range(64):
            assert oracle.hilbert(x, y) == textbook_hilbert(32, x, y)


def test_hilbert_matches_textbook_random():
    rng = np.random.default_rng(11)
    for x, y in rng.integers(0, 1 << 32, (500, 2), dtype=np.uint64):
        x, y = int(x), int(y)
        assert oracle.hilbert(x, y) == textbook_hilbert(32, x, y)


def test_hilbert_endpoints():
    assert oracle.hilbert(0, 0) == 0
    assert oracle.hilbert(M32, 0) == (1 << 64) - 1     # the curve ends at (2^32-1, 0)
    assert oracle.hilbert(1, 0) == 1
    assert oracle.hilbert(0, 1) == 3


@pytest.mark.parametrize("origin", [(0, 0), (1 << 31, 1 << 31), (0x12345640, 0x9ABCDEC0)])
def test_hilbert_consecutive_keys_are_neighbours(origin):
    # Inside an aligned 64x64 block the keys are 4096 consecutive integers and
    # the walk in key order moves by one grid step each time.
    ox, oy = origin
    pts = {}
    for x in range(64):
        for y in range(64):
            pts[oracle.hilbert(ox + x, oy + y)] = (x, y)
    ks = sorted(pts)
    assert ks[-1] - ks[0] == 4095 and len(ks) == 4096
    for a, b in zip(ks, ks[1:]):
        (x0, y0), (x1, y1) = pts[a], pts[b]
        assert abs(x0 - x1) + abs(y0 - y1) == 1


# ---- RSFC properties (Def. 1, Def. 3, Lemma 1) --------------------------------------


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_rsfc_blocks_are_contiguous_intervals(curve):
    # Def. 1: each aligned 2^l x 2^l square is one contiguous run of the order.
    keys = np.array([[oracle.key(curve, x, y) for y in range(32)] for x in range(32)],
                    dtype=np.uint64)
    for lvl in range(6):
        side = 1 << lvl
        for bx in range(0, 32, side):
            for by in range(0, 32, side):
                blk = keys[bx:bx + side, by:by + side].ravel()
                lo = int(blk.min())
                assert lo % (side * side) == 0
                assert sorted(int(v) for v in blk) == list(range(lo, lo + side * side))


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_prefix_property(curve):
    # Def. 3: the label of a level-l cell is a prefix of the labels inside it.
    rng = np.random.default_rng(5 + curve)
    for x, y in rng.integers(0, 1 << 32, (300, 2), dtype=np.uint64):
        x, y = int(x), int(y)
        k = oracle.key(curve, x, y)
        for lvl in range(0, 33, 3):
            mask = (1 << lvl) - 1
            kc = oracle.key(curve, x & ~mask & M32, y & ~mask & M32)
            assert k >> (2 * lvl) == kc >> (2 * lvl)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_bijective_on_corner(curve):
    ks = {oracle.key(curve, x, y) for x in range(128) for y in range(128)}
    assert ks == set(range(128 * 128))


# ---- quantisation --------------------------------------------------------------------------


def test_quantize_values():
    xy = np.array([[0.0, 0.5], [2.0 ** -32, np.nextafter(2.0 ** -32, 0)],
                   [workload.ONE_BELOW, 0.25], [-0.0, 0.75]])
    ux, uy = oracle.quantize(xy)
    assert list(ux) == [0, 1, M32, 0]
    assert list(uy) == [1 << 31, 0, 1 << 30, 3 << 30]


@pytest.mark.parametrize("bad", [1.0, -1e-300, float("nan"), float("inf"), 2.0])
def test_quantize_domain(bad):
    with pytest.raises(oracle.DomainError):
        oracle.keys(np.array([[0.5, 0.5], [bad, 0.1]]), MORTON)


# ---- sort (textbook: lexicographic order of (key, id)) --------------------------------------


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_build_is_lexicographic_sort(curve):
    rng = np.random.default_rng(3)
    pts = rng.random((3000, 2))
    pts[1000:1500] = pts[0:500]                       # exact duplicates
    pts[1500:1600] = np.floor(pts[1500:1600] * 2 ** 32) / 2 ** 32 + 2.0 ** -40   # same cell
    pts[1600:1700] = np.floor(pts[1500:1600] * 2 ** 32) / 2 ** 32
    k, i, s = oracle.build(pts, curve)
    raw = oracle.keys(pts, curve)
    order = np.lexsort((np.arange(len(pts)), raw))    # numpy's stable sort by key, then id
    assert np.array_equal(k, raw[order])
    assert np.array_equal(i, order.astype(np.uint32))
    assert np.array_equal(s, pts[order])


# ---- query box ---------------------------------------------------------------------------


def test_box_hand_values():
    h = 1 << 31
    assert oracle.box(0.5, 0.5, 0.0) == (h - 1, h + 1, h - 1, h + 1)
    # delta = 2^-4 around 0.5: [0.4375, 0.5625] * 2^32, widened by one quantum.
    assert oracle.box(0.5, 0.25, 2.0 ** -4) == (
        7 * 2 ** 28 - 1, 9 * 2 ** 28 + 1, 3 * 2 ** 28 - 1, 5 * 2 ** 28 + 1)
    assert oracle.box(0.0, 0.0, 0.0) == (0, 1, 0, 1)                  # clamped at 0
    assert oracle.box(5.0, 0.5, 1.0) is None                          # misses the domain
    assert oracle.box(-3.0, 0.5, 10.0) == (0, M32, 0, M32)
    # Far query, huge radius: w = 1 + floor((|qx| + delta) 2^-19) = 129 quanta
    # on the x axis; qx - delta = 1/2 + 2^-27 exactly.
    qx = 2.0 ** 25 + 0.5 + 2.0 ** -27
    assert oracle.box(qx, 0.5, 2.0 ** 25)[0] == 2 ** 31 + 32 - 129


@pytest.mark.parametrize("bad", [(0.5, 0.5, -1e-9), (0.5, 0.5, float("nan")),
                                 (float("inf"), 0.5, 0.1), (0.5, 0.5, float("inf"))])
def test_invalid_queries(bad):
    with pytest.raises(oracle.InvalidQuery):
        oracle.box(*bad)


# ---- cells(Q) and its key ranges ---------------------------------------------------------------

WORKED_BOXES = [
    # (box, Morton ranges, Hilbert ranges), hand-worked from the 4x4/8x8 grids.
    ((3, 4, 3, 4), [(12, 15), (24, 27), (36, 39), (48, 51)], [(8, 11), (28, 35), (52, 55)]),
    ((5, 6, 5, 6), [(48, 63)], [(32, 47)]),
    ((1, 2, 1, 2), [(0, 15)], [(0, 15)]),
    ((7, 7, 0, 0), [(21, 21)], [(21, 21)]),
]


@pytest.mark.parametrize("b,mr,hr", WORKED_BOXES)
def test_box_ranges_worked(b, mr, hr):
    assert oracle.box_ranges(*b, MORTON) == mr
    assert oracle.box_ranges(*b, HILBERT) == hr


def _inverse_corner(curve, side=32):
    inv = {}
    for x in range(side):
        for y in range(side):
            inv[oracle.key(curve, x, y)] = (x, y)
    return inv


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_box_ranges_exhaustive_small(curve):
    """Every box in [0,16)^2: at most four ranges (P covered by <= 2^d cells),
    sorted, disjoint and merged; together they are exactly the level-l cells
    that meet the box, with l = ceil(log2 side) so that side <= 2^l < 2 side;
    every integer point of the box lies in them (Observation)."""
    inv = _inverse_corner(curve)
    for lx in range(16):
        for hx in range(lx, 16):
            for ly in range(16):
                for hy in range(ly, 16):
                    rs = oracle.box_ranges(lx, hx, ly, hy, curve)
                    assert 1 <= len(rs) <= 4
                    for (a, b), (c, _) in zip(rs, rs[1:]):
                        assert b + 1 < c
                    side = max(hx - lx + 1, hy - ly + 1)
                    lvl = max(0, math.ceil(math.log2(side)))
                    assert side <= 1 << lvl < 2 * side or side == 1
                    cells = {(x >> lvl, y >> lvl) for x in range(lx, hx + 1)
                             for y in range(ly, hy + 1)}
                    covered = set()
                    for a, b in rs:
                        covered.update(inv[k] for k in range(a, b + 1))
                    want = {(cx * (1 << lvl) + i, cy * (1 << lvl) + j)
                            for cx, cy in cells for i in range(1 << lvl) for j in range(1 << lvl)}
                    assert covered == want


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_box_ranges_whole_domain(curve):
    assert oracle.box_ranges(0, M32, 0, M32, curve) == [(0, (1 << 64) - 1)]
    assert oracle.box_ranges(0, 1 << 31, 5, 6, curve) == [(0, (1 << 64) - 1)]


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_ranges_contain_query_cell_keys(curve):
    # Any point inside the (widened) box has its key inside some range.
    rng = np.random.default_rng(17 + curve)
    for _ in range(300):
        q = rng.random(2)
        d = 10 ** rng.uniform(-9, -0.5)
        rs = oracle.ranges(q[0], q[1], d, curve)
        assert 1 <= len(rs) <= 4
        b = oracle.box(q[0], q[1], d)
        for _ in range(20):
            x = int(rng.integers(b[0], b[1] + 1))
            y = int(rng.integers(b[2], b[3] + 1))
            k = oracle.key(curve, x, y)
            assert any(a <= k <= c for a, c in rs)


# ---- result sets vs brute force --------------------------------------------------------------


def _adversarial(rng, n=1500):
    """Points and queries built to hit the edge cases of the rounding and the
    box: duplicates, border points, points one ulp inside and outside the
    circle, points on and one ulp below a quantum edge."""
    pts = list(rng.random((n // 3, 2)))
    qs, ds = [], []
    for _ in range(60):
        q = rng.random(2)
        d = 10 ** rng.uniform(-8, -1)
        qs.append(q)
        ds.append(d)
        for ang in rng.uniform(0, 2 * np.pi, 6):
            p = q + d * np.array([np.cos(ang), np.sin(ang)])
            for t in (p, np.nextafter(p, q), np.nextafter(p, 2 * p - q)):
                if np.all(t >= 0) and np.all(t < 1):
                    pts.append(t)
        for sx in (-1, 1):
            e = np.floor((q[0] + sx * d) * 2 ** 32) / 2 ** 32
            for ex in (e, np.nextafter(e, 0), np.nextafter(e, 1)):
                p = np.array([ex, q[1]])
                if np.all(p >= 0) and np.all(p < 1):
                    pts.append(p)
    pts += [np.array([0.0, 0.0]), np.array([workload.ONE_BELOW, workload.ONE_BELOW]),
            np.array([0.0, workload.ONE_BELOW])]
    pts = np.array(pts)
    pts = np.concatenate([pts, pts[:200]])            # duplicates
    qs += [np.array([0.5, 0.5]), pts[5], pts[7], np.array([-0.2, 0.5]),
           np.array([1.3, 1.3]), np.array([0.3, 0.9])]
    ds += [2.0, 0.0, 0.0, 0.25, 0.5, 1e-300]
    qs = np.array(qs)
    return pts, qs, np.array(ds)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_query_equals_brute_force_adversarial(curve):
    rng = np.random.default_rng(23 + curve)
    pts, qs, ds = _adversarial(rng)
    idx = oracle.build(pts, curve)
    got = oracle.query(idx, qs, ds, curve)
    ref = oracle.brute(pts, qs, ds)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))
    assert ref[1].size > 0
    # delta = 0 reports the coincident points only; delta >= sqrt(2) reports all.
    offs = ref[0]
    j = len(qs) - 6
    assert offs[j + 1] - offs[j] == len(pts)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_query_output_in_curve_order(curve):
    rng = np.random.default_rng(29)
    pts = rng.random((4000, 2))
    qs = rng.random((100, 2))
    ds = np.full(100, 0.05)
    k, i, s = oracle.build(pts, curve)
    off, ids = oracle.query((k, i, s), qs, ds, curve)
    rank = np.empty(len(pts), np.int64)
    rank[i] = np.arange(len(pts))
    for j in range(100):
        r = rank[ids[off[j]:off[j + 1]]]
        assert np.all(np.diff(r) > 0)


def test_query_threads_same_output():
    rng = np.random.default_rng(31)
    pts = rng.random((5000, 2))
    qs = rng.random((301, 2))
    ds = 10 ** rng.uniform(-3, -1, 301)
    idx = oracle.build(pts, HILBERT)
    a = oracle.query(idx, qs, ds, HILBERT, nthreads=1)
    b = oracle.query(idx, qs, ds, HILBERT, nthreads=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 2 ** 31), n=st.integers(0, 300), m=st.integers(0, 40),
       curve=st.sampled_from([MORTON, HILBERT]), scale=st.floats(-7, 0.3))
def test_query_equals_brute_force_random(seed, n, m, curve, scale):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    if n > 10:
        pts[n // 2:] = pts[: n - n // 2]      # duplicates
    qs = rng.uniform(-0.1, 1.1, (m, 2))
    ds = 10 ** (scale + rng.uniform(-1, 1, m))
    idx = oracle.build(pts, curve)
    got = oracle.query(idx, qs, ds, curve)
    ref = oracle.brute(pts, qs, ds)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))


def test_expected_output_closed_form():
    """Uniform points and queries in the unit square: the chance that a point
    lies within delta of a query is pi d^2 - 8 d^3/3 + d^4/2 (the distance CDF
    of two uniform points, d <= 1).  For n = 2^16 and delta = sqrt(10/(pi n))
    that is 9.941 reports per query."""
    wl = workload.uniform_fixed_radius(n=1 << 16, m=10_000, curve=MORTON)
    d = wl.delta[0]
    n = wl.points.shape[0]
    expect = n * (math.pi * d ** 2 - 8 * d ** 3 / 3 + d ** 4 / 2)
    assert abs(expect - 9.941) < 1e-3
    idx = oracle.build(wl.points, MORTON)
    off, _ = oracle.query(idx, wl.queries, wl.delta, MORTON, nthreads=4)
    mean = off[-1] / 10_000
    assert abs(mean - expect) < 0.25


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_closed_ball_exact_distances(curve):
    """The ball is closed: points at exactly distance delta are reported.  The
    points are dyadic and form 3-4-5 triangles with the query, so every
    operation of the test is exact and the expected set is known by hand."""
    q = (0.5, 0.5)
    a = 1.0 / 32
    on = [(0.5 + 3 * a, 0.5 + 4 * a), (0.5 - 4 * a, 0.5 + 3 * a), (0.5, 0.5 - 5 * a),
          (0.5 + 5 * a, 0.5)]                                    # |p - q| = 5a exactly
    inside = [(0.5 + 3 * a, 0.5 + 3 * a), (0.5, 0.5)]             # strictly inside
    outside = [(0.5 + 4 * a, 0.5 + 4 * a), (0.5 + 5 * a + 2.0 ** -40, 0.5)]
    pts = np.array(on + inside + outside)
    idx = oracle.build(pts, curve)
    off, ids = oracle.query(idx, np.array([q, q]), np.array([5 * a, 0.0]), curve)
    assert sorted(ids[off[0]:off[1]].tolist()) == [0, 1, 2, 3, 4, 5]
    assert ids[off[1]:off[2]].tolist() == [5]                     # delta = 0: coincident only


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_far_query_large_radius_widening(curve):
    """A query far outside the square with a huge radius: the rounded test
    accepts points several quanta beyond the exact box edge (dx rounds to the
    spacing of doubles near 2^25), so the box must widen with |q| + delta.
    For q = (2^25 + 1/2, 1/2), delta = 2^25, the points (1/2 - k 2^-32, 1/2)
    are accepted exactly for k <= 16: doubles near 2^25 are 2^-27 = 32 quanta
    apart, so dx rounds to -2^25 up to the tie at k = 16."""
    k = np.arange(0, 24)
    pts = np.stack([0.5 - k * 2.0 ** -32, np.full(k.shape, 0.5)], 1)
    q = np.array([[2.0 ** 25 + 0.5, 0.5]])
    d = np.array([2.0 ** 25])
    ref = oracle.brute(pts, q, d)
    assert ref[1].tolist() == list(range(17))
    got = oracle.query(oracle.build(pts, curve), q, d, curve)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))


TOP = 1 - 2.0 ** -53
# Queries at and just past the far corner of the square: their widened boxes
# clamp to the single last grid cell (2^32 - 1, 2^32 - 1), at level 0.
CORNER_PTS = np.array([[TOP, TOP]] * 3 + [[TOP, 0.5], [0.5, TOP], [TOP, TOP - 2.0 ** -40]])
CORNER_Q = np.array([[1.0, 1.0], [1.0, 1.0], [1.0, 1.0], [1.0 + 2.0 ** -33, 1.0], [1.0, TOP],
                     [TOP, 1.0], [1.5, 1.5], [1.0, 0.5]])
CORNER_D = np.array([0.0, 2.0 ** -40, 2.0 ** -30, 2.0 ** -35, 2.0 ** -45, 0.0, 0.1, 1e-12])


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_far_corner_single_last_cell(curve):
    """The box of a query at (1, 1) with a tiny radius is the last grid cell
    alone; the three copies of (TOP, TOP) lie 2^-52.5 away, inside radii
    2^-40 and 2^-30 and outside 0 and 2^-45."""
    assert oracle.box(1.0, 1.0, 0.0) == (M32, M32, M32, M32)
    assert len(oracle.ranges(1.0, 1.0, 0.0, curve)) == 1
    rng = np.random.default_rng(5 + curve)
    pts = np.concatenate([rng.random((2000, 2)), CORNER_PTS])
    ref = oracle.brute(pts, CORNER_Q, CORNER_D)
    assert np.diff(ref[0].astype(np.int64)).tolist() == [0, 3, 4, 0, 3, 0, 0, 1]
    got = oracle.query(oracle.build(pts, curve), CORNER_Q, CORNER_D, curve)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))


# ---- square windows (the experiments' queries, Sec. 4) ---------------------------------------

LINF = oracle.LINF


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_window_grid_counts_closed_form(curve):
    """Points on the dyadic grid (i h, j h), h = 2^-7: every difference and
    comparison is exact, so the closed window of half side r around a grid
    point (a h, b h) holds exactly the grid points with |i - a| <= k and
    |j - b| <= k for r in [k h, (k+1) h), clipped to the square: the ids
    follow from integer arithmetic alone."""
    g = 128
    h = 1.0 / g
    ii, jj = np.meshgrid(np.arange(g), np.arange(g), indexing="ij")
    pts = np.stack([ii.ravel() * h, jj.ravel() * h], 1)       # id = i * g + j
    idx = oracle.build(pts, curve)
    rng = np.random.default_rng(41)
    cases = [(0, 0, 0), (0, 0, 3), (127, 127, 2), (64, 5, 7), (10, 120, 0)]
    cases += [tuple(int(v) for v in t) for t in zip(rng.integers(0, g, 20),
                                                    rng.integers(0, g, 20),
                                                    rng.integers(0, 12, 20))]
    qs, ds, want = [], [], []
    for a, b, k in cases:
        for r in (k * h, k * h + h / 2):                       # on a grid line, between lines
            qs.append((a * h, b * h))
            ds.append(r)
            xs = [i for i in range(g) if abs(i - a) <= k]
            ys = [j for j in range(g) if abs(j - b) <= k]
            want.append(sorted(i * g + j for i in xs for j in ys))
    off, ids = oracle.query(idx, np.array(qs), np.array(ds), curve, metric=LINF)
    for t, w in enumerate(want):
        assert sorted(ids[off[t]:off[t + 1]].tolist()) == w, cases[t // 2]
    # The count is the product of the clipped side counts.
    a, b, k = 64, 5, 7
    assert len(want[cases.index((a, b, k)) * 2]) == (2 * k + 1) * (b + k + 1)


def test_window_between_ball_and_scaled_ball():
    """Geometry: the ball of radius r lies in the square of half side r,
    which lies in the ball of radius r sqrt 2 (a relative margin of 1e-9
    covers the rounding of either test)."""
    rng = np.random.default_rng(42)
    pts = rng.random((3000, 2))
    qs = rng.random((200, 2))
    ds = 10 ** rng.uniform(-2.5, -0.7, 200)
    ball = oracle.brute(pts, qs, ds)
    win = oracle.brute(pts, qs, ds, metric=LINF)
    big = oracle.brute(pts, qs, ds * math.sqrt(2) * (1 + 1e-9))
    for j in range(200):
        b = set(ball[1][ball[0][j]:ball[0][j + 1]].tolist())
        w = set(win[1][win[0][j]:win[0][j + 1]].tolist())
        g = set(big[1][big[0][j]:big[0][j + 1]].tolist())
        assert b <= w <= g
    assert win[0][-1] > ball[0][-1]


def test_window_expected_output_closed_form():
    """Uniform points; windows of half side r whose centres keep them inside
    the square: a point lies in a window with probability (2r)^2, here 10 / n
    (10 reports per query on average)."""
    n, m = 1 << 16, 10_000
    r = math.sqrt(10.0 / n) / 2
    rng = np.random.default_rng(43)
    pts = rng.random((n, 2))
    qs = rng.uniform(r, 1 - r, (m, 2))
    off, _ = oracle.query(oracle.build(pts, MORTON), qs, np.full(m, r), MORTON, nthreads=4,
                          metric=LINF)
    assert abs(off[-1] / m - 10.0) < 0.25


def _window_adversarial(rng):
    """Points one ulp inside and outside every side and corner of the
    windows, on quantum edges, and duplicates."""
    pts = list(rng.random((400, 2)))
    qs, ds = [], []
    for _ in range(50):
        q = rng.random(2)
        d = 10 ** rng.uniform(-9, -1)
        qs.append(q)
        ds.append(d)
        for sx in (-1, 0, 1):
            for sy in (-1, 0, 1):
                p = q + d * np.array([sx, sy])
                for t in (p, np.nextafter(p, q), np.nextafter(p, 2 * p - q)):
                    if np.all(t >= 0) and np.all(t < 1):
                        pts.append(t)
        for sx in (-1, 1):
            e = np.floor((q[0] + sx * d) * 2 ** 32) / 2 ** 32
            for ex in (e, np.nextafter(e, 0), np.nextafter(e, 1)):
                p = np.array([ex, q[1]])
                if np.all(p >= 0) and np.all(p < 1):
                    pts.append(p)
    pts = np.array(pts)
    pts = np.concatenate([pts, pts[:100]])
    qs += [np.array([0.5, 0.5]), pts[3], np.array([-0.3, 0.5]), np.array([1.2, -0.1])]
    ds += [0.5, 0.0, 0.31, 0.25]
    return pts, np.array(qs), np.array(ds)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_window_query_equals_brute_force_adversarial(curve):
    rng = np.random.default_rng(44 + curve)
    pts, qs, ds = _window_adversarial(rng)
    got = oracle.query(oracle.build(pts, curve), qs, ds, curve, metric=LINF)
    ref = oracle.brute(pts, qs, ds, metric=LINF)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))
    # half side 1/2 around the centre covers the square [0, 1)^2 whole
    j = len(qs) - 4
    assert ref[0][j + 1] - ref[0][j] == len(pts)


@settings(max_examples=30, deadline=None)
@given(seed=st.integers(0, 2 ** 31), n=st.integers(0, 300), m=st.integers(0, 30),
       curve=st.sampled_from([MORTON, HILBERT]), scale=st.floats(-7, 0.3))
def test_window_query_equals_brute_force_random(seed, n, m, curve, scale):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    qs = rng.uniform(-0.1, 1.1, (m, 2))
    ds = 10 ** (scale + rng.uniform(-1, 1, m))
    got = oracle.query(oracle.build(pts, curve), qs, ds, curve, metric=LINF)
    ref = oracle.brute(pts, qs, ds, metric=LINF)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_window_far_query_large_half_side(curve):
    """The widened box under the window test: for q = (2^25 + 1/2, 1/2) and
    half side 2^25 the rounded |dx| <= r accepts (1/2 - k 2^-32, 1/2) exactly
    for k <= 16 (doubles near 2^25 are 32 quanta apart; k = 16 is the tie,
    rounded to even), several quanta past the exact edge."""
    k = np.arange(0, 24)
    pts = np.stack([0.5 - k * 2.0 ** -32, np.full(k.shape, 0.5)], 1)
    q = np.array([[2.0 ** 25 + 0.5, 0.5]])
    d = np.array([2.0 ** 25])
    ref = oracle.brute(pts, q, d, metric=LINF)
    assert ref[1].tolist() == list(range(17))
    got = oracle.query(oracle.build(pts, curve), q, d, curve, metric=LINF)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))


def test_metric_must_be_known():
    with pytest.raises(oracle.InvalidQuery):
        oracle.brute(np.zeros((1, 2)), np.zeros((1, 2)), np.zeros(1), metric=2)

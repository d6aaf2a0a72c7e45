"""Pins of the three-dimensional oracle (d = 3 Morton codes; Sec. 1 and
Sec. 2.1: the Z-order method generalises to R^d).  As for the plane: keys
worked by hand from the bit-interleaving definition, the octree prefix and
contiguity properties on an exhaustive corner, the at-most-2^d-ranges bound
and exact cover, brute force on adversarial inputs, a far query where the
widening matters, and closed forms (ball volume, cube counts on a grid)."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import L2, LINF

M21 = (1 << 21) - 1

# Hand-worked: x bit i -> key bit 3i, y bit i -> 3i+1, z bit i -> 3i+2.
MORTON3_HAND = [
    ((0, 0, 0), 0),
    ((1, 0, 0), 1),
    ((0, 1, 0), 2),
    ((0, 0, 1), 4),
    ((1, 1, 1), 7),
    ((2, 0, 0), 8),
    ((3, 5, 6), 427),             # 011, 101, 110 -> 3 + 40 + 384
    ((M21, 0, 0), int("001" * 21, 2)),
    ((0, 0, M21), int("100" * 21, 2)),
    ((M21, M21, M21), (1 << 63) - 1),
    ((1 << 20, 0, 0), 1 << 60),
]


@pytest.mark.parametrize("xyz,key", MORTON3_HAND)
def test_morton3_hand_worked(xyz, key):
    assert oracle.morton3(*xyz) == key


def test_morton3_each_bit_position():
    for i in range(21):
        assert oracle.morton3(1 << i, 0, 0) == 1 << (3 * i)
        assert oracle.morton3(0, 1 << i, 0) == 1 << (3 * i + 1)
        assert oracle.morton3(0, 0, 1 << i) == 1 << (3 * i + 2)


def test_octree_blocks_are_contiguous():
    """On the 8^3 corner the keys are a permutation of 0..511, and every
    aligned cube of side 2^l holds exactly one aligned run of 8^l keys."""
    g = 8
    keys = np.array([[[oracle.morton3(x, y, z) for z in range(g)] for y in range(g)]
                     for x in range(g)])
    assert sorted(keys.ravel().tolist()) == list(range(g ** 3))
    for lv in range(4):
        s = 1 << lv
        for x0 in range(0, g, s):
            for y0 in range(0, g, s):
                for z0 in range(0, g, s):
                    blk = keys[x0:x0 + s, y0:y0 + s, z0:z0 + s].ravel()
                    lo = blk.min()
                    assert lo % (s ** 3) == 0 and blk.max() == lo + s ** 3 - 1


def test_box_ranges3_cover_exactly():
    """At most 8 ranges; each range is a union of whole level-l cubes that
    meet the box; every grid point of the box lies in a range."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        lo = rng.integers(0, 40, 3)
        hi = lo + rng.integers(0, 12, 3)
        box = [int(v) for pair in zip(lo, hi) for v in pair]
        rs = oracle.box_ranges3(box)
        assert 1 <= len(rs) <= 8
        side = int((hi - lo + 1).max())
        lv = max(0, math.ceil(math.log2(side)))
        for a, b in rs:
            assert a % (8 ** lv) == 0 and (b + 1) % (8 ** lv) == 0
        for _ in range(30):
            p = [int(rng.integers(lo[a], hi[a] + 1)) for a in range(3)]
            k = oracle.morton3(*p)
            assert any(a <= k <= b for a, b in rs)
        # no range holds a cube that misses the box: its corner cubes meet it
        for a, b in rs:
            for start in range(a, b + 1, 8 ** lv):
                c = [0, 0, 0]
                for i in range(21):          # de-interleave the cube's first key
                    for ax in range(3):
                        c[ax] |= ((start >> (3 * i + ax)) & 1) << i
                assert all(c[ax] <= hi[ax] and c[ax] + (1 << lv) - 1 >= lo[ax]
                           for ax in range(3))


def test_whole_domain_is_one_range():
    assert oracle.ranges3([0.5, 0.5, 0.5], 2.0) == [(0, (1 << 63) - 1)]


def _adversarial3(rng, n=900):
    pts = list(rng.random((n // 3, 3)))
    qs, ds = [], []
    for _ in range(40):
        q = rng.random(3)
        d = 10 ** rng.uniform(-7, -1)
        qs.append(q)
        ds.append(d)
        for _ in range(5):
            v = rng.standard_normal(3)
            p = q + d * v / np.linalg.norm(v)
            for t in (p, np.nextafter(p, q), np.nextafter(p, 2 * p - q)):
                if np.all(t >= 0) and np.all(t < 1):
                    pts.append(t)
        e = np.floor((q[0] - d) * 2 ** 21) / 2 ** 21
        for ex in (e, np.nextafter(e, 0), np.nextafter(e, 1)):
            p = np.array([ex, q[1], q[2]])
            if np.all(p >= 0) and np.all(p < 1):
                pts.append(p)
    pts = np.array(pts)
    pts = np.concatenate([pts, pts[:100]])
    qs += [np.array([0.5, 0.5, 0.5]), pts[3], np.array([-0.2, 0.5, 0.5])]
    ds += [1.8, 0.0, 0.3]
    return pts, np.array(qs), np.array(ds)


@pytest.mark.parametrize("metric", [L2, LINF])
def test_query3_equals_brute_force_adversarial(metric):
    rng = np.random.default_rng(2 + metric)
    pts, qs, ds = _adversarial3(rng)
    got = oracle.query3(oracle.build3(pts), qs, ds, metric=metric)
    ref = oracle.brute3(pts, qs, ds, metric=metric)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))
    j = len(qs) - 3                      # radius 1.8 > sqrt 3 covers the cube
    assert ref[0][j + 1] - ref[0][j] == len(pts)


@settings(max_examples=30, deadline=None)
@given(seed=st.integers(0, 2 ** 31), n=st.integers(0, 250), m=st.integers(0, 25),
       scale=st.floats(-6, 0.3), metric=st.sampled_from([L2, LINF]))
def test_query3_equals_brute_force_random(seed, n, m, scale, metric):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    qs = rng.uniform(-0.1, 1.1, (m, 3))
    ds = 10 ** (scale + rng.uniform(-1, 1, m))
    got = oracle.query3(oracle.build3(pts), qs, ds, metric=metric)
    ref = oracle.brute3(pts, qs, ds, metric=metric)
    assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))


def test_far_query_needs_the_widening():
    """q = (2^33 + 1/2, 1/2, 1/2), delta = 2^33: doubles near 2^33 are 2^-19
    apart, 4 quanta of 2^-21, so dx rounds to -2^33 for the points
    (1/2 - k 2^-21, 1/2, 1/2) with k <= 2 (k = 2 is the tie, rounded to
    even): the test accepts points 2 quanta past the exact box edge."""
    k = np.arange(0, 8)
    pts = np.stack([0.5 - k * 2.0 ** -21, np.full(8, 0.5), np.full(8, 0.5)], 1)
    q = np.array([[2.0 ** 33 + 0.5, 0.5, 0.5]])
    d = np.array([2.0 ** 33])
    for metric in (L2, LINF):
        ref = oracle.brute3(pts, q, d, metric=metric)
        assert ref[1].tolist() == [0, 1, 2]
        got = oracle.query3(oracle.build3(pts), q, d, metric=metric)
        assert np.array_equal(oracle.canonical(*got), oracle.canonical(*ref))
    assert oracle.box3(q[0], d[0])[0] <= (1 << 20) - 2


def test_ball_volume_closed_form():
    """Uniform points; balls kept inside the cube: mean count n (4/3) pi d^3,
    here 10."""
    n, m = 1 << 16, 4000
    d = (10.0 / (n * 4.0 / 3.0 * math.pi)) ** (1 / 3)
    rng = np.random.default_rng(5)
    pts = rng.random((n, 3))
    qs = rng.uniform(d, 1 - d, (m, 3))
    off, _ = oracle.query3(oracle.build3(pts), qs, np.full(m, d), nthreads=4)
    assert abs(off[-1] / m - 10.0) < 0.4


def test_cube_window_grid_counts():
    """Dyadic grid (i, j, k) / 32: a cube window of half side r in
    [t/32, (t+1)/32) around a grid point holds the clipped (2t+1)^3 block."""
    g = 32
    ii, jj, kk = np.meshgrid(np.arange(g), np.arange(g), np.arange(g), indexing="ij")
    pts = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1) / g
    rng = np.random.default_rng(6)
    a = rng.integers(0, g, (60, 3))
    t = rng.integers(0, 5, 60)
    qs = a / g
    ds = (t + rng.choice([0.0, 0.5], 60)) / g
    off, ids = oracle.query3(oracle.build3(pts), qs, ds, metric=LINF)
    lo = np.clip(a - t[:, None], 0, g - 1)
    hi = np.clip(a + t[:, None], 0, g - 1)
    want = np.prod(hi - lo + 1, axis=1)
    assert np.array_equal(np.diff(off.astype(np.int64)), want)
    for j in range(60):      # and the ids themselves, from integer arithmetic
        got = sorted(ids[off[j]:off[j + 1]].tolist())
        exp = sorted(int(x * g * g + y * g + z) for x in range(lo[j, 0], hi[j, 0] + 1)
                     for y in range(lo[j, 1], hi[j, 1] + 1) for z in range(lo[j, 2], hi[j, 2] + 1))
        assert got == exp


def test_build3_sorts_pairs_and_rejects_domain():
    rng = np.random.default_rng(7)
    pts = rng.random((3000, 3))
    pts[100:200] = pts[:100]
    k, i, s = oracle.build3(pts)
    assert np.all(np.diff(k.astype(object)) >= 0)
    kk = oracle.keys3(pts)
    assert np.array_equal(k, kk[i]) and np.array_equal(s, pts[i])
    pairs = list(zip(k.tolist(), i.tolist()))
    assert pairs == sorted(pairs)
    with pytest.raises(oracle.DomainError):
        oracle.build3(np.array([[0.5, 1.0, 0.2]]))

"""The search lane of the HIP library (query_lane.inc with query_lane.h,
learned.h, stree.h and curve.h) compiled as host C++ under the address and
undefined-behaviour sanitizers, on the CPU: its index ranges, scanned with
the exact test, give the oracle's whole output id for id in curve order, for
both curves, the method's ranges and the refined cells, binary search, the
static search tree and the learned index (a model built here: leaves at key
quantiles, pieces of 256 keys, exact windows over the stored keys, some
pieces with empty windows so that the fallback runs), and early
termination's occupancy bits.  Any access outside an array, any undefined
shift or overflow aborts the harness."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import HILBERT, MORTON
from paper_2508_19891_amd import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpu", "lane_check.cpp")
CSRC = os.path.join(ROOT, "paper_2508_19891_amd", "csrc")
ROCM_INCLUDE = "/opt/rocm/include"

LEAVES, ROUTE_SLOTS, PIECE, DIRECT_BITS = 4096, 1 << 16, 256, 20


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("HIP headers not installed")
    exe = str(tmp_path_factory.mktemp("lane") / "lane_check")
    subprocess.check_call([
        "g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
        "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE, "-I", CSRC,
        "-I", os.path.join(ROOT, "include"), SRC, "-o", exe])
    return exe


def learned_model(keys, rng, empty_frac=0.1):
    """Arrays of a learned index over sorted keys in the library's layout:
    router boundaries at key quantiles (input X = key >> 40), its bracket
    table, leaves cut into pieces of 256 keys, per piece its first index, a
    slope and the exact window of (lower bound - prediction) over the
    stored keys up to the next piece's first key, and the table of how many
    pieces start below each 20-bit key prefix; a fraction of pieces get an
    empty window instead."""
    n = len(keys)
    X = (keys >> np.uint64(40)).astype(np.int64)
    inner = np.floor(np.quantile(X, np.arange(1, LEAVES) / LEAVES)).astype(np.int64)
    xb = np.concatenate([[0], np.maximum.accumulate(inner), [1 << 24]]).astype(np.uint32)
    t = np.minimum(np.arange(ROUTE_SLOTS + 1, dtype=np.int64) << 8, (1 << 24) - 1)
    rt = np.minimum(np.searchsorted(xb, t, side="right") - 1, LEAVES - 1).astype(np.uint32)
    S = np.searchsorted(X, xb.astype(np.int64), side="left")   # first key of each leaf
    S[LEAVES] = n
    counts = np.diff(S)
    pieces = (counts + PIECE - 1) // PIECE
    P = np.concatenate([[0], np.cumsum(pieces)])
    lp = np.stack([S, P], 1).astype(np.uint32)
    npieces = int(P[-1])
    leaf_of_piece = np.repeat(np.arange(LEAVES), pieces)
    R = S[leaf_of_piece] + (np.arange(npieces) - P[leaf_of_piece]) * PIECE
    E = S[leaf_of_piece + 1]
    Rn = np.minimum(R + PIECE, E)
    fk = keys[R]
    ps = np.concatenate([R, [n]]).astype(np.uint32)
    prefix = np.arange((1 << DIRECT_BITS) + 1, dtype=np.uint64) << np.uint64(64 - DIRECT_BITS)
    dt = np.searchsorted(fk, prefix[:-1], side="left")
    dt = np.concatenate([dt, [npieces]]).astype(np.uint32)
    last = keys[Rn - 1]
    span = (last - fk).astype(np.float64)
    slope = np.where(span > 0, (Rn - R).astype(np.float64) / np.maximum(span, 1.0), 0.0)
    # exact windows over the stored keys a piece brackets (its keys above fk)
    piece_of_idx = np.repeat(np.arange(npieces), Rn - R)
    idx = np.arange(n)
    k = keys
    lb = np.searchsorted(keys, keys, side="left")
    u = (k - fk[piece_of_idx]).astype(np.float64)
    pred = R[piece_of_idx] + np.floor(slope[piece_of_idx] * u + 0.5)
    pred = np.clip(pred, R[piece_of_idx] + 1, Rn[piece_of_idx]).astype(np.int64)
    err = lb - pred
    above = k > fk[piece_of_idx]
    err_lo = np.full(npieces, 0, np.int64)
    err_hi = np.full(npieces, 0, np.int64)
    if above.any():
        np.minimum.at(err_lo, piece_of_idx[above], err[above])
        np.maximum.at(err_hi, piece_of_idx[above], err[above])
    empty = rng.random(npieces) < empty_frac
    err_lo[empty] = 0
    err_hi[empty] = 0
    pr = np.zeros(npieces, dtype=[("s", "<f8"), ("elo", "<i4"), ("ehi", "<i4")])
    pr["s"], pr["elo"], pr["ehi"] = slope, err_lo, err_hi
    del idx
    return xb, rt, lp, fk.astype(np.uint64), pr, ps, dt


def occupancy_bits(keys):
    """Bit (4^k - 1) / 3 + p for every key prefix p of depth k <= 12."""
    words = np.zeros(((4 ** 13 - 1) // 3 + 31) // 32, np.uint32)
    for k in range(13):
        p = np.unique(keys >> np.uint64(64 - 2 * k)) if k else np.zeros(1, np.uint64)
        bit = (4 ** k - 1) // 3 + p.astype(np.int64)
        np.bitwise_or.at(words, bit >> 5, (np.uint32(1) << (bit & 31).astype(np.uint32)))
    return words


def run_harness(exe, tmp_path, keys, q, d, curve, refine, search, model=None, occ=None,
                refine_min=32, ball=True):
    job, out = str(tmp_path / "job.bin"), str(tmp_path / "out.bin")
    n, m = len(keys), len(q)
    with open(job, "wb") as f:
        np.array([n, m, curve, int(refine), search, refine_min, int(ball), int(occ is not None)],
                 np.uint64).tofile(f)
        keys.astype(np.uint64).tofile(f)
        np.ascontiguousarray(q, np.float64).tofile(f)
        np.ascontiguousarray(d, np.float64).tofile(f)
        if search == 1:
            xb, rt, lp, fk, pr, ps, dt = model
            xb.tofile(f)
            rt.tofile(f)
            lp.tofile(f)
            np.array([len(fk)], np.uint64).tofile(f)
            fk.tofile(f)
            pr.tofile(f)
            ps.tofile(f)
            dt.tofile(f)
        if occ is not None:
            np.array([len(occ)], np.uint64).tofile(f)
            occ.tofile(f)
    r = subprocess.run([exe, job, out], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    raw = np.fromfile(out, np.uint8)
    slots = raw[:32 * 4 * m].view(np.uint64).reshape(m, 4, 4)
    nr = raw[32 * 4 * m:].view(np.uint32)
    return slots, nr


def scan_slots(index, q, d, slots, refine):
    """The CSR the kernels after the search produce from the slots: every
    range in slot order, each candidate tested exactly (binary64, fixed
    order, no fused multiply-add)."""
    sk, si, sxy = index
    m = len(q)
    counts = np.zeros(m, np.int64)
    out = []
    cols = (0, 2) if refine else (0,)
    for j in range(m):
        got = []
        for r in range(4):
            for c in cols:
                b, e = int(slots[j, r, c]), int(slots[j, r, c + 1])
                assert 0 <= b <= e <= len(sk), (j, r, c, b, e)
                if e > b:
                    p = sxy[b:e]
                    dx = p[:, 0] - q[j, 0]
                    dy = p[:, 1] - q[j, 1]
                    got.append(si[b:e][dx * dx + dy * dy <= d[j] * d[j]])
        row = np.concatenate(got) if got else np.zeros(0, np.uint32)
        counts[j] = len(row)
        out.append(row)
    off = np.zeros(m + 1, np.uint64)
    off[1:] = np.cumsum(counts)
    return off, (np.concatenate(out).astype(np.uint32) if out else np.zeros(0, np.uint32))


def check(exe, tmp_path, pts, q, d, curve, refine, search, occ=False, seed=0):
    index = oracle.build(pts, curve)
    model = learned_model(index[0], np.random.default_rng(seed)) if search == 1 else None
    bits = occupancy_bits(index[0]) if occ else None
    slots, nr = run_harness(exe, tmp_path, index[0], q, d, curve, refine, search, model, bits)
    got = scan_slots(index, q, d, slots, refine)
    want = oracle.query(index, q, d, curve, nthreads=4)
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1], want[1])
    assert (nr <= 4).all()
    return slots


def test_learned_refined_clustered_morton(harness, tmp_path):
    """The clustered Morton batch (seed 8, 3e5 points, 2e4 queries, refined
    cells) on which an earlier variant of the cell ordering lost reports in
    the learned-index kernel: the lane code agrees with the oracle."""
    wl = workload.clustered_loguniform(n=300_000, m=20_000, curve=MORTON, seed=8)
    check(harness, tmp_path, wl.points, wl.queries, wl.delta, MORTON, True, 1, seed=1)


@pytest.mark.parametrize("search", [0, 1, 2])
@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_lane_matches_oracle(harness, tmp_path, curve, refine, search):
    wl = workload.clustered_loguniform(n=60_000, m=4000, curve=curve, seed=11)
    q, d = wl.queries.copy(), wl.delta.copy()
    # edge cases: outside the square, zero and huge radii, the far corner
    q[:6] = [[-0.5, 0.5], [0.5, 0.5], [1.5, 1.5], [1.0 - 2.0 ** -53, 1.0 - 2.0 ** -53],
             [0.0, 0.0], [0.25, 0.75]]
    d[:6] = [0.6, 2.0, 0.01, 1e-12, 0.0, 1e-300]
    check(harness, tmp_path, wl.points, q, d, curve, refine, search, seed=2)


@pytest.mark.parametrize("refine", [False, True])
def test_lane_early_termination(harness, tmp_path, refine):
    """Sparse uniform queries over clustered points with the occupancy bits:
    skipped cells hold no point, so the output is the oracle's."""
    wl = workload.clustered_loguniform(n=80_000, m=3000, curve=HILBERT, seed=12)
    q = workload.uniform_points(3000, 77)
    d = np.full(3000, workload.radius_for_count(1.0, 80_000))
    check(harness, tmp_path, wl.points, q, d, HILBERT, refine, 0, occ=True)


@pytest.mark.parametrize("search", [0, 1, 2])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_lane_cell_corner_points(harness, tmp_path, curve, search):
    """Points in the corner grid cells of aligned blocks (a cell's first and
    last keys: the inclusive ends of each key interval) and queries centred
    on them whose cells are those blocks."""
    rng = np.random.default_rng(13)
    pts, qs, ds = [], [], []
    for s in (4, 10, 16, 20, 24, 28):
        j = rng.integers(1, (1 << (32 - s)) - 1, size=(300, 2))
        off = rng.integers(0, 2, size=(300, 2))       # block's last cell (-1) or first (0)
        cell = j * (1 << s) - 1 + off
        p = (cell + 0.5) / 2.0 ** 32
        pts.append(p)
        qs.append(p[:100])
        ds.append(2.0 ** (s - 32) * rng.uniform(0.3, 0.5, 100))
    pts = np.concatenate([np.concatenate(pts), rng.random((20_000, 2))])
    check(harness, tmp_path, pts, np.concatenate(qs), np.concatenate(ds), curve, True, search,
          seed=3)
    check(harness, tmp_path, pts, np.concatenate(qs), np.concatenate(ds), curve, False, search,
          seed=3)


def test_lockstep_search(tmp_path):
    """The lockstep search of several key intervals (one shared chain while
    the probes fall outside every interval, then one chain per bound), both
    index widths, against std::lower_bound / std::upper_bound under the
    sanitizers: every array length up to 300 and some around powers of two,
    repeated keys, unused and empty intervals, keys at both ends of the
    64-bit range."""
    if not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("HIP headers not installed")
    exe = str(tmp_path / "search_check")
    subprocess.check_call([
        "g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
        "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE, "-I", CSRC,
        "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "cpu", "search_check.cpp"),
        "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr

"""Parity of the HIP path with the oracle, step by step, through the C ABI.

Bit-exact everywhere: keys, the sorted (key, id, point) arrays, key ranges
and index ranges, and the CSR output (offsets and ids, in curve order, which
is unique because both sides scan ranges in ascending (key, id) order).
"""
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


def adversarial_points(rng, n):
    pts = rng.random((n, 2))
    k = n // 8
    if k:
        pts[k:2 * k] = pts[:k]                                       # duplicates
        pts[2 * k:3 * k] = np.floor(pts[2 * k:3 * k] * 2 ** 32) / 2 ** 32   # on quantum edges
        pts[3 * k:3 * k + 3] = [[0.0, 0.0], [workload.ONE_BELOW] * 2, [0.0, workload.ONE_BELOW]]
    return pts


SIZES = [1, 2, 63, 64, 65, 1000, 4095, 4096, 4097, 70_001, 300_000]


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
@pytest.mark.parametrize("n", [1, 65, 4097, 100_003])
def test_keys(curve, n):
    rng = np.random.default_rng(n + curve)
    pts = adversarial_points(rng, n)
    got = sfc.u64(sfc.sfc_keys(dev(pts), curve))
    assert np.array_equal(got, oracle.keys(pts, curve))


@pytest.mark.parametrize("bad", [1.0, -1e-300, float("nan"), float("inf")])
def test_keys_domain_error(bad):
    pts = np.random.default_rng(0).random((5000, 2))
    pts[4321, 1] = bad
    with pytest.raises(sfc.DomainError):
        sfc.sfc_keys(dev(pts), MORTON)
    with pytest.raises(sfc.DomainError):
        sfc.Index(dev(pts), MORTON)


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
@pytest.mark.parametrize("n", SIZES)
def test_build_sorted_arrays(curve, n):
    rng = np.random.default_rng(10 + n)
    pts = adversarial_points(rng, n)
    idx = sfc.Index(dev(pts), curve)
    k, i, s = idx.sorted_arrays()
    ok, oi, os_ = oracle.build(pts, curve)
    assert np.array_equal(sfc.u64(k), ok)
    assert np.array_equal(i.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(s.cpu().numpy(), os_)
    idx.close()


def test_build_empty():
    idx = sfc.Index(torch.empty((0, 2), dtype=torch.float64, device=DEV))
    assert idx.size() == 0
    off, ids = idx.query(dev([[0.5, 0.5]]), dev([0.1]))
    assert off.cpu().tolist() == [0, 0] and ids.numel() == 0


def _queries(rng, m, scale=(-4, -1)):
    qs = rng.uniform(-0.05, 1.05, (m, 2))
    ds = 10 ** rng.uniform(*scale, m)
    return qs, ds


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_ranges_match_oracle(curve):
    rng = np.random.default_rng(5)
    pts = adversarial_points(rng, 50_000)
    qs, ds = _queries(rng, 3000, (-7, 0.3))
    qs[:5] = [[0.5, 0.5], [-3, 0.5], [5, 5], [0.0, 0.0], [0.999, 0.2]]
    ds[:5] = [0.0, 10.0, 1.0, 2.0, 1e-300]
    idx = sfc.Index(dev(pts), curve)
    klo, khi, b, e, nr = idx.query_ranges(dev(qs), dev(ds))
    klo, khi = sfc.u64(klo), sfc.u64(khi)
    b, e, nr = b.cpu().numpy(), e.cpu().numpy(), nr.cpu().numpy()
    sk = oracle.build(pts, curve)[0]
    for j in range(len(qs)):
        rs = oracle.ranges(qs[j, 0], qs[j, 1], ds[j], curve)
        assert nr[j] == len(rs), j
        ir = oracle.index_ranges(sk, qs[j, 0], qs[j, 1], ds[j], curve)
        for r, ((lo, hi), (bb, ee)) in enumerate(zip(rs, ir)):
            assert (int(klo[j, r]), int(khi[j, r]), int(b[j, r]), int(e[j, r])) == (lo, hi, bb, ee)


def check_query(pts, qs, ds, curve, nthreads=4, refine=False):
    idx = sfc.Index(dev(pts), curve, refine=refine)
    off, ids = idx.query(dev(qs), dev(ds))
    ref_off, ref_ids = oracle.query(oracle.build(pts, curve), qs, ds, curve, nthreads=nthreads)
    got_off = off.cpu().numpy().view(np.uint64)
    got_ids = ids.cpu().numpy().view(np.uint32)
    assert np.array_equal(got_off, ref_off)
    assert np.array_equal(got_ids, ref_ids)
    return idx, ref_off


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
@pytest.mark.parametrize("n,m", [(1, 1), (100, 7), (4097, 1000), (65_536, 10_000), (250_000, 20_000)])
def test_query_matches_oracle(curve, n, m, refine):
    rng = np.random.default_rng(n + m)
    pts = adversarial_points(rng, n)
    qs, ds = _queries(rng, m)
    check_query(pts, qs, ds, curve, refine=refine)


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_query_clustered(curve, refine):
    wl = workload.clustered_loguniform(n=300_000, m=30_000, curve=curve)
    check_query(wl.points, wl.queries, wl.delta, curve, refine=refine)


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_query_edge_cases(curve, refine):
    rng = np.random.default_rng(77)
    pts = adversarial_points(rng, 20_000)
    qs, ds = _queries(rng, 500)
    special_q = [[0.5, 0.5], pts[5], pts[9], [-0.2, 0.5], [1.3, 1.3], [0.3, 0.9], [7.0, 7.0],
                 [0.0, 0.0], [workload.ONE_BELOW] * 2]
    special_d = [2.0, 0.0, 0.0, 0.25, 0.5, 1e-300, 0.1, 0.0, 1e-12]
    qs = np.concatenate([special_q, qs, special_q])
    ds = np.concatenate([special_d, ds, special_d])
    check_query(pts, qs, ds, curve, refine=refine)


@pytest.mark.parametrize("refine", [False, True])
def test_query_all_empty_and_trailing_empty(refine):
    rng = np.random.default_rng(3)
    pts = rng.random((5000, 2))
    far = np.full((300, 2), 5.0)
    check_query(pts, far, np.full(300, 0.1), MORTON, refine=refine)
    qs = np.concatenate([rng.random((50, 2)), far])
    check_query(pts, qs, np.full(350, 0.05), MORTON, refine=refine)
    qs = np.concatenate([far, rng.random((50, 2)), far])
    check_query(pts, qs, np.full(650, 0.05), HILBERT, refine=refine)


def test_query_zero_queries():
    pts = np.random.default_rng(1).random((1000, 2))
    idx = sfc.Index(dev(pts), MORTON)
    off, ids = idx.query(torch.empty((0, 2), dtype=torch.float64, device=DEV),
                         torch.empty(0, dtype=torch.float64, device=DEV))
    assert off.cpu().tolist() == [0] and ids.numel() == 0


@pytest.mark.parametrize("bad", [(0.5, 0.5, -1.0), (0.5, 0.5, float("nan")),
                                 (float("inf"), 0.5, 0.1), (0.5, float("nan"), 0.1)])
def test_query_invalid(bad):
    pts = np.random.default_rng(1).random((1000, 2))
    idx = sfc.Index(dev(pts), MORTON)
    qs = np.full((100, 2), 0.5)
    ds = np.full(100, 0.01)
    qs[37] = bad[:2]
    ds[37] = bad[2]
    with pytest.raises(sfc.SfcError) as ei:
        idx.query(dev(qs), dev(ds))
    assert ei.value.status == sfc.SFC_ERR_INVALID


def test_query_capacity():
    rng = np.random.default_rng(4)
    pts = rng.random((10_000, 2))
    qs = rng.random((100, 2))
    ds = np.full(100, 0.05)
    idx = sfc.Index(dev(pts), MORTON)
    with pytest.raises(sfc.CapacityError) as ei:
        idx.query(dev(qs), dev(ds), ids_cap=10)
    ref_off, ref_ids = oracle.query(oracle.build(pts, MORTON), qs, ds, MORTON)
    assert ei.value.total == len(ref_ids)
    off, ids = idx.query(dev(qs), dev(ds), ids_cap=len(ref_ids))
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref_ids)


@pytest.mark.parametrize("refine", [False, True])
def test_query_large_outputs_many_tiles(refine):
    # Huge radii: every query reports every point; candidates span many tiles.
    rng = np.random.default_rng(8)
    pts = rng.random((30_000, 2))
    qs = rng.random((300, 2))
    ds = np.full(300, 1.5)
    check_query(pts, qs, ds, HILBERT, refine=refine)
    ds = np.full(300, 0.3)
    check_query(pts, qs, ds, MORTON, refine=refine)


def test_query_repeatable():
    rng = np.random.default_rng(9)
    pts = rng.random((200_000, 2))
    qs, ds = _queries(rng, 30_000)
    idx = sfc.Index(dev(pts), MORTON)
    a = idx.query(dev(qs), dev(ds))
    for _ in range(3):
        b = idx.query(dev(qs), dev(ds))
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_uniform_fixed_radius_workload():
    wl = workload.uniform_fixed_radius(n=1 << 16, m=10_000, curve=MORTON)
    _, ref_off = check_query(wl.points, wl.queries, wl.delta, MORTON)
    assert abs(ref_off[-1] / 10_000 - 9.941) < 0.25


@pytest.mark.parametrize("refine", [False, True])
def test_capacity_keeps_ids_and_retry_writes_only(refine):
    rng = np.random.default_rng(41)
    pts = rng.random((50_000, 2))
    qs = rng.random((3000, 2))
    ds = np.full(3000, 0.02)
    ref_off, ref_ids = oracle.query(oracle.build(pts, HILBERT), qs, ds, HILBERT)
    idx = sfc.Index(dev(pts), HILBERT, refine=refine)
    q, d = dev(qs), dev(ds)
    offsets = torch.empty(3001, dtype=torch.int64, device=DEV)
    small = torch.full((100,), 0x7FFFFFFF, dtype=torch.int32, device=DEV)
    with pytest.raises(sfc.CapacityError) as ei:
        idx.query(q, d, out_ids=small, out_offsets=offsets)
    assert ei.value.total == len(ref_ids)
    assert bool((small == 0x7FFFFFFF).all())                      # ids untouched
    assert np.array_equal(offsets.cpu().numpy().view(np.uint64), ref_off)
    with pytest.raises(sfc.CapacityError):                          # still too small
        idx.query_retry(offsets, small)
    big = torch.empty(len(ref_ids), dtype=torch.int32, device=DEV)
    assert idx.query_retry(offsets, big) == len(ref_ids)
    assert np.array_equal(big.cpu().numpy().view(np.uint32), ref_ids)
    with pytest.raises(sfc.SfcError):                               # nothing kept any more
        idx.query_retry(offsets, big)
    # Any later query drops the kept batch; the binding then reruns instead.
    with pytest.raises(sfc.CapacityError):
        idx.query(q, d, out_ids=small, out_offsets=offsets)
    idx.query(q[:10], d[:10])
    with pytest.raises(sfc.SfcError):
        idx.query_retry(offsets, big)
    off2, ids2 = idx.query(q, d)                                    # binding's own retry
    assert np.array_equal(ids2.cpu().numpy().view(np.uint32), ref_ids)


def test_capacity_many_chunks_writes_prefix_and_reruns():
    rng = np.random.default_rng(42)
    pts = rng.random((40_000, 2))
    qs = rng.random((2000, 2))
    ds = np.full(2000, 0.03)
    ref_off, ref_ids = oracle.query(oracle.build(pts, MORTON), qs, ds, MORTON)
    try:
        sfc.debug_chunk_tiles(2)
        idx = sfc.Index(dev(pts), MORTON)
        small = torch.full((50,), -1, dtype=torch.int32, device=DEV)
        offsets = torch.empty(2001, dtype=torch.int64, device=DEV)
        with pytest.raises(sfc.CapacityError):
            idx.query(dev(qs), dev(ds), out_ids=small, out_offsets=offsets)
        assert np.array_equal(small.cpu().numpy().view(np.uint32), ref_ids[:50])
        with pytest.raises(sfc.SfcError):
            idx.query_retry(offsets, torch.empty(len(ref_ids), dtype=torch.int32, device=DEV))
        off, ids = idx.query(dev(qs), dev(ds), ids_cap=None)
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref_ids)
    finally:
        sfc.debug_chunk_tiles(0)

"""The learned index on the GPU: exact agreement with binary search and the
oracle, the fallback path, and the trainer's gradients against the FP64
reference of the router."""
import numpy as np
import pytest
import torch

import oracle
from oracle import HILBERT, MORTON, learned
from paper_2508_19891_amd import sfc, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(DEV)


def _clustered(n, m, curve, seed=7):
    wl = workload.clustered_loguniform(n=n, m=m, curve=curve, seed=seed)
    return wl.points, wl.queries, wl.delta


@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_learned_index_ranges_equal_binary_search(curve):
    pts, qs, ds = _clustered(200_000, 5000, curve)
    qs[:3] = [[-1.0, 0.5], [0.5, 0.5], [2.0, 2.0]]
    ds[:3] = [0.1, 2.0, 0.5]
    idx = sfc.Index(dev(pts), curve, search=sfc.LEARNED)
    info = idx.learned_info()
    assert info["fitted"] == 1 and info["leaves_nonempty"] > 100
    klo, khi, b, e, nr = idx.query_ranges(dev(qs), dev(ds))
    sk = oracle.build(pts, curve)[0]
    b, e, nr = b.cpu().numpy(), e.cpu().numpy(), nr.cpu().numpy()
    for j in range(len(qs)):
        ir = oracle.index_ranges(sk, qs[j, 0], qs[j, 1], ds[j], curve)
        assert nr[j] == len(ir)
        for r, (bb, ee) in enumerate(ir):
            assert (int(b[j, r]), int(e[j, r])) == (bb, ee), (j, r)
    # A monotone router with exact windows never needs the fallback.
    info = idx.learned_info()
    assert info["endpoints_last"] > 0
    assert info["fallbacks_last"] == 0


@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("curve", [MORTON, HILBERT])
def test_learned_query_matches_oracle(curve, refine):
    pts, qs, ds = _clustered(300_000, 20_000, curve, seed=8)
    idx = sfc.Index(dev(pts), curve, search=sfc.LEARNED, refine=refine)
    off, ids = idx.query(dev(qs), dev(ds))
    ref_off, ref_ids = oracle.query(oracle.build(pts, curve), qs, ds, curve, nthreads=4)
    assert np.array_equal(off.cpu().numpy().view(np.uint64), ref_off)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref_ids)
    assert idx.learned_info()["fallbacks_last"] == 0


def test_forced_fallback_keeps_results():
    pts, qs, ds = _clustered(150_000, 10_000, MORTON, seed=9)
    idx = sfc.Index(dev(pts), MORTON, search=sfc.LEARNED)
    want = idx.query(dev(qs), dev(ds))
    idx.learned_shrink_windows()
    got = idx.query(dev(qs), dev(ds))
    assert torch.equal(want[0], got[0]) and torch.equal(want[1], got[1])
    assert idx.learned_info()["fallbacks_last"] > 0


def test_switching_search_modes():
    pts, qs, ds = _clustered(100_000, 5000, HILBERT, seed=10)
    idx = sfc.Index(dev(pts), HILBERT)
    a = idx.query(dev(qs), dev(ds))
    idx.set_search(sfc.LEARNED)
    b = idx.query(dev(qs), dev(ds))
    idx.set_search(sfc.BINARY)
    c = idx.query(dev(qs), dev(ds))
    for x, y in ((a, b), (a, c)):
        assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])


def test_learned_duplicates_and_tiny_sets():
    rng = np.random.default_rng(11)
    base = rng.random((50, 2))
    pts = base[rng.integers(0, 50, 20_000)]              # heavy duplicates
    qs = rng.random((2000, 2))
    ds = 10 ** rng.uniform(-3, -0.5, 2000)
    for n in (2, 3, 17, 20_000):
        idx = sfc.Index(dev(pts[:n]), MORTON, search=sfc.LEARNED)
        off, ids = idx.query(dev(qs), dev(ds))
        ref = oracle.query(oracle.build(pts[:n], MORTON), qs, ds, MORTON)
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])


def test_trained_router_is_monotone_and_learns():
    pts, _, _ = _clustered(400_000, 10, MORTON, seed=12)
    idx = sfc.Index(dev(pts), MORTON, search=sfc.LEARNED, learn_steps=512)
    p = idx.learned_params().astype(np.float64)
    w1, b1, W2, b2, w3, b3 = learned.unpack(p)
    assert (w1 >= 0).all() and (W2 >= 0).all() and (w3 >= 0).all()
    info = idx.learned_info()
    assert info["steps"] == 512
    assert info["loss_final"] < info["loss_init"]
    # The FP64 forward of the trained parameters is a CDF estimate of the keys.
    keys = np.sort(oracle.keys(pts, MORTON))
    x = (keys >> np.uint64(40)).astype(np.float64) / 2.0 ** 24
    y, _ = learned.forward(p, x[:: 97])
    assert np.all(np.diff(y) >= -1e-9)
    rank = np.arange(0, len(keys), 97) / len(keys)
    assert np.sqrt(np.mean((y - rank) ** 2)) < 0.1


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_gpu_gradient_matches_fp64_reference(seed):
    rng = np.random.default_rng(seed)
    w1, b1, W2, b2, w3, b3 = learned.unpack(rng.normal(0, 1, learned.NPARAM))
    p = learned.pack(np.abs(w1) * 3, b1 * 0.5, np.abs(W2) / 8, b2 * 0.2, np.abs(w3) / 4, b3 * 0.1)
    p32 = p.astype(np.float32).astype(np.float64)       # the values the GPU sees
    cnt = [128, 77, 1, 128][seed]
    x = rng.random(cnt).astype(np.float32).astype(np.float64)
    t = np.sort(rng.random(cnt)).astype(np.float32).astype(np.float64)
    g_gpu, loss_gpu = sfc.learned_grad(p32, x, t)
    g_ref = learned.grad(p32, x, t)
    assert abs(loss_gpu - learned.loss(p32, x, t)) <= 1e-4 * max(1.0, learned.loss(p32, x, t))
    # every entry, against the scale of the whole gradient (FP32 arithmetic
    # on the GPU, FP64 in the reference) ...
    tol = 1e-3 * np.abs(g_ref).max() + 1e-6
    bad = np.nonzero(np.abs(g_gpu - g_ref) > tol)[0]
    assert bad.size == 0, (bad[:10], g_gpu[bad[:10]], g_ref[bad[:10]])
    # ... and every parameter block against its own scale, so that a wrong
    # small block (b3, b1) cannot hide under the large W2 block
    o = 0
    for name, size in (("w1", 32), ("b1", 32), ("W2", 1024), ("b2", 32), ("w3", 32),
                       ("b3", 1)):
        gb, rb = g_gpu[o:o + size], g_ref[o:o + size]
        o += size
        assert np.abs(gb - rb).max() <= 1e-3 * np.abs(rb).max() + 1e-6, name
    assert o == learned.NPARAM


def test_tabulated_router_equals_network_for_every_input():
    """Every 24-bit router input (each X << 40, and the key just below it)
    gets the same leaf from the network and from the tabulation."""
    pts, _, _ = _clustered(200_000, 10, MORTON, seed=13)
    idx = sfc.Index(dev(pts), MORTON, search=sfc.LEARNED)
    X = torch.arange(1 << 24, dtype=torch.int64, device=DEV)
    for keys in (X << 40, (X << 40) | ((1 << 40) - 1)):
        d, t = idx.learned_route(keys)
        assert torch.equal(d, t)
        assert bool((d[1:] >= d[:-1]).all())          # monotone


def test_learned_search_takes_fewer_steps_than_binary_search():
    pts, qs, ds = _clustered(1 << 20, 20_000, MORTON, seed=14)
    idx = sfc.Index(dev(pts), MORTON, search=sfc.LEARNED, refine=True)
    info = idx.learned_info()
    print("learned info", info)
    assert info["pieces"] >= (1 << 20) // 256
    assert info["search_steps"] < 0.6 * 20
    idx.query(dev(qs), dev(ds))
    assert idx.learned_info()["fallbacks_last"] == 0


def test_trained_router_against_its_initialisation():
    """What training buys over the router's quantile initialisation: the
    sample loss drops, and the search after routing takes no more steps."""
    pts, qs, ds = _clustered(1 << 20, 20_000, HILBERT, seed=15)
    init = sfc.Index(dev(pts), HILBERT, search=sfc.LEARNED, learn_steps=0)
    trained = sfc.Index(dev(pts), HILBERT, search=sfc.LEARNED, learn_steps=512)
    a, b = init.learned_info(), trained.learned_info()
    print("init", a["loss_final"], a["search_steps"], a["max_leaf"],
          "trained", b["loss_final"], b["search_steps"], b["max_leaf"])
    assert b["loss_final"] < a["loss_final"]
    assert b["search_steps"] <= a["search_steps"] + 0.25
    for ix in (init, trained):
        off, ids = ix.query(dev(qs), dev(ds))
        assert ix.learned_info()["fallbacks_last"] == 0
    ref = oracle.query(oracle.build(pts, HILBERT), qs, ds, HILBERT, nthreads=4)
    assert np.array_equal(ids.cpu().numpy().view(np.uint32), ref[1])


def test_learned_search_in_a_recorded_graph():
    pts, qs, ds = _clustered(150_000, 8_000, MORTON, seed=16)
    idx = sfc.Index(dev(pts), MORTON, search=sfc.LEARNED, refine=True)
    q, d = dev(qs), dev(ds)
    want = idx.query(q, d)
    g = sfc.Graph.query(idx, q, d, max_rows=idx.last_stats()["rows"] + 64,
                        ids_cap=want[1].numel() + 1)
    for _ in range(3):
        g.launch()
        off, ids = g.result()
        assert torch.equal(off, want[0]) and torch.equal(ids, want[1])
    g.close()

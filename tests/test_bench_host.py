"""Host-side checks of the benchmark script and the workload generators it
uses (no GPU): the multi-GPU refusal, the JSON contract's algorithmic-byte
bookkeeping inputs, and the seeded 3-D and window workloads."""
import math
import os
import subprocess
import sys

import numpy as np

from paper_2508_19891_amd import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_square_windows_workload():
    wl = workload.square_windows(n=20_000, m=500, side=1e-3, points="normal")
    assert wl.points.shape == (20_000, 2) and wl.queries.shape == (500, 2)
    assert np.all(wl.delta == 5e-4)
    assert ((wl.points >= 0) & (wl.points < 1)).all()
    # normal around the centre with sigma 1/8: about 68% within one sigma per axis
    frac = np.mean(np.abs(wl.points[:, 0] - 0.5) < 0.125)
    assert abs(frac - 0.683) < 0.02


def test_clustered3_radii_aim_at_counts():
    """delta = (3c / (4 pi n f))^(1/3) inverts the ball volume: n f (4/3) pi
    delta^3 = c, with c in [1, 300]."""
    wl = workload.clustered3(n=10_000, m=2_000, seed=3)
    assert wl.points.shape == (10_000, 3) and ((wl.points >= 0) & (wl.points < 1)).all()
    rng_c = workload.loguniform(workload._rng(3003), 1.0, 300.0, 2_000)
    # recover c from delta with the analytic density
    centres = workload._rng(503).random((16, 3))
    d2 = ((wl.queries[:, None, :] - centres[None]) ** 2).sum(-1)
    f = 0.2 + (0.8 / 16) * (np.exp(-d2 / (2 * 0.02 ** 2)) / (2 * math.pi * 0.02 ** 2) ** 1.5).sum(1)
    c = 10_000 * f * 4.0 / 3.0 * math.pi * wl.delta ** 3
    assert np.allclose(c, rng_c, rtol=1e-9)


def test_mixture_density_slices_equal_whole():
    mix = workload.make_mixture(7)
    q = np.random.default_rng(1).random((300_000, 2))
    got = mix.density(q)
    k = mix.centres.shape[0]
    d2 = ((q[:, None, :] - mix.centres[None, :, :]) ** 2).sum(-1)
    g = np.exp(-d2 / (2.0 * mix.sigma ** 2)) / (2.0 * math.pi * mix.sigma ** 2)
    assert np.array_equal(got, (1.0 - mix.frac) + (mix.frac / k) * g.sum(1))


def test_headline_is_compact_and_complete():
    """The bench's last stdout line stays a few KB (the record of a run keeps
    only the tail of its output) and carries the contract's fields."""
    import importlib.util
    import json
    import types
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    lvb = {"search_ms_learned": 0.5, "search_ms_bsearch": 0.53, "search_ms_stree": 0.52,
           "ms_per_batch_learned": 1.9, "ms_per_batch_bsearch": 1.95,
           "model": {"fallbacks_last": 0}}
    big = {f"k{i}": list(range(50)) for i in range(200)}   # detail that must not leak in
    load = {"requests": 10000, "requests_per_s": 4000.0, "p50_ms": 4.0, "p99_ms": 12.0}
    detail = {
        "config": {"workload": "clustered_n16777216_m1048576_hilbert", "n": 1 << 24,
                   "m": 1 << 20, "curve": "hilbert", "search": "binary", "ranges": "refined",
                   "step": "build + one query batch"},
        "reported_pts_per_s": 6e10, "candidates_per_report": 2.14, "build_ms_per_step": 0.87,
        "roofline": {"bound": "hbm", "kernel": "compact_test", "achieved": 4430.123456,
                     "peak": 8000.0, "unit": "GB/s", "frac": 0.5537, "traffic": 3.48e9,
                     "traffic_gbs": 6312.0, "bytes_per_launch": 3.1e9, "read_gbs": 6034.0,
                     "copy_gbs": 4993.0,
                     "frac_16B_per_candidate": 1.05},
        "learned_vs_bsearch": lvb,
        "learned_large": {"n": 1 << 26, "m": 1 << 22, "learned": {"search_ms": 0.9,
                                                                 "ms_per_batch": 2.8},
                          "bsearch": {"search_ms": 1.05, "ms_per_batch": 2.98}},
        "early_termination": {"speedup_batch": 0.92, "plain": {"ms_per_batch": 0.65},
                              "early_term": {"ms_per_batch": 0.70},
                              "paper_windows": {"sides": [{"side": 1e-7, "speedup_batch": 1.2},
                                                          {"side": 1e-5, "speedup_batch": 1.1},
                                                          {"side": 1e-4, "speedup_batch": 1.15}]}},
        "serving": {"overlap": {"saturation": load, "load_0.95": load}},
        "cpu_baseline": {"value": 2.8e5, "unit": "queries/s", "cores": 16, "kind": "oracle",
                         "sample": "oracle build of all 16777216 points on 1 thread (3.09 s) + "
                                   "all 1048576 queries on 16 threads (0.64 s)"},
        "paper_windows": big,
    }
    args = types.SimpleNamespace(steps=20, warmup=5)
    line = bench.headline(args, detail, 1 << 24, 1 << 20, 2.87, 2.85)
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) <= 2048, len(text)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in line, key
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in line["roofline"], key
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in line["cpu_baseline"], key
    assert line["learned_vs_bsearch"]["large"]["n"] == 1 << 26

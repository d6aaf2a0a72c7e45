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

"""Pins of the FP64 router reference (oracle/learned.py): the analytic
gradient against central finite differences of the loss, monotonicity of the
network for non-negative weights, and the quantile initialisation against the
empirical CDF it interpolates."""
import numpy as np
import pytest

from oracle import learned


def random_params(rng):
    w1, b1, W2, b2, w3, b3 = learned.unpack(rng.normal(0, 1, learned.NPARAM))
    return learned.pack(np.abs(w1) * 4, b1, np.abs(W2) / 4, b2 * 0.3, np.abs(w3), b3)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    p = random_params(rng)
    x = rng.random(64)
    t = np.sort(rng.random(64))
    g = learned.grad(p, x, t)
    eps = 1e-6
    # Every parameter whose finite difference does not straddle a kink of the
    # clipped units (checked by comparing one-sided differences).
    checked = 0
    for i in range(learned.NPARAM):
        e = np.zeros(learned.NPARAM)
        e[i] = eps
        lp, l0, lm = learned.loss(p + e, x, t), learned.loss(p, x, t), learned.loss(p - e, x, t)
        fwd, bwd = (lp - l0) / eps, (l0 - lm) / eps
        if abs(fwd - bwd) > 1e-6 * max(1.0, abs(fwd)):
            continue
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])
        checked += 1
    assert checked > learned.NPARAM * 0.9


def test_monotone_for_nonnegative_weights():
    rng = np.random.default_rng(5)
    for _ in range(20):
        p = random_params(rng)
        x = np.sort(rng.random(5000))
        y, _ = learned.forward(p, x)
        assert np.all(np.diff(y) >= -1e-12)


def test_quantile_init_interpolates_cdf():
    rng = np.random.default_rng(6)
    xs = np.sort(rng.beta(2, 5, 4096))
    p = learned.quantile_init(xs)
    y, _ = learned.forward(p, xs)
    ecdf = np.arange(len(xs)) / len(xs)
    assert np.max(np.abs(y - ecdf)) < 1.5 / 32

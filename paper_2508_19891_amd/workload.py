"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the method's
arithmetic (no keys, boxes, ranges or distance tests).  Both the HIP path and
the oracle consume the arrays it returns, byte for byte.

Distributions:
  * uniform points in [0,1)^2 (the paper's Uniform distribution, Sec. 3
    "Data", rescaled from [0, 2^32) to [0,1));
  * clustered points: a fraction ``frac`` (exactly floor(frac*n) points) from
    an equal-weight mixture of ``k`` isotropic Gaussians with uniform centres
    and standard deviation ``sigma``, the rest uniform, clamped to
    [0, 1 - 2^-53] (the largest double below 1) and shuffled;
  * query radii that aim at a given expected output size c: for a query at q
    over n points of density f, delta = sqrt(c / (pi * n * f(q))), with c
    log-uniform in [c_lo, c_hi].

Generators are numpy PCG64 streams; every function takes an explicit seed.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os

import numpy as np

ONE_BELOW = float(np.nextafter(1.0, 0.0))   # 1 - 2^-53


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass(frozen=True)
class Mixture:
    """Clustered distribution: weight ``frac`` on k Gaussians, rest uniform."""
    centres: np.ndarray      # (k, 2)
    sigma: float
    frac: float

    def density(self, q: np.ndarray) -> np.ndarray:
        """Analytic density of the (unclamped) mixture at the rows of q
        (evaluated in slices of rows, each row as a whole)."""
        q = np.asarray(q, np.float64)
        k = self.centres.shape[0]
        out = np.empty(q.shape[0])
        step = 1 << 16

        def part(a):
            qa = q[a:a + step]
            d2 = ((qa[:, None, :] - self.centres[None, :, :]) ** 2).sum(-1)
            g = np.exp(-d2 / (2.0 * self.sigma ** 2)) / (2.0 * math.pi * self.sigma ** 2)
            out[a:a + step] = (1.0 - self.frac) + (self.frac / k) * g.sum(1)

        starts = range(0, q.shape[0], step)
        if q.shape[0] <= 4 * step:
            for a in starts:
                part(a)
        else:   # numpy releases the interpreter lock inside these operations
            with concurrent.futures.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(part, starts))
        return out

    def sample(self, n: int, rng: np.random.Generator) -> np.ndarray:
        nc = (int(round(self.frac * 1000)) * n) // 1000   # floor(frac * n)
        comp = rng.integers(0, self.centres.shape[0], nc)
        pc = self.centres[comp] + self.sigma * rng.standard_normal((nc, 2))
        pu = rng.random((n - nc, 2))
        p = np.concatenate([pc, pu], axis=0)
        np.clip(p, 0.0, ONE_BELOW, out=p)
        return p[rng.permutation(n)]


def uniform_points(n: int, seed: int) -> np.ndarray:
    return _rng(seed).random((n, 2))


def normal_points(n: int, seed: int, sigma: float = 0.125) -> np.ndarray:
    """The paper's normal distribution (Sec. 4 "Data"): both coordinates
    normal around the centre of the domain with standard deviation sigma
    times its side (1/8), clamped to [0, 1 - 2^-53]."""
    p = 0.5 + sigma * _rng(seed).standard_normal((n, 2))
    np.clip(p, 0.0, ONE_BELOW, out=p)
    return p


def make_mixture(seed: int, k: int = 16, sigma: float = 0.01, frac: float = 0.8) -> Mixture:
    return Mixture(centres=_rng(seed).random((k, 2)), sigma=sigma, frac=frac)


def clustered_points(n: int, seed: int, mixture: Mixture) -> np.ndarray:
    return mixture.sample(n, _rng(seed))


def radius_for_count(c: float, n: int) -> float:
    """delta with expected c reports per query over n uniform points."""
    return math.sqrt(c / (math.pi * n))


def loguniform(rng: np.random.Generator, lo: float, hi: float, size: int) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def density_radii(q: np.ndarray, n: int, seed: int, c_lo: float = 1.0, c_hi: float = 1000.0,
                  mixture: Mixture | None = None) -> np.ndarray:
    """delta per query such that the expected output is c ~ logU[c_lo, c_hi]
    (density 1 when ``mixture`` is None)."""
    rng = _rng(seed)
    c = loguniform(rng, c_lo, c_hi, q.shape[0])
    f = np.ones(q.shape[0]) if mixture is None else mixture.density(q)
    return np.sqrt(c / (math.pi * n * f))


# ---- named workloads --------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    points: np.ndarray       # (n, 2) float64
    queries: np.ndarray      # (m, 2) float64
    delta: np.ndarray        # (m,) float64
    curve: int               # 0 Z-order, 1 Hilbert


def uniform_fixed_radius(n: int = 1 << 16, m: int = 10_000, curve: int = 0,
                         expected: float = 10.0, seed: int = 1) -> Workload:
    """Uniform points and queries, one radius giving ``expected`` reports."""
    pts = uniform_points(n, 1000 + seed)
    q = uniform_points(m, 2000 + seed)
    d = np.full(m, radius_for_count(expected, n))
    return Workload(f"uniform_n{n}_m{m}_fixed", pts, q, d, curve)


def clustered_loguniform(n: int = 1 << 24, m: int = 1 << 20, curve: int = 1,
                         seed: int = 2, c_lo: float = 1.0, c_hi: float = 1000.0) -> Workload:
    """80% of the points from 16 Gaussians (sigma 0.01), 20% uniform; queries
    from the same mixture; delta aimed at an output log-uniform in
    [c_lo, c_hi]."""
    mix = make_mixture(500 + seed)
    pts = clustered_points(n, 1000 + seed, mix)
    q = clustered_points(m, 2000 + seed, mix)
    d = density_radii(q, n, 3000 + seed, c_lo, c_hi, mix)
    return Workload(f"clustered_n{n}_m{m}_loguniform", pts, q, d, curve)


def clustered_uniform_queries(n: int = 1 << 26, m: int = 1 << 22, curve: int = 0,
                              seed: int = 3, expected: float = 10.0) -> Workload:
    """Clustered points as above; uniform queries with one radius aimed at
    ``expected`` reports at unit density."""
    mix = make_mixture(500 + seed)
    pts = clustered_points(n, 1000 + seed, mix)
    q = uniform_points(m, 2000 + seed)
    d = np.full(m, radius_for_count(expected, n))
    return Workload(f"clustered_n{n}_m{m}_uniformq", pts, q, d, curve)


def square_windows(n: int = 10_000_000, m: int = 1_000_000, side: float = 1e-3, curve: int = 0,
                   seed: int = 6, points: str = "uniform") -> Workload:
    """The experiments' query shape (Sec. 4): uniform centres and square
    windows whose side is ``side`` times the side of the domain (delta =
    side / 2, the half side; the domain is the unit square); uniform,
    normal (the paper's query experiments) or clustered points."""
    if points == "uniform":
        pts = uniform_points(n, 1000 + seed)
    elif points == "normal":
        pts = normal_points(n, 1000 + seed)
    elif points == "clustered":
        pts = clustered_points(n, 1000 + seed, make_mixture(500 + seed))
    else:
        raise ValueError("points must be 'uniform', 'normal' or 'clustered'")
    q = uniform_points(m, 2000 + seed)
    d = np.full(m, side / 2)
    return Workload(f"{points}_n{n}_m{m}_window{side:g}", pts, q, d, curve)


def clustered3(n: int = 1 << 24, m: int = 1 << 20, seed: int = 9, c_lo: float = 1.0,
               c_hi: float = 300.0, frac: float = 0.8, sigma: float = 0.02,
               k: int = 16) -> Workload:
    """Three dimensions: a fraction ``frac`` of the points from k isotropic
    Gaussians (uniform centres, standard deviation sigma), the rest uniform in
    [0,1)^3, clamped and shuffled; queries from the same mixture, delta aimed
    at c ~ logU[c_lo, c_hi] reports: delta = (3 c / (4 pi n f(q)))^(1/3) with
    f the mixture's analytic density.  curve is 2 (d = 3 Morton)."""
    rng = _rng(1000 + seed)
    centres = _rng(500 + seed).random((k, 3))

    def sample(cnt, r):
        nc = (int(round(frac * 1000)) * cnt) // 1000
        comp = r.integers(0, k, nc)
        pc = centres[comp] + sigma * r.standard_normal((nc, 3))
        p = np.concatenate([pc, r.random((cnt - nc, 3))], axis=0)
        np.clip(p, 0.0, ONE_BELOW, out=p)
        return p[r.permutation(cnt)]

    pts = sample(n, rng)
    q = sample(m, _rng(2000 + seed))
    d2 = ((q[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    g = np.exp(-d2 / (2.0 * sigma ** 2)) / (2.0 * math.pi * sigma ** 2) ** 1.5
    f = (1.0 - frac) + (frac / k) * g.sum(1)
    c = loguniform(_rng(3000 + seed), c_lo, c_hi, m)
    d = np.cbrt(3.0 * c / (4.0 * math.pi * n * f))
    return Workload(f"clustered3_n{n}_m{m}_loguniform", pts, q, d, 2)


@dataclasses.dataclass
class BatchedWorkload:
    name: str
    points: np.ndarray       # (N, 2) concatenated
    set_off: np.ndarray      # (S+1,) uint64
    queries: np.ndarray      # (M, 2)
    delta: np.ndarray        # (M,)
    qset: np.ndarray         # (M,) uint32, queries grouped by set
    curve: int


def batched_uneven(n_sets: int = 256, log2_n: tuple = (10, 20), log2_m: tuple = (8, 16),
                   curve: int = 0, seed: int = 4, c_lo: float = 1.0,
                   c_hi: float = 1000.0) -> BatchedWorkload:
    """Independent sets with sizes round(2^U[log2_n]) and query counts
    round(2^U[log2_m]); each set uniform or clustered by a fair coin."""
    rng = _rng(4000 + seed)
    ns = np.rint(2.0 ** rng.uniform(*log2_n, n_sets)).astype(np.int64)
    ms = np.rint(2.0 ** rng.uniform(*log2_m, n_sets)).astype(np.int64)
    coin = rng.integers(0, 2, n_sets)
    pts, qs, ds, qset = [], [], [], []
    for s in range(n_sets):
        if coin[s]:
            mix = make_mixture(10_000 + 3 * s)
            p = clustered_points(int(ns[s]), 10_001 + 3 * s, mix)
            q = clustered_points(int(ms[s]), 10_002 + 3 * s, mix)
        else:
            mix = None
            p = uniform_points(int(ns[s]), 10_001 + 3 * s)
            q = uniform_points(int(ms[s]), 10_002 + 3 * s)
        pts.append(p)
        qs.append(q)
        ds.append(density_radii(q, int(ns[s]), 20_000 + s, c_lo, c_hi, mix))
        qset.append(np.full(int(ms[s]), s, np.uint32))
    set_off = np.zeros(n_sets + 1, np.uint64)
    set_off[1:] = np.cumsum(ns)
    return BatchedWorkload(f"batched_{n_sets}sets", np.concatenate(pts), set_off,
                           np.concatenate(qs), np.concatenate(ds), np.concatenate(qset), curve)


# ---- serving trace ------------------------------------------------------------

QUERY, INSERT, ERASE = 0, 1, 2


@dataclasses.dataclass
class ServingTrace:
    """A request stream over an initial point set.  Request r has a kind, a
    size and the start of its payload in the pool of its kind; gaps are
    Exp(1) inter-arrival draws (a Poisson process once divided by the
    rate).  Erase payloads are ids live at that point of the stream, drawn
    uniformly without replacement (ids: 0..n0-1 for the initial points, then
    consecutive ids per insert in stream order)."""
    name: str
    initial: np.ndarray      # (n0, 2)
    kind: np.ndarray         # (R,) int8
    size: np.ndarray         # (R,) int64
    start: np.ndarray        # (R,) int64, offset into the kind's pool
    gaps: np.ndarray         # (R,) float64
    queries: np.ndarray      # (Mq, 2)
    delta: np.ndarray        # (Mq,)
    inserts: np.ndarray      # (Mi, 2)
    erase_ids: np.ndarray    # (Me,) uint32
    curve: int


def serving_trace(n0: int = 1 << 25, requests: int = 2000, seed: int = 5, curve: int = 0,
                  mix: tuple = (0.4, 0.4, 0.2), log2_size: tuple = (10, 16),
                  c_lo: float = 1.0, c_hi: float = 1000.0) -> ServingTrace:
    """Clustered initial points; query, insert and erase requests in the
    proportions ``mix`` with sizes round(2^U[log2_size]); queries and
    inserted points from the same mixture, radii aimed at an output
    log-uniform in [c_lo, c_hi] over the live count at that point."""
    rng = _rng(5000 + seed)
    mixture = make_mixture(500 + seed)
    initial = clustered_points(n0, 1000 + seed, mixture)
    kind = rng.choice(3, size=requests, p=np.asarray(mix, np.float64)).astype(np.int8)
    size = np.rint(2.0 ** rng.uniform(*log2_size, requests)).astype(np.int64)
    gaps = rng.exponential(1.0, requests)
    start = np.zeros(requests, np.int64)
    tot = [0, 0, 0]
    for r in range(requests):
        start[r] = tot[kind[r]]
        tot[kind[r]] += size[r]
    queries = clustered_points(tot[QUERY], 2000 + seed, mixture)
    inserts = clustered_points(tot[INSERT], 3000 + seed, mixture)
    # The live id set, simulated along the stream (swap-remove array).
    live = np.empty(n0 + tot[INSERT], np.int64)
    live[:n0] = np.arange(n0)
    count, next_id = n0, n0
    erase_ids = np.empty(tot[ERASE], np.uint32)
    live_at_query = np.empty(tot[QUERY], np.int64)
    for r in range(requests):
        k = int(size[r])
        if kind[r] == INSERT:
            live[count:count + k] = np.arange(next_id, next_id + k)
            count += k
            next_id += k
        elif kind[r] == ERASE:
            k = min(k, count)
            size[r] = k
            pos = rng.choice(count, size=k, replace=False)
            erase_ids[start[r]:start[r] + k] = live[pos]
            new_count = count - k
            holes = pos[pos < new_count]
            tail = np.arange(new_count, count)
            keep_tail = tail[~np.isin(tail, pos)]
            live[holes] = live[keep_tail]
            count = new_count
        else:
            live_at_query[start[r]:start[r] + k] = count
    delta = np.empty(tot[QUERY])
    c = loguniform(_rng(4000 + seed), c_lo, c_hi, tot[QUERY])
    delta[:] = np.sqrt(c / (math.pi * np.maximum(live_at_query, 1) * mixture.density(queries)))
    return ServingTrace(f"serving_n{n0}_r{requests}", initial, kind, size, start, gaps, queries,
                        delta, inserts, erase_ids, curve)

"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws input series.  It holds none of the symbolic
approximation's arithmetic, so both the CPU oracle (under ``oracle/``) and
the HIP path are fed from it without sharing any of the method.

Every series is drawn from its own ``PCG64`` stream seeded with
``SeedSequence([seed, workload_id, series_id])`` and z-normalised on the host
(population standard deviation) before being handed, bit-identical, to both
sides.  The paper's own workloads are Gaussian blobs, the UEA multivariate
archive and N(0,1) noise (Sec. 7); the archive is not available here, so the
generators below stand in for it with random walks, sinusoid mixtures and
noisy piecewise-linear signals of the same scale.

Workloads:

1. ``tiny``        16 random walks x 1,000 points, one domain per series,
                   tol = alpha = 0.1.
2. ``scale``       4,096 series x 10,000 points in equal thirds (random walk,
                   3-sinusoid mix + N(0, 0.1^2), piecewise linear with 5..50
                   knots + N(0, 0.05^2)); 1,000-interval domains,
                   tol = alpha = 0.05.
3. ``uneven``      50,000 series, length log-uniform in [100, 100,000], same
                   three-way mix; 2,000-interval domains, tol = alpha = 0.05.
4. ``multivar``    1,024 samples x 64 channels x 5,000 points; channel =
                   0.7 * shared walk + 0.3 * own walk, each channel
                   z-normalised; one domain per channel, tol = alpha = 0.02.
5. ``serving``     request stream: Poisson arrivals, 1..256 random walks per
                   request, length log-uniform in [500, 50,000]; compressed at
                   tol = 0.05 with 2,000-interval domains and encoded against
                   the dictionary built from workload 1.

Points for the Gaussian-blob experiment (Sec. 7.1) come from
``gaussian_blobs``: N 2-D points around ``centers`` centers drawn uniformly
in [-box, box]^2 with isotropic deviation ``std``, each coordinate
z-normalised.  The paper does not state its blob parameters; one centre
reproduces its serial cluster counts (Table 2) within a few per cent.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "series_rng",
    "random_walk",
    "sine_mix",
    "piecewise_linear",
    "znorm",
    "pack",
    "gaussian_blobs",
    "BLOBS_ID",
    "make_workload",
    "WORKLOADS",
    "Request",
    "request_stream",
    "request_pool",
]


def series_rng(seed: int, workload_id: int, series_id: int) -> np.random.Generator:
    """Independent stream per (seed, workload, series)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, workload_id, series_id])))


def random_walk(rng: np.random.Generator, n: int) -> np.ndarray:
    """Cumulative sum of N(0, 1) steps."""
    return np.cumsum(rng.standard_normal(n))


def sine_mix(rng: np.random.Generator, n: int) -> np.ndarray:
    """Three unit-amplitude sinusoids, periods U[20, 500], phases U[0, 2pi), + N(0, 0.1^2)."""
    periods = rng.uniform(20.0, 500.0, 3)
    phases = rng.uniform(0.0, 2.0 * math.pi, 3)
    i = np.arange(n, dtype=np.float64)
    s = np.zeros(n)
    for p, f in zip(periods, phases):
        s += np.sin(2.0 * math.pi * i / p + f)
    return s + rng.normal(0.0, 0.1, n)


def piecewise_linear(rng: np.random.Generator, n: int) -> np.ndarray:
    """5..50 distinct interior knots, N(0,1) knot values (ends included), + N(0, 0.05^2)."""
    if n < 3:
        return rng.standard_normal(n)
    k = int(rng.integers(5, 51))
    k = min(k, n - 2)
    knots = np.sort(rng.choice(np.arange(1, n - 1), size=k, replace=False))
    xs = np.concatenate(([0], knots, [n - 1])).astype(np.float64)
    vals = rng.standard_normal(xs.size)
    return np.interp(np.arange(n, dtype=np.float64), xs, vals) + rng.normal(0.0, 0.05, n)


def znorm(x: np.ndarray) -> np.ndarray:
    """(x - mean) / std with the population std; a constant series is only centred."""
    m = x.mean() if x.size else 0.0
    s = x.std() if x.size else 0.0
    return (x - m) / s if s > 0 else x - m


BLOBS_ID = 8  # generator stream id of the Gaussian-blob points


def gaussian_blobs(seed: int, n: int, centers: int = 1, std: float = 1.0, box: float = 10.0,
                   normalise: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """n points (x, y) around `centers` random centres; coordinates z-normalised when `normalise`."""
    rng = series_rng(seed, BLOBS_ID, 0)
    c = rng.uniform(-box, box, (centers, 2))
    pick = rng.integers(0, centers, n)
    p = c[pick] + rng.normal(0.0, std, (n, 2))
    x, y = np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1])
    if normalise:
        x, y = znorm(x), znorm(y)
    return x, y


def pack(series: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate series into (values f64[total], series_off i64[n_series + 1])."""
    off = np.zeros(len(series) + 1, dtype=np.int64)
    if series:
        off[1:] = np.cumsum([s.size for s in series])
    vals = np.concatenate(series).astype(np.float64) if series else np.zeros(0)
    return np.ascontiguousarray(vals), off


_MIX = (random_walk, sine_mix, piecewise_linear)


@dataclass
class Workload:
    name: str
    workload_id: int
    values: np.ndarray
    series_off: np.ndarray
    D: int
    tol: float
    alpha: float
    scl: float = 1.0
    max_len: int = 0
    B: int = 4096
    meta: dict = field(default_factory=dict)

    @property
    def n_series(self) -> int:
        return int(self.series_off.size - 1)

    @property
    def n_points(self) -> int:
        return int(self.values.size)


def _tiny(seed: int, scale: float) -> Workload:
    n_series = max(1, int(round(16 * scale)))
    ser = [znorm(random_walk(series_rng(seed, 1, s), 1000)) for s in range(n_series)]
    v, off = pack(ser)
    return Workload("tiny", 1, v, off, D=999, tol=0.1, alpha=0.1)


def _scale(seed: int, scale: float) -> Workload:
    n_series = max(3, int(round(4096 * scale)))
    ser = []
    for s in range(n_series):
        gen = _MIX[(3 * s) // n_series]
        ser.append(znorm(gen(series_rng(seed, 2, s), 10_000)))
    v, off = pack(ser)
    return Workload("scale", 2, v, off, D=1000, tol=0.05, alpha=0.05)


def _uneven(seed: int, scale: float) -> Workload:
    n_series = max(3, int(round(50_000 * scale)))
    ser = []
    for s in range(n_series):
        rng = series_rng(seed, 3, s)
        n = int(math.floor(math.exp(rng.uniform(math.log(100.0), math.log(100_000.0)))))
        gen = _MIX[(3 * s) // n_series]
        ser.append(znorm(gen(rng, n)))
    v, off = pack(ser)
    return Workload("uneven", 3, v, off, D=2000, tol=0.05, alpha=0.05)


def _multivar(seed: int, scale: float) -> Workload:
    n_samples = max(1, int(round(1024 * scale)))
    n_ch, n = 64, 5000
    ser = []
    for smp in range(n_samples):
        rng = series_rng(seed, 4, smp)
        w = random_walk(rng, n)
        for _c in range(n_ch):
            ser.append(znorm(0.7 * w + 0.3 * random_walk(rng, n)))
    v, off = pack(ser)
    return Workload("multivar", 4, v, off, D=n - 1, tol=0.02, alpha=0.02,
                    meta={"samples": n_samples, "channels": n_ch})


WORKLOADS = {1: _tiny, 2: _scale, 3: _uneven, 4: _multivar}


def make_workload(workload_id: int, seed: int = 0, scale: float = 1.0) -> Workload:
    """Build workload 1..4; ``scale`` shrinks the series count for quick tests."""
    return WORKLOADS[workload_id](seed, scale)


@dataclass
class Request:
    rid: int
    arrival_s: float
    values: np.ndarray
    series_off: np.ndarray


def _request_body(seed: int, r: int, max_series: int, min_len: int, max_len: int):
    rng = series_rng(seed, 5, r + 1)
    ns = int(rng.integers(1, max_series + 1))
    ser = []
    for _ in range(ns):
        n = int(math.floor(math.exp(rng.uniform(math.log(min_len), math.log(max_len)))))
        ser.append(znorm(random_walk(rng, n)))
    return pack(ser)


def request_stream(seed: int, n_requests: int, rate_hz: float, max_series: int = 256,
                   min_len: int = 500, max_len: int = 50_000, first_id: int = 0,
                   pool: list[tuple[np.ndarray, np.ndarray]] | None = None) -> list[Request]:
    """Poisson arrivals (exponential gaps at ``rate_hz``); 1..max_series random walks each.

    With ``pool`` (bodies from ``request_pool``) request r carries body
    r mod len(pool) instead of freshly drawn series, so long request streams
    need no more host memory than the pool."""
    out = []
    t = 0.0
    arr = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5, 0x5EED])))
    for r in range(first_id, first_id + n_requests):
        t += float(arr.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        v, off = pool[r % len(pool)] if pool else _request_body(seed, r, max_series, min_len, max_len)
        out.append(Request(r, t, v, off))
    return out


def request_pool(seed: int, n_bodies: int, max_series: int = 256, min_len: int = 500,
                 max_len: int = 50_000) -> list[tuple[np.ndarray, np.ndarray]]:
    """n_bodies request bodies (values, series_off) drawn as request_stream draws them."""
    return [_request_body(seed, r, max_series, min_len, max_len) for r in range(n_bodies)]

"""Seeded synthetic inputs for the hull workloads.

This module holds data generation only -- none of the method's arithmetic --
and is the one piece shared by the GPU path's tests/benchmarks and the CPU
oracle's tests.  Every generator draws from numpy ``Generator(PCG64(seed))`` in
float64 and quantizes to the 2^-20 grid:

    k = clip(floor(v * 2^20), 0, 2^20 - 1);   x = float32(k) * 2^-20

Points are interleaved float32 (x, y) pairs, shape (n, 2), C-contiguous.

The paper evaluates an "average case" (normal distribution) and a "worst case"
(points on a circumference) without giving their parameters (Sec. IV); the
parameters below are this project's choices and are listed in the design
notes.  Large inputs are drawn in fixed-size chunks (``CHUNK`` points); the
chunking is part of the recipe, so a given (n, seed) always yields the same
array.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GRID = 1 << 20
CHUNK = 1 << 22

KINDS = ("uniform", "normal", "annulus")


def quantize(v: np.ndarray) -> np.ndarray:
    """float64 values -> float32 on the 2^-20 grid inside [0, 1)."""
    k = np.floor(v * GRID)
    np.clip(k, 0, GRID - 1, out=k)
    return (k.astype(np.float32) * np.float32(1.0 / GRID)).astype(np.float32)


def _fill(n: int, rng: np.random.Generator, draw) -> np.ndarray:
    out = np.empty((n, 2), np.float32)
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        out[lo:hi] = quantize(draw(rng, hi - lo))
    return out


def uniform(n: int, seed: int = 0) -> np.ndarray:
    """Uniform in [0,1)^2."""
    return _fill(n, np.random.Generator(np.random.PCG64(seed)), lambda r, c: r.random((c, 2)))


def normal(n: int, seed: int = 1, mean: float = 0.5, sigma: float = 0.1) -> np.ndarray:
    """Bivariate normal, independent axes, clipped into [0,1) by quantization."""
    return _fill(n, np.random.Generator(np.random.PCG64(seed)),
                 lambda r, c: r.normal(mean, sigma, (c, 2)))


def annulus(n: int, seed: int = 2, r0: float = 0.499, r1: float = 0.5) -> np.ndarray:
    """Uniform angle, area-uniform radius in [r0, r1], centred at (0.5, 0.5).
    Per chunk: theta for the whole chunk first, then the radii."""
    def draw(r, c):
        th = r.uniform(0.0, 2.0 * math.pi, c)
        rad = np.sqrt(r.uniform(r0 * r0, r1 * r1, c))
        return np.stack([0.5 + rad * np.cos(th), 0.5 + rad * np.sin(th)], axis=1)
    return _fill(n, np.random.Generator(np.random.PCG64(seed)), draw)


def by_kind(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "uniform":
        return uniform(n, seed)
    if kind == "normal":
        return normal(n, seed)
    if kind == "annulus":
        return annulus(n, seed)
    if kind == "annulus_wide":
        return annulus(n, seed, 0.49, 0.5)
    raise ValueError(kind)


# The single-set configurations: (name, kind, n, seed).
SINGLE = {
    "uniform_1e6": ("uniform", 1_000_000, 0),
    "normal_1e8": ("normal", 100_000_000, 1),
    "annulus_1e8": ("annulus", 100_000_000, 2),
    "uniform_1e8": ("uniform", 100_000_000, 5),
}


_DESCRIBE = {
    "uniform": "uniform in [0,1)^2",
    "normal": "normal mean 0.5 sigma 0.1 per axis, clipped to [0,1)",
    "annulus": "annulus 0.499-0.5 about (0.5, 0.5), uniform angle, area-uniform radius",
}


def describe(name: str) -> str:
    """One line saying what a single-set workload is."""
    kind, n, _ = SINGLE[name]
    return f"{_DESCRIBE[kind]}, {n} float32 points on the 2^-20 grid"


def seed_of(name: str) -> int:
    return SINGLE[name][2]


def single(name: str, n: int | None = None) -> np.ndarray:
    """One of the single-set workloads, optionally at a reduced size n (same
    kind and seed; the first n points of the reduced draw, not of the full one)."""
    kind, n0, seed = SINGLE[name]
    return by_kind(kind, n0 if n is None else n, seed)


def batch_sets(nsets: int = 4096, seed: int = 3, lo: float = 1e3, hi: float = 1e6,
               scale: float = 1.0):
    """Independent point sets of log-uniform size, each of a kind drawn
    uniformly from {uniform, normal, wide annulus 0.49-0.5}.

    Returns (xy (N,2) float32 concatenated, offsets uint64[nsets+1], kinds list).
    ``scale`` shrinks every size (for small test batches)."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(nsets)
    sizes = np.empty(nsets, np.int64)
    kinds = []
    for s, ch in enumerate(children):
        r = np.random.Generator(np.random.PCG64(ch))
        sizes[s] = max(0, int(math.floor(math.exp(r.uniform(math.log(lo), math.log(hi))) * scale)))
        kinds.append(("uniform", "normal", "annulus_wide")[int(r.integers(0, 3))])
    off = np.zeros(nsets + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    xy = np.empty((int(off[-1]), 2), np.float32)

    def fill(s):
        sub = int(children[s].generate_state(1)[0])
        a, b = int(off[s]), int(off[s + 1])
        xy[a:b] = by_kind(kinds[s], b - a, sub)

    # Every set has its own generator, so filling them in parallel threads
    # gives the same array as filling them in order.
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(nsets)))
    return xy, off, kinds


def serve_trace(rate_hz: float, duration_s: float, seed: int = 4, lo: float = 1e2,
                hi: float = 1e7, max_requests: int | None = None):
    """Poisson arrivals: (arrival times in s, sizes, kinds, per-request seeds)."""
    r = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    times, sizes, kinds, seeds = [], [], [], []
    while True:
        t += float(r.exponential(1.0 / rate_hz))
        if t >= duration_s or (max_requests is not None and len(times) >= max_requests):
            break
        times.append(t)
        sizes.append(int(math.floor(math.exp(r.uniform(math.log(lo), math.log(hi))))))
        kinds.append(("uniform", "normal", "annulus_wide")[int(r.integers(0, 3))])
        seeds.append(int(r.integers(0, 2**31 - 1)))
    return np.array(times), np.array(sizes, np.int64), kinds, seeds

"""Closed-form point sets used by the GPU parity tests (no method arithmetic)."""
import math

import numpy as np


def lattice_circle(r: int, centre: int = 1 << 19):
    rel = []
    for x in range(-r, r + 1):
        y2 = r * r - x * x
        y = math.isqrt(y2)
        if y * y == y2:
            rel.append((x, y))
            if y:
                rel.append((x, -y))
    return [(centre + x, centre + y) for x, y in rel]


def convex_lattice_polygon(m: int):
    """All primitive vectors of the box [-m, m]^2 chained in angular order: a
    polygon whose every vertex is strict (consecutive edge directions differ)."""
    vecs = [(a, b) for a in range(-m, m + 1) for b in range(-m, m + 1)
            if (a, b) != (0, 0) and math.gcd(abs(a), abs(b)) == 1]
    vecs.sort(key=lambda v: math.atan2(v[1], v[0]))
    pts = []
    x = y = 0
    for a, b in vecs:
        pts.append((x, y))
        x += a
        y += b
    assert (x, y) == (0, 0)
    mx = min(p[0] for p in pts)
    my = min(p[1] for p in pts)
    return [(p[0] - mx, p[1] - my) for p in pts]


def to_xy(pts) -> np.ndarray:
    a = np.asarray(pts, dtype=np.int64).reshape(-1, 2)
    return (a.astype(np.float32) * np.float32(2.0 ** -20)).astype(np.float32)

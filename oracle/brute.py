"""Brute-force geometry in plain Python integers, for tiny inputs only.

TEST INFRASTRUCTURE, independent of ``oracle.c``: these routines restate the
definitions (not the algorithms) and are what the oracle is pinned against.

* ``hull_brute``   -- the convex hull by its definition (Sec. I: the smallest
  convex set holding S; its vertices are the extreme points).  A directed pair
  a -> b of distinct points is a hull edge when every other point lies strictly
  to its left or strictly inside the segment.  O(n^3); the paper's Table I
  lists an O(n^4) brute force, this is the edge-test variant.
* ``extremes_keys`` -- the 8 octagon vertices as argmax of linear keys over
  x, y, x+y, x-y (an algebraic restatement of the Manhattan-corner search,
  valid because every point lies inside the box of the axis extremes).
* ``keep_winding`` -- the discard rule of Sec. I (inside the octagon or on a
  side without being a vertex) restated with a winding number and an
  on-segment test instead of half-plane signs.
"""
from __future__ import annotations


def orient(a, b, c) -> int:
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def _strictly_between(a, b, c) -> bool:
    """c on the open segment (a, b), assuming a, b, c collinear."""
    return (min(a[0], b[0]) <= c[0] <= max(a[0], b[0]) and
            min(a[1], b[1]) <= c[1] <= max(a[1], b[1]) and c != a and c != b)


def hull_brute(pts: list[tuple[int, int]]) -> list[int]:
    """Counter-clockwise strict hull vertices from the lexicographic minimum,
    each as the smallest index holding its coordinates."""
    rep: dict[tuple[int, int], int] = {}
    for i, p in enumerate(pts):
        rep.setdefault(tuple(p), i)
    u = sorted(rep)
    if not u:
        return []
    if len(u) == 1:
        return [rep[u[0]]]
    nxt: dict[tuple[int, int], tuple[int, int]] = {}
    for a in u:
        for b in u:
            if a == b:
                continue
            ok = True
            for c in u:
                if c == a or c == b:
                    continue
                o = orient(a, b, c)
                if o < 0 or (o == 0 and not _strictly_between(a, b, c)):
                    ok = False
                    break
            if ok:
                nxt[a] = b
    start = u[0]
    out = [start]
    cur = nxt[start]
    while cur != start:
        out.append(cur)
        cur = nxt[cur]
    return [rep[p] for p in out]


# Slot keys: (primary, tie-break) maximised lexicographically, tie-break being
# the direction turned 90 degrees counter-clockwise.
_KEYS = (
    lambda x, y: (x, y),            # E
    lambda x, y: (x + y, y - x),    # NE
    lambda x, y: (y, -x),           # N
    lambda x, y: (y - x, -x - y),   # NW
    lambda x, y: (-x, -y),          # W
    lambda x, y: (-x - y, x - y),   # SW
    lambda x, y: (-y, x),           # S
    lambda x, y: (x - y, x + y),    # SE
)


def extremes_keys(pts) -> list[tuple[int, int]]:
    """The 8 vertex coordinates by direct argmax of the slot keys."""
    return [max(pts, key=lambda p, f=f: f(*p)) for f in _KEYS]


def _winding(p, poly) -> int:
    w = 0
    n = len(poly)
    for i in range(n):
        a, b = poly[i], poly[(i + 1) % n]
        if a[1] <= p[1]:
            if b[1] > p[1] and orient(a, b, p) > 0:
                w += 1
        else:
            if b[1] <= p[1] and orient(a, b, p) < 0:
                w -= 1
    return w


def _on_segment(p, a, b) -> bool:
    if orient(a, b, p) != 0:
        return False
    return (min(a[0], b[0]) <= p[0] <= max(a[0], b[0]) and
            min(a[1], b[1]) <= p[1] <= max(a[1], b[1]))


def keep_winding(p, verts) -> bool:
    """True when p survives the octagon filter with vertices ``verts``."""
    p = tuple(p)
    if p in [tuple(v) for v in verts]:
        return True
    n = len(verts)
    if any(_on_segment(p, verts[i], verts[(i + 1) % n]) for i in range(n)):
        return False
    return _winding(p, verts) == 0

"""Pins for the CPU oracle (runs without a GPU).

The oracle is checked against things other than itself: the brute-force
definition of the hull, an argmax-of-keys restatement of the extremes, a
winding-number restatement of the discard rule, closed cases whose hull is
known in closed form, hand-worked fixtures under tests/golden/, invariants of
any convex hull, scipy's Qhull on general-position data, and a battery showing
that planted mistakes (a transposed operand, a dropped term, a reversed
tie-break, ...) are caught.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2209_12310_amd import workloads
from tests._util import golden_names, grid_to_xy, load_golden


def setup_module(_):
    oracle.build()


def _rand_small(rng, n, span):
    return [(int(rng.integers(0, span)), int(rng.integers(0, span))) for _ in range(n)]


# ------------------------------------------------------------------ domain

def test_domain_accepts_grid_values():
    xy = np.array([[0.0, 0.0], [1 - 2 ** -20, 0.5], [2 ** -20, 0.25]], np.float32)
    kx, ky = oracle.to_grid(xy)
    assert kx.tolist() == [0, (1 << 20) - 1, 1]
    assert ky.tolist() == [0, 1 << 19, 1 << 18]


def test_domain_negative_zero_is_zero():
    kx, ky = oracle.to_grid(np.array([[-0.0, 0.5]], np.float32))
    assert kx.tolist() == [0]


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf"), 1.0, -2 ** -20,
                                 2 ** -21, 0.5 + 2 ** -22, 3.0])
def test_domain_rejects(bad):
    xy = np.array([[0.25, 0.25], [0.5, bad], [0.75, 0.75]], np.float32)
    with pytest.raises(oracle.DomainError) as e:
        oracle.to_grid(xy)
    assert e.value.index == 1


# ---------------------------------------------------------------- extremes

def test_extremes_match_key_argmax():
    rng = np.random.default_rng(10)
    for trial in range(200):
        n = int(rng.integers(1, 40))
        pts = _rand_small(rng, n, int(rng.integers(1, 9)))
        kx = np.array([p[0] for p in pts], np.int32)
        ky = np.array([p[1] for p in pts], np.int32)
        idx = oracle.extremes(kx, ky)
        got = [(int(kx[i]), int(ky[i])) for i in idx]
        assert got == brute.extremes_keys(pts), (trial, pts)
        for k, i in enumerate(idx):  # smallest index holding the coordinates
            assert pts.index(got[k]) == i


def test_extremes_full_grid():
    k = 7
    pts = [(x, y) for y in range(k) for x in range(k)]
    kx = np.array([p[0] for p in pts], np.int32)
    ky = np.array([p[1] for p in pts], np.int32)
    idx = oracle.extremes(kx, ky)
    got = [pts[i] for i in idx]
    m = k - 1
    assert got == [(m, m), (m, m), (0, m), (0, m), (0, 0), (0, 0), (m, 0), (m, 0)]


# ------------------------------------------------------------------ filter

def test_filter_matches_winding_rule():
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(1, 50))
        pts = _rand_small(rng, n, int(rng.integers(2, 12)))
        kx = np.array([p[0] for p in pts], np.int32)
        ky = np.array([p[1] for p in pts], np.int32)
        surv, lab = oracle.filter(kx, ky)
        verts = brute.extremes_keys(pts)
        want = [j for j, p in enumerate(pts) if brute.keep_winding(p, verts)]
        assert surv.tolist() == want, (trial, pts)
        assert ((lab > 0) == np.isin(np.arange(n), want)).all()
        assert lab.max(initial=0) <= 4


def test_filter_full_grid_keeps_corners_only():
    k = 9
    pts = [(x, y) for x in range(k) for y in range(k)] + [(0, 0), (k - 1, k - 1)]
    kx = np.array([p[0] for p in pts], np.int32)
    ky = np.array([p[1] for p in pts], np.int32)
    surv, _ = oracle.filter(kx, ky)
    corners = {(0, 0), (k - 1, 0), (k - 1, k - 1), (0, k - 1)}
    assert surv.tolist() == [j for j, p in enumerate(pts) if p in corners]


@pytest.mark.parametrize("kind", workloads.KINDS)
def test_filter_keeps_every_hull_vertex(kind):
    xy = workloads.by_kind(kind, 200_000, 5)
    kx, ky = oracle.to_grid(xy)
    surv, _ = oracle.filter(kx, ky)
    plain = oracle.chain(kx, ky)
    assert np.isin(plain, surv).all()


@pytest.mark.parametrize("nthreads", [1, 2, 3, 8])
def test_parallel_filter_equals_sequential(nthreads):
    xy = workloads.normal(300_001, 7)
    kx, ky = oracle.to_grid(xy)
    oct_seq = oracle.extremes(kx, ky)
    surv_seq, _ = oracle.filter(kx, ky, oct_seq)
    oct_par, surv_par = oracle.filter_parallel(kx, ky, nthreads)
    assert oct_par.tolist() == oct_seq.tolist()
    assert np.array_equal(surv_par, surv_seq)


def test_normal_filter_rate_sanity():
    """Sec. IV reports more than 99.99% of normal points filtered on average and
    99.87% at 10^4 points; a sanity check, not a pin (the paper's sigma is not
    given)."""
    kx, ky = oracle.to_grid(workloads.normal(1_000_000, 1))
    surv, _ = oracle.filter(kx, ky)
    assert surv.size / kx.size < 1e-3


# -------------------------------------------------------------------- hull

def test_hull_matches_brute_force():
    rng = np.random.default_rng(12)
    for trial in range(300):
        n = int(rng.integers(0, 45))
        pts = _rand_small(rng, n, int(rng.integers(1, 10)))
        want = brute.hull_brute(pts)
        kx = np.array([p[0] for p in pts], np.int32)
        ky = np.array([p[1] for p in pts], np.int32)
        assert oracle.chain(kx, ky).tolist() == want, (trial, pts)
        assert oracle.heaphull(kx, ky).tolist() == want, (trial, pts)


def test_hull_brute_force_wide_coordinates():
    rng = np.random.default_rng(13)
    for trial in range(60):
        n = int(rng.integers(3, 40))
        pts = _rand_small(rng, n, 1 << 20)
        kx = np.array([p[0] for p in pts], np.int32)
        ky = np.array([p[1] for p in pts], np.int32)
        assert oracle.heaphull(kx, ky).tolist() == brute.hull_brute(pts)


@pytest.mark.parametrize("name", golden_names())
def test_golden_fixture(name):
    g = load_golden(name)
    xy = grid_to_xy(g["points"])
    kx, ky = oracle.to_grid(xy)
    o = oracle.octagon(xy)
    assert o["kx"].tolist() == g["octagon_kx"]
    assert o["ky"].tolist() == g["octagon_ky"]
    assert o["idx"].tolist() == g["octagon_idx"]
    surv, lab = oracle.filter(kx, ky)
    assert surv.tolist() == g["survivors"]
    assert lab.tolist() == g["labels"]
    assert oracle.hull(xy).tolist() == g["hull"]
    assert brute.hull_brute(g["points"]) == g["hull"]


def _lattice_circle(r):
    pts = []
    for x in range(-r, r + 1):
        y2 = r * r - x * x
        y = math.isqrt(y2)
        if y * y == y2:
            pts.append((x, y))
            if y:
                pts.append((x, -y))
    return pts


def test_lattice_circle_all_on_hull():
    r = 5 * 13 * 17 * 29  # 4 * 3^4 = 324 lattice points on x^2 + y^2 = r^2
    rel = _lattice_circle(r)
    assert len(rel) == 324
    c = 1 << 19
    pts = [(c + x, c + y) for x, y in rel]
    perm = np.random.default_rng(14).permutation(len(pts))
    pts = [pts[i] for i in perm]
    xy = grid_to_xy(pts)
    got = oracle.hull(xy).tolist()
    ang = [math.atan2(p[1] - c, p[0] - c) for p in pts]
    order = sorted(range(len(pts)), key=lambda i: ang[i])
    start = order.index(min(range(len(pts)), key=lambda i: pts[i]))
    want = order[start:] + order[:start]
    assert got == want


def test_parabola_all_on_hull():
    pts = [(i, i * i) for i in range(1024)]
    perm = np.random.default_rng(15).permutation(1024)
    shuffled = [pts[i] for i in perm]
    got = oracle.hull(grid_to_xy(shuffled)).tolist()
    inv = np.argsort(perm)
    assert got == inv.tolist()


def test_full_grid_hull_is_square():
    k = 50
    pts = [(x, y) for x in range(k) for y in range(k)]
    got = oracle.hull(grid_to_xy(pts)).tolist()
    m = k - 1
    assert [pts[i] for i in got] == [(0, 0), (m, 0), (m, m), (0, m)]


def test_square_boundary_with_edge_points():
    pts = [(x, 0) for x in range(0, 101, 10)] + [(100, y) for y in range(0, 101, 5)]
    pts += [(x, 100) for x in range(0, 101, 4)] + [(0, y) for y in range(0, 101, 20)]
    got = oracle.hull(grid_to_xy(pts)).tolist()
    assert [pts[i] for i in got] == [(0, 0), (100, 0), (100, 100), (0, 100)]
    assert got == [0, 10, 31, 32]


def test_collinear_with_duplicates():
    pts = [(x, 2 * x + 3) for x in (5, 1, 9, 9, 1, 4, 7)]
    assert oracle.hull(grid_to_xy(pts)).tolist() == [1, 2]


def test_degenerate_sizes():
    assert oracle.hull(np.zeros((0, 2), np.float32)).tolist() == []
    assert oracle.hull(grid_to_xy([(3, 4)])).tolist() == [0]
    assert oracle.hull(grid_to_xy([(3, 4), (3, 4)])).tolist() == [0]
    assert oracle.hull(grid_to_xy([(9, 4), (3, 4)])).tolist() == [1, 0]
    assert oracle.hull(grid_to_xy([(5, 5)] * 17)).tolist() == [0]


def _orient_np(ax, ay, bx, by, px, py):
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax)


@pytest.mark.parametrize("kind,n", [("uniform", 100_000), ("normal", 100_000), ("annulus", 50_000)])
def test_hull_invariants(kind, n):
    xy = workloads.by_kind(kind, n, 21)
    kx, ky = oracle.to_grid(xy)
    x = kx.astype(np.int64)
    y = ky.astype(np.int64)
    hull = oracle.hull(xy)
    h = hull.size
    assert h >= 3
    hx, hy = x[hull], y[hull]
    # starts at the lexicographic minimum
    lex = np.lexsort((y, x))[0]
    assert (hx[0], hy[0]) == (x[lex], y[lex])
    # containment: every point on the inner side of every edge
    for i in range(h):
        j = (i + 1) % h
        assert (_orient_np(hx[i], hy[i], hx[j], hy[j], x, y) >= 0).all()
    # strict convexity and counter-clockwise turns
    for i in range(h):
        a, b, c = i, (i + 1) % h, (i + 2) % h
        assert _orient_np(hx[a], hy[a], hx[b], hy[b], hx[c], hy[c]) > 0
    # each vertex carries the smallest index holding its coordinates
    for v in hull:
        assert np.flatnonzero((x == x[v]) & (y == y[v]))[0] == v
    # the hull of the hull is the hull
    sub = oracle.hull(xy[hull])
    assert sub.tolist() == list(range(h))


def test_permutation_invariance():
    xy = workloads.uniform(20_000, 22)
    kx, ky = oracle.to_grid(xy)
    assert np.unique(kx.astype(np.int64) << 20 | ky).size == kx.size  # no duplicates
    base = oracle.hull(xy)
    perm = np.random.default_rng(23).permutation(xy.shape[0])
    got = perm[oracle.hull(xy[perm])]
    assert got.tolist() == base.tolist()


def test_matches_qhull_general_position():
    from scipy.spatial import ConvexHull
    for seed in range(5):
        xy = workloads.uniform(2_000, 100 + seed)
        got = oracle.hull(xy)
        qh = ConvexHull(xy.astype(np.float64))
        assert set(got.tolist()) == set(qh.vertices.tolist())


@pytest.mark.parametrize("name", list(workloads.SINGLE))
def test_heaphull_equals_plain_chain(name):
    xy = workloads.single(name, 300_000)
    kx, ky = oracle.to_grid(xy)
    assert np.array_equal(oracle.heaphull(kx, ky), oracle.chain(kx, ky))


# ------------------------------------------- the four queues of Alg. 1

def _queues(pts):
    kx = np.array([p[0] for p in pts], np.int32)
    ky = np.array([p[1] for p in pts], np.int32)
    _, lab = oracle.filter(kx, ky)
    return kx, ky, lab


def test_queue_heaphull_matches_brute_force():
    """Alg. 1 with its four queues (a hull per queue, then the union) gives
    the brute-force hull on small sets full of duplicates, collinear runs and
    coinciding extremes."""
    rng = np.random.default_rng(31)
    for trial in range(400):
        n = int(rng.integers(1, 45))
        pts = _rand_small(rng, n, int(rng.integers(1, 10)))
        kx, ky, lab = _queues(pts)
        got, qc = oracle.heaphull_queues(kx, ky, lab)
        assert got.tolist() == brute.hull_brute(pts), (trial, pts)
        assert qc.tolist() == [int((lab == q).sum()) for q in (1, 2, 3, 4)]


@pytest.mark.parametrize("case", ["grid", "circle", "parabola", "collinear", "identical", "two",
                                  "square_sides", "diagonal", "vertical"])
def test_queue_heaphull_closed_cases(case):
    c = 1 << 19
    pts = {
        "grid": [(x, y) for x in range(20) for y in range(20)],
        "circle": [(c + x, c + y) for x, y in _lattice_circle(5 * 13 * 17 * 29)],
        "parabola": [(i, i * i) for i in range(1024)],
        "collinear": [(x, 2 * x + 3) for x in (5, 1, 9, 9, 1, 4, 7)],
        "identical": [(7, 7)] * 9,
        "two": [(1, 2), (3, 4), (1, 2)],
        "square_sides": [(x, 0) for x in range(0, 101, 10)] + [(100, y) for y in range(0, 101, 5)]
        + [(x, 100) for x in range(0, 101, 4)] + [(0, y) for y in range(0, 101, 20)],
        "diagonal": [(x, x) for x in range(50)],
        "vertical": [(9, y) for y in range(40)],
    }[case]
    perm = np.random.default_rng(32).permutation(len(pts))
    pts = [pts[i] for i in perm]
    kx, ky, lab = _queues(pts)
    got, _ = oracle.heaphull_queues(kx, ky, lab)
    assert got.tolist() == oracle.heaphull(kx, ky).tolist()
    if len(pts) <= 60:
        assert got.tolist() == brute.hull_brute(pts)


@pytest.mark.parametrize("name", golden_names())
def test_queue_heaphull_golden(name):
    g = load_golden(name)
    kx, ky = oracle.to_grid(grid_to_xy(g["points"]))
    got, _ = oracle.heaphull_queues(kx, ky, np.asarray(g["labels"], np.uint8))
    assert got.tolist() == g["hull"]


@pytest.mark.parametrize("kind", ["uniform", "normal", "annulus"])
def test_parallel_heaphull_equals_sequential(kind):
    xy = workloads.by_kind(kind, 300_000, 33)
    kx, ky = oracle.to_grid(xy)
    want = oracle.heaphull(kx, ky)
    _, lab = oracle.filter(kx, ky)
    for t in (1, 3, 8):
        assert np.array_equal(oracle.heaphull_parallel(kx, ky, t), want), t
        assert np.array_equal(oracle.chain_parallel(kx, ky, None, t), want), t
        assert np.array_equal(oracle.heaphull_queues(kx, ky, lab, None, t)[0], want), t


def test_native_build_matches():
    """The -O3 -march=native copy timed as the CPU baseline computes the same
    hulls (same source, planted-mistake switch compiled out)."""
    nat = oracle.native()
    for kind in ("uniform", "annulus"):
        xy = workloads.by_kind(kind, 100_000, 34)
        kx, ky = oracle.to_grid(xy)
        want = oracle.heaphull(kx, ky)
        assert np.array_equal(nat.heaphull(kx, ky), want)
        assert np.array_equal(nat.heaphull_parallel(kx, ky), want)


# ----------------------------------------------------- planted mistakes bite

def _battery() -> list[str]:
    """Run a compact set of the pins above; return the names that failed."""
    failed = []
    for name in golden_names():
        g = load_golden(name)
        xy = grid_to_xy(g["points"])
        kx, ky = oracle.to_grid(xy)
        surv, lab = oracle.filter(kx, ky)
        o = oracle.octagon(xy)
        if (surv.tolist() != g["survivors"] or lab.tolist() != g["labels"]
                or o["kx"].tolist() != g["octagon_kx"] or o["ky"].tolist() != g["octagon_ky"]
                or oracle.hull(xy).tolist() != g["hull"]):
            failed.append("golden:" + name)
    rng = np.random.default_rng(99)
    for trial in range(60):
        pts = _rand_small(rng, int(rng.integers(3, 30)), int(rng.integers(2, 8)))
        kx = np.array([p[0] for p in pts], np.int32)
        ky = np.array([p[1] for p in pts], np.int32)
        if oracle.heaphull(kx, ky).tolist() != brute.hull_brute(pts):
            failed.append("brute_hull")
            break
        _, lab = oracle.filter(kx, ky)
        if oracle.heaphull_queues(kx, ky, lab)[0].tolist() != brute.hull_brute(pts):
            failed.append("queue_hull")
            break
        idx = oracle.extremes(kx, ky)
        if [pts[i] for i in idx] != brute.extremes_keys(pts):
            failed.append("extremes_keys")
            break
        verts = brute.extremes_keys(pts)
        surv, _ = oracle.filter(kx, ky)
        if surv.tolist() != [j for j, p in enumerate(pts) if brute.keep_winding(p, verts)]:
            failed.append("winding")
            break
    return failed


def test_battery_passes_unmutated():
    oracle.set_mutation(0)
    assert _battery() == []


@pytest.mark.parametrize("mutation", range(1, 10))
def test_planted_mistake_is_caught(mutation):
    try:
        oracle.set_mutation(mutation)
        assert _battery() != [], f"mutation {mutation} went unnoticed"
    finally:
        oracle.set_mutation(0)

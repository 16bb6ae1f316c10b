"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every comparison is exact (tolerance 0): hull indices, survivor lists,
labels and octagons are integers decided by exact predicates on both sides.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2209_12310_amd import workloads
from tests._shapes import convex_lattice_polygon, lattice_circle, to_xy
from tests._util import golden_names, grid_to_xy, load_golden

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2209_12310_amd as ch
    c = ch.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _dev(xy):
    import torch
    return torch.from_numpy(np.ascontiguousarray(xy, np.float32)).to("cuda:0")


def _say(msg):
    print(msg, flush=True)


def _check_filter(ctx, xy, t=None, labels=True):
    kx, ky = oracle.to_grid(xy)
    want_s, want_l = oracle.filter(kx, ky)
    t = _dev(xy) if t is None else t
    fr = ctx.filter(t, labels=labels, octagon=True)
    got_s = fr.survivors.cpu().numpy().view(np.uint32)
    assert fr.count == want_s.size
    assert np.array_equal(got_s, want_s)
    if labels:
        assert np.array_equal(fr.labels.cpu().numpy(), want_l)
    if xy.shape[0]:
        o = oracle.octagon(xy)
        assert fr.octagon["kx"].tolist() == o["kx"].tolist()
        assert fr.octagon["ky"].tolist() == o["ky"].tolist()
        assert fr.octagon["idx"].tolist() == o["idx"].tolist()
    return fr


def _check_hull(ctx, xy, t=None):
    want = oracle.hull(xy)
    got = ctx.hull(_dev(xy) if t is None else t)
    assert np.array_equal(got, want), (got[:20], want[:20])
    return got


# ------------------------------------------------------------ small cases

@pytest.mark.parametrize("name", golden_names())
def test_golden(ctx, name):
    _say(f"golden {name}")
    g = load_golden(name)
    xy = grid_to_xy(g["points"])
    fr = ctx.filter(_dev(xy), labels=True, octagon=True)
    assert fr.survivors.cpu().numpy().view(np.uint32).tolist() == g["survivors"]
    assert fr.labels.cpu().numpy().tolist() == g["labels"]
    assert fr.octagon["kx"].tolist() == g["octagon_kx"]
    assert fr.octagon["ky"].tolist() == g["octagon_ky"]
    assert fr.octagon["idx"].tolist() == g["octagon_idx"]
    assert ctx.hull(_dev(xy)).tolist() == g["hull"]


def test_degenerate_sizes(ctx):
    _say("degenerate sizes")
    import torch
    empty = torch.zeros((0, 2), dtype=torch.float32, device="cuda:0")
    assert ctx.hull(empty).tolist() == []
    assert ctx.filter(empty).count == 0
    for pts in ([(3, 4)], [(3, 4), (3, 4)], [(9, 4), (3, 4)], [(5, 5)] * 17, [(1, 1), (2, 2), (3, 3)]):
        xy = grid_to_xy(pts)
        _check_filter(ctx, xy)
        assert ctx.hull(_dev(xy)).tolist() == brute.hull_brute(pts)


def test_random_tiny_sets_vs_brute_force(ctx):
    _say("random tiny sets")
    rng = np.random.default_rng(31)
    for trial in range(150):
        n = int(rng.integers(1, 60))
        span = int(rng.integers(1, 12))
        pts = [(int(rng.integers(0, span)), int(rng.integers(0, span))) for _ in range(n)]
        xy = grid_to_xy(pts)
        assert ctx.hull(_dev(xy)).tolist() == brute.hull_brute(pts), (trial, pts)
        _check_filter(ctx, xy)


def test_closed_cases(ctx):
    _say("closed cases")
    k = 100
    grid = [(x, y) for x in range(k) for y in range(k)]
    got = ctx.hull(_dev(grid_to_xy(grid)))
    assert [grid[i] for i in got] == [(0, 0), (k - 1, 0), (k - 1, k - 1), (0, k - 1)]
    _check_filter(ctx, grid_to_xy(grid))
    circ = lattice_circle(5 * 13 * 17 * 29)
    perm = np.random.default_rng(32).permutation(len(circ))
    xy = to_xy([circ[i] for i in perm])
    assert ctx.hull(_dev(xy)).size == 324
    _check_hull(ctx, xy)
    par = [(i, i * i) for i in range(1024)]
    xy = to_xy([par[i] for i in np.random.default_rng(33).permutation(1024)])
    assert ctx.hull(_dev(xy)).size == 1024
    _check_hull(ctx, xy)
    line = [(x, 2 * x + 3) for x in np.random.default_rng(34).integers(0, 100000, 5000).tolist()]
    assert ctx.hull(_dev(to_xy(line))).size == 2
    _check_hull(ctx, to_xy(line))


@pytest.mark.parametrize("n", [2, 3, 255, 256, 4095, 4096, 4097, 8191, 8192, 8193, 12345, 65537])
@pytest.mark.parametrize("kind", workloads.KINDS)
def test_ragged_sizes(ctx, kind, n):
    _say(f"ragged {kind} n={n}")
    xy = workloads.by_kind(kind, n, 40 + n % 7)
    _check_filter(ctx, xy)
    _check_hull(ctx, xy)


@pytest.mark.parametrize("kind", workloads.KINDS)
def test_unaligned_points(ctx, kind):
    """A view starting 8 bytes into an allocation (not 16-byte aligned)."""
    _say(f"unaligned {kind}")
    xy = workloads.by_kind(kind, 100_001, 41)
    full = _dev(xy)
    view = full[1:]
    assert view.data_ptr() % 16 == 8
    _check_filter(ctx, xy[1:], view)
    _check_hull(ctx, xy[1:], view)


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), 1.0, -2 ** -20, 2 ** -21, 7.0])
def test_domain_errors(ctx, bad):
    _say(f"domain {bad}")
    import paper_2209_12310_amd as ch
    xy = workloads.uniform(50_000, 42)
    for pos in (0, 12_345, 49_999):
        bad_xy = xy.copy()
        bad_xy[pos, pos % 2] = np.float32(bad)
        t = _dev(bad_xy)
        with pytest.raises(ch.DomainError):
            ctx.filter(t)
        with pytest.raises(ch.DomainError):
            ctx.hull(t)
    _check_hull(ctx, xy)  # the context recovers


def test_capacity_error(ctx):
    _say("capacity")
    import paper_2209_12310_amd as ch
    xy = to_xy(lattice_circle(5 * 13 * 17 * 29))
    with pytest.raises(ch.CapacityError):
        ctx.hull(_dev(xy), cap=10)


# ------------------------------------------------------ large-hull path

def test_strictly_convex_polygon_many_vertices(ctx):
    """~24k vertices in strictly convex position: no tile round can shrink
    the list, so the column table and windowed chains produce the hull."""
    _say("convex polygon m=100")
    poly = convex_lattice_polygon(100)
    rng = np.random.default_rng(35)
    pts = [poly[i] for i in rng.permutation(len(poly))]
    xy = to_xy(pts)
    got = _check_hull(ctx, xy)
    assert got.size == len(poly)


def test_convex_polygon_with_duplicates_and_interior(ctx):
    _say("convex polygon with duplicates")
    poly = convex_lattice_polygon(40)
    xs = [p[0] for p in poly]
    ys = [p[1] for p in poly]
    cx, cy = (min(xs) + max(xs)) // 2, (min(ys) + max(ys)) // 2
    rng = np.random.default_rng(36)
    inner = [(cx + int(a), cy + int(b)) for a, b in rng.integers(-200, 200, (20000, 2))]
    pts = poly * 3 + inner
    pts = [pts[i] for i in rng.permutation(len(pts))]
    _check_hull(ctx, to_xy(pts))


@pytest.mark.parametrize("n", [10_000, 300_000])
def test_dense_annulus_large_hull(ctx, n):
    _say(f"dense annulus {n}")
    xy = workloads.annulus(n, 43)
    _check_hull(ctx, xy)
    _check_filter(ctx, xy)


def test_many_survivors_go_straight_to_large_path(ctx):
    """A ring ten grid units wide, every point twice (the copy at the larger
    index first): most points survive every filter, so the hull pass skips
    the tile rounds and runs the column table on the survivors directly;
    copies still report their smallest index."""
    _say("ring with duplicates, direct large path")
    ring = workloads.annulus(1_000_000, 44, 0.49999, 0.5)
    xy = np.concatenate([ring[::-1], ring])
    _check_hull(ctx, xy)
    info = ctx.last_hull_info()
    assert info["survivors"] > (1 << 18), info
    assert info["large_path"] == 1 and info["rounds"] == 0, info


@pytest.mark.parametrize("wait", ["poll", "stream"])
@pytest.mark.parametrize("case", ["uniform", "ring", "polygon", "parabola"])
def test_tile_round_path(case, wait):
    """The hull path through the tile rounds (CH_LARGE_DIRECT above the
    survivor count, and no second polygon: tile hulls, then a block hull, or
    the large-hull path when a round stops shrinking), with either wait for
    the block hull's result (watching its status word or the stream),
    against the oracle."""
    import os
    import paper_2209_12310_amd as ch
    _say(f"tile round path: {case}, wait {wait}")
    if case == "uniform":
        xy = workloads.uniform(10_000_000, 48)
    elif case == "ring":
        xy = workloads.annulus(300_000, 49)
    elif case == "polygon":
        xy = to_xy(convex_lattice_polygon(60))
    else:
        i = np.arange(20_000, dtype=np.int64)
        xy = to_xy(np.stack([48 * i, (i * i) >> 9], 1))
    old = {k: os.environ.get(k) for k in ("CH_LARGE_DIRECT", "CH_HULL_WAIT", "CH_SECOND_POLY")}
    os.environ["CH_LARGE_DIRECT"] = str(1 << 30)
    os.environ["CH_HULL_WAIT"] = wait
    os.environ["CH_SECOND_POLY"] = "0"
    try:
        c = ch.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    try:
        _check_hull(c, xy)
        info = c.last_hull_info()
        assert info["refined"] == 0, info
        if info["survivors"] > 4096:
            assert info["rounds"] >= 1, info
    finally:
        c.close()


@pytest.mark.parametrize("case", ["uniform", "ring", "wide_ring", "wide_ring_dense", "square_sides",
                                  "polygon", "dup_ring"])
def test_second_polygon(ctx, case):
    """Inputs whose survivors are too many for one workgroup: the second
    polygon from the survivors drops those strictly inside it, then the block
    hull, the rounds or the large-hull path finish; the hull equals the
    oracle's. A lattice square's whole boundary, many points in convex
    position, and every point twice are included."""
    _say(f"second polygon: {case}")
    if case == "uniform":
        xy = workloads.uniform(30_000_000, 51)
    elif case == "ring":
        xy = workloads.annulus(2_000_000, 52)
    elif case == "wide_ring":
        xy = workloads.annulus(1_000_000, 53, 0.3, 0.5)
    elif case == "wide_ring_dense":
        xy = workloads.annulus(8_000_000, 57, 0.49, 0.5)
    elif case == "square_sides":
        rng = np.random.default_rng(54)
        side = 30000
        t = np.arange(side)
        lo = 5000
        edge = np.concatenate([
            np.stack([lo + t, np.full(side, lo)], 1), np.stack([np.full(side, lo + side), lo + t], 1),
            np.stack([lo + side - t, np.full(side, lo + side)], 1), np.stack([np.full(side, lo), lo + side - t], 1)])
        inner = rng.integers(lo + 1, lo + side, (400_000, 2))
        pts = np.concatenate([edge, inner])
        xy = to_xy(pts[rng.permutation(len(pts))])
    elif case == "polygon":
        rng = np.random.default_rng(55)
        poly = np.asarray(convex_lattice_polygon(60), np.int64) + 3000
        c = (poly.min(0) + poly.max(0)) // 2
        inner = rng.integers(-3000, 3000, (300_000, 2)) + c
        pts = np.concatenate([poly, inner])
        xy = to_xy(pts[rng.permutation(len(pts))])
    else:
        ring = workloads.annulus(500_000, 56, 0.4999, 0.5)
        xy = np.concatenate([ring[::-1], ring])
    _check_hull(ctx, xy)
    info = ctx.last_hull_info()
    # The second polygon runs exactly when one workgroup (4096 records)
    # cannot take the survivors and there are at most 2^18 of them; these
    # two always are in that range (the square's side points already fall to
    # the octagon test, the rings keep more).
    assert (info["refined"] > 0) == (4096 < info["survivors"] <= 1 << 18), info
    assert info["refined"] <= info["survivors"], info
    if case in ("polygon", "wide_ring_dense"):
        assert info["refined"] > 0, info


def test_max_points(ctx):
    """CH_MAX_POINTS = 2^31 - 1 points (17 GB of input, ~112 GB of workspace):
    uniform interior points strictly inside the grid square, its four corners
    at the largest indices (the last one the odd tail point), and a second
    copy of one corner at index 5. The hull is known by construction: the
    corners, counter-clockwise from the lexicographic minimum, the duplicated
    one reported by its smaller index."""
    import torch
    from paper_2209_12310_amd import _capi
    n = _capi.CH_MAX_POINTS
    _say(f"max points n={n}: generating on the device")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(47)
    k = torch.randint(1, (1 << 20) - 1, (n, 2), dtype=torch.int32, device="cuda:0", generator=g)
    top = (1 << 20) - 1
    corners = torch.tensor([[0, 0], [0, 0], [top, 0], [top, top], [0, top]], dtype=torch.int32,
                           device="cuda:0")
    k[5] = corners[0]
    k[n - 4:] = corners[1:]
    xy = k.to(torch.float32).mul_(2.0 ** -20)
    del k
    torch.cuda.synchronize()
    _say("max points: hull")
    got = ctx.hull(xy)
    assert got.tolist() == [5, n - 3, n - 2, n - 1]
    info = ctx.last_hull_info()
    assert info["n"] == n and info["h"] == 4
    del xy
    ctx._ws = None
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_read_stream_diagnostic(ctx):
    """The diagnostic read stream runs on a device buffer and rejects a
    length that is not a multiple of 16 bytes."""
    import ctypes
    import torch
    from paper_2209_12310_amd import _capi
    _say("read stream diagnostic")
    buf = torch.zeros(1 << 20, dtype=torch.float32, device="cuda:0")
    assert ctx.read_stream_async(buf) == 4 << 20
    assert ctx.read_stream_async(buf, 7) == 4 << 20
    torch.cuda.synchronize()
    st = ctx._lib.ch_diag_read_stream(ctx._h, ctypes.c_void_p(buf.data_ptr()), 24, 0,
                                      ctx.stream_handle())
    assert st == _capi.CH_E_INVALID_ARG


# --------------------------------------------------- workload configurations

@pytest.mark.parametrize("name", list(workloads.SINGLE))
def test_configs_reduced(ctx, name):
    for n in (1_000, 100_000, 1_000_000):
        _say(f"config {name} n={n}")
        xy = workloads.single(name, n)
        _check_filter(ctx, xy)
        _check_hull(ctx, xy)


def test_uniform_1e6_full(ctx):
    _say("uniform_1e6 full")
    xy = workloads.single("uniform_1e6")
    _check_filter(ctx, xy)
    _check_hull(ctx, xy)


@pytest.mark.parametrize("name", ["normal_1e8", "annulus_1e8", "uniform_1e8"])
def test_full_size(ctx, name):
    """Full 10^8-point configurations: complete survivor list and hull."""
    _say(f"full {name}: generating")
    xy = workloads.single(name)
    t = _dev(xy)
    _say(f"full {name}: oracle")
    kx, ky = oracle.to_grid(xy)
    oct_idx, want_s = oracle.filter_parallel(kx, ky, 0)
    want_h = oracle.chain(kx, ky, want_s)
    _say(f"full {name}: gpu (survivors={want_s.size}, h={want_h.size})")
    got_h = ctx.hull(t)
    assert np.array_equal(got_h, want_h)
    # the single read used the sample polygon, with the inner region and
    # grid its data call for (bit 1: octagon, else disc; bit 2: whole grid)
    mode = ctx.last_hull_info()["single_read"]
    assert mode & 1
    assert bool(mode & 2) == (name == "uniform_1e8"), mode
    if name != "uniform_1e8":
        assert bool(mode & 4) == (name == "annulus_1e8"), mode
    fr = ctx.filter(t, octagon=True)
    assert fr.count == want_s.size
    assert np.array_equal(fr.survivors.cpu().numpy().view(np.uint32), want_s)
    assert fr.octagon["kx"].tolist() == kx[oct_idx].tolist()
    assert fr.octagon["ky"].tolist() == ky[oct_idx].tolist()
    if name == "normal_1e8":
        assert want_s.size / xy.shape[0] < 1e-4  # Sec. IV: > 99.99% filtered


def test_repeatable(ctx):
    _say("repeatable")
    xy = workloads.annulus(200_000, 44)
    t = _dev(xy)
    first = ctx.hull(t)
    s0 = ctx.filter(t).survivors.cpu().numpy()
    for _ in range(20):
        assert np.array_equal(ctx.hull(t), first)
        assert np.array_equal(ctx.filter(t).survivors.cpu().numpy(), s0)

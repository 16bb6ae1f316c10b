"""GPU parity of the hull path's refined filter (the sample polygon): inputs
large enough to build it (ch_hull from 2^17 points, batch sets from 2^15)
whose structure stresses it -- copies of sample points at smaller indices,
points on the polygon's sides, points in convex position, degenerate
samples, domain errors at sampled positions. Every hull is compared with
the oracle's, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2209_12310_amd import workloads
from tests._shapes import convex_lattice_polygon, lattice_circle, to_xy

pytestmark = pytest.mark.gpu

SAMPLE_MIN = 1 << 17
BATCH_SAMPLE_MIN = 1 << 15


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


def _grid(pts):
    return to_xy(np.asarray(pts, np.int64))


def _square_boundary_with_interior(n, side, seed):
    """Every lattice point on the boundary of a square, the rest strictly
    inside it, shuffled: the sample polygon's sides carry many input points."""
    rng = np.random.default_rng(seed)
    lo = 1000
    t = np.arange(side)
    edge = np.concatenate([
        np.stack([lo + t, np.full(side, lo)], 1), np.stack([np.full(side, lo + side), lo + t], 1),
        np.stack([lo + side - t, np.full(side, lo + side)], 1), np.stack([np.full(side, lo), lo + side - t], 1)])
    inner = rng.integers(lo + 1, lo + side, (n - len(edge), 2))
    pts = np.concatenate([edge, inner])
    return _grid(pts[rng.permutation(len(pts))])


def _cases(scale_min, m=60):
    """Inputs of scale_min + 4321 points (or about that); m sets the size of
    the strictly convex lattice polygon (about 0.6 (2m+1)^2 vertices)."""
    rng = np.random.default_rng(81)
    n = scale_min + 4321
    ann = workloads.annulus(n // 2, 82, 0.49, 0.5)
    poly = np.asarray(convex_lattice_polygon(m), np.int64) + 5000
    c = (poly.min(0) + poly.max(0)) // 2
    half = int(0.3 * (poly.max() - poly.min()))
    inner = rng.integers(-half, half, (n, 2)) + c
    convex = np.concatenate([poly, inner])
    k = np.arange(n) % 100000
    line = np.stack([7 * k, 3 * k + 11], 1)
    circle = np.asarray(lattice_circle(5 * 13 * 17 * 29), np.int64)
    circ_inner = rng.integers(-22000, 22000, (n, 2)) + (1 << 19)
    # points on rays from the centre (through the polygon's vertices and
    # their wedge boundaries), to the ray ends, which are the hull
    dirs = np.array([(1, 0), (3, 1), (2, 1), (1, 1), (1, 2), (1, 3), (0, 1), (-1, 3), (-1, 1),
                     (-3, 1), (-1, 0), (-2, -1), (-1, -1), (-1, -2), (0, -1), (1, -1), (3, -2)])
    reps = n // len(dirs) + 1
    t = np.arange(1, reps + 1) * (60000 // reps + 1) // 8
    rays = ((1 << 19) + dirs[:, None, :] * t[None, :, None]).reshape(-1, 2)[:n]
    return {
        "rays": _grid(rays[rng.permutation(len(rays))]),
        # every point twice; the copy at the smaller index is the one reported
        "reversed_duplicates": np.concatenate([ann[::-1], ann]),
        "square_sides": _square_boundary_with_interior(n, 4096, 83),
        "convex_position": _grid(convex[rng.permutation(len(convex))]),
        "collinear": _grid(line[rng.permutation(n)]),
        "identical": _grid(np.full((n, 2), 777)),
        "two_points": _grid(np.where((np.arange(n) % 5 == 0)[:, None], [[10, 20]], [[30000, 40]])),
        "circle_lattice": _grid(np.concatenate([circ_inner, circle])),
        "annulus_thin": workloads.annulus(n, 84),
        "normal": workloads.normal(n, 85),
    }


CASES = list(_cases(SAMPLE_MIN))


@pytest.mark.parametrize("name", CASES)
def test_hull_refined(ctx, name):
    _say(f"refined {name}")
    xy = _cases(SAMPLE_MIN)[name]
    assert xy.shape[0] >= SAMPLE_MIN
    want = oracle.hull(xy)
    assert np.array_equal(ctx.hull(_dev(xy)), want)


@pytest.mark.parametrize("n", [SAMPLE_MIN - 1, SAMPLE_MIN, SAMPLE_MIN + 1])
def test_threshold_sizes(ctx, n):
    _say(f"refined threshold {n}")
    for kind in ("annulus_wide", "uniform"):
        xy = workloads.by_kind(kind, n, 86)
        assert np.array_equal(ctx.hull(_dev(xy)), oracle.hull(xy))


@pytest.mark.parametrize("where", [0, 8, "sampled", "last"])
def test_domain_error_at_sampled_points(ctx, where):
    """A sample point outside the domain is skipped by the sampler; pass 1
    still reports the call's domain error."""
    _say(f"refined domain error at {where}")
    import paper_2209_12310_amd as ch
    n = SAMPLE_MIN + 999
    xy = workloads.annulus(n, 87, 0.49, 0.5)
    i = {"sampled": (5 * n) // 16384, "last": n - 1}.get(where, where)
    xy[i, 1] = np.float32(np.nan)
    with pytest.raises(ch.DomainError):
        ctx.hull(_dev(xy))


@pytest.mark.parametrize("kind", ["normal", "uniform"])
@pytest.mark.parametrize("where", [1, 4097, "middle", "second_last", "last"])
def test_domain_error_inside_polygon(ctx, where, kind):
    """Off-grid values deep inside the data (inside the sample polygon's
    inner region -- its disc for normal data, its octagon for the uniform
    square -- where the single-read pass skips the extreme keys) still give
    the call's domain error: half a grid step and a sixteenth of one."""
    import paper_2209_12310_amd as ch
    n = SAMPLE_MIN + 999
    base = workloads.by_kind(kind, n, 95)
    i = {"middle": n // 2, "second_last": n - 2, "last": n - 1}.get(where, where)
    for off in (2.0 ** -21, 2.0 ** -24):
        _say(f"refined domain error inside the polygon ({kind}) at {where}, offset {off}")
        xy = base.copy()
        xy[i] = (np.float32(0.5 + off), np.float32(0.5))
        with pytest.raises(ch.DomainError):
            ctx.hull(_dev(xy))
    # the same inputs on the grid are accepted
    xy = base.copy()
    xy[i] = (np.float32(0.5), np.float32(0.5))
    assert np.array_equal(ctx.hull(_dev(xy)), oracle.hull(xy))


def test_batch_refined(ctx):
    _say("refined batch")
    import torch
    cases = _cases(BATCH_SAMPLE_MIN)
    sets = list(cases.values()) + [workloads.annulus(BATCH_SAMPLE_MIN - 1, 88, 0.49, 0.5),
                                   workloads.annulus(BATCH_SAMPLE_MIN, 89, 0.49, 0.5)]
    off = np.zeros(len(sets) + 1, np.int64)
    off[1:] = np.cumsum([s.shape[0] for s in sets])
    t = _dev(np.concatenate(sets))
    idx, cnt = ctx.hull_batch(t, torch.from_numpy(off).to("cuda:0"))
    for k, s in enumerate(sets):
        want = oracle.hull(s)
        assert cnt[k] == len(want), k
        assert np.array_equal(idx[off[k]: off[k] + cnt[k]], want), k


def test_fused_path_counts(ctx):
    """The single-read path is taken from 2^17 points and keeps few
    candidates on ring data; below that size, or with a degenerate sample,
    the two-read path runs (no candidates). Hulls match the oracle."""
    _say("refined fused-path counts")
    ring = workloads.annulus(SAMPLE_MIN + 100, 93, 0.49, 0.5)
    assert np.array_equal(ctx.hull(_dev(ring)), oracle.hull(ring))
    info = ctx.last_hull_info()
    assert info["n"] == ring.shape[0] and 0 < info["candidates"] < ring.shape[0] // 10
    assert info["survivors"] <= info["candidates"]
    assert info["single_read"] & 1
    small = workloads.annulus(SAMPLE_MIN - 1, 94, 0.49, 0.5)
    assert np.array_equal(ctx.hull(_dev(small)), oracle.hull(small))
    assert ctx.last_hull_info()["candidates"] == 0
    assert ctx.last_hull_info()["single_read"] == 0
    line = _cases(SAMPLE_MIN)["collinear"]
    assert np.array_equal(ctx.hull(_dev(line)), oracle.hull(line))
    assert ctx.last_hull_info()["candidates"] == 0

"""GPU parity of the paper's own stages (Alg. 1 with its four queues, Alg. 2,
and Sec. III's two-kernel extreme search) through the C ABI, against the CPU
oracle. Every comparison is exact (tolerance 0).

* ch_gpufilter: the label array Q of Alg. 2 and the octagon, with either
  extreme search, equal oracle.filter's labels and oracle.octagon.
* ch_hull_queues: the hull built queue by queue equals oracle.hull (the hull
  is unique, so the queue route must give it exactly), and the queue sizes
  equal the oracle's count of each label.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2209_12310_amd import workloads
from tests._shapes import convex_lattice_polygon, lattice_circle, to_xy
from tests._util import golden_names, grid_to_xy, load_golden

pytestmark = pytest.mark.gpu

MODES = ("two_kernels", "fused")


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


def _want_queues(labels):
    return np.array([(labels == q).sum() for q in (1, 2, 3, 4)], np.uint32)


def _check(ctx, xy, t=None, modes=MODES, labels_too=True):
    """Alg. 2's labels and octagon, and Alg. 1's queue hull, against the
    oracle for each extreme search."""
    t = _dev(xy) if t is None else t
    want_h = oracle.hull(xy)
    kx, ky = oracle.to_grid(xy)
    _, want_l = oracle.filter(kx, ky) if xy.shape[0] else (None, np.zeros(0, np.uint8))
    o = oracle.octagon(xy) if xy.shape[0] else None
    for mode in modes:
        if labels_too:
            lab, octd, cnt = ctx.gpufilter(t, extremes=mode)
            assert np.array_equal(lab.cpu().numpy(), want_l), mode
            assert cnt == int((want_l != 0).sum()), mode
            if o is not None:
                assert octd["kx"].tolist() == o["kx"].tolist(), mode
                assert octd["ky"].tolist() == o["ky"].tolist(), mode
                assert octd["idx"].tolist() == o["idx"].tolist(), mode
        got, qc = ctx.hull_queues(t, extremes=mode)
        assert np.array_equal(got, want_h), (mode, got[:12], want_h[:12])
        assert np.array_equal(qc, _want_queues(want_l)), (mode, qc)
    return want_h


@pytest.mark.parametrize("name", golden_names())
def test_golden(ctx, name):
    """The hand-worked fixtures: labels, octagon and hull."""
    _say(f"queues golden {name}")
    g = load_golden(name)
    xy = grid_to_xy(g["points"])
    t = _dev(xy)
    for mode in MODES:
        lab, octd, _ = ctx.gpufilter(t, extremes=mode)
        assert lab.cpu().numpy().tolist() == g["labels"], mode
        assert octd["kx"].tolist() == g["octagon_kx"], mode
        assert octd["ky"].tolist() == g["octagon_ky"], mode
        assert octd["idx"].tolist() == g["octagon_idx"], mode
        got, _ = ctx.hull_queues(t, extremes=mode)
        assert got.tolist() == g["hull"], mode


def test_degenerate_sizes(ctx):
    _say("queues degenerate sizes")
    import torch
    empty = torch.zeros((0, 2), dtype=torch.float32, device="cuda:0")
    for mode in MODES:
        got, qc = ctx.hull_queues(empty, extremes=mode)
        assert got.tolist() == [] and qc.tolist() == [0, 0, 0, 0]
    for pts in ([(3, 4)], [(3, 4), (3, 4)], [(9, 4), (3, 4)], [(5, 5)] * 17, [(1, 1), (2, 2), (3, 3)],
                [(7, 1), (7, 9), (7, 5)], [(1, 7), (9, 7), (5, 7), (9, 7)], [(0, 0), (5, 5), (0, 5), (5, 0)]):
        xy = grid_to_xy(pts)
        got = _check(ctx, xy)
        assert got.tolist() == brute.hull_brute(pts), pts


def test_random_tiny_sets_vs_brute_force(ctx):
    """Small sets with heavy duplication and collinearity: every extreme may
    coincide with others, and arcs may be empty."""
    _say("queues random tiny sets")
    rng = np.random.default_rng(61)
    for trial in range(120):
        n = int(rng.integers(1, 60))
        span = int(rng.integers(1, 12))
        pts = [(int(rng.integers(0, span)), int(rng.integers(0, span))) for _ in range(n)]
        xy = grid_to_xy(pts)
        t = _dev(xy)
        want = brute.hull_brute(pts)
        for mode in MODES:
            got, _ = ctx.hull_queues(t, extremes=mode)
            assert got.tolist() == want, (trial, mode, pts)
        if trial % 10 == 0:
            _check(ctx, xy, t)


def test_closed_cases(ctx):
    _say("queues closed cases")
    k = 100
    grid = [(x, y) for x in range(k) for y in range(k)]
    got = _check(ctx, grid_to_xy(grid))
    assert [grid[i] for i in got] == [(0, 0), (k - 1, 0), (k - 1, k - 1), (0, k - 1)]
    circ = lattice_circle(5 * 13 * 17 * 29)
    perm = np.random.default_rng(62).permutation(len(circ))
    assert _check(ctx, to_xy([circ[i] for i in perm])).size == 324
    par = [(i, i * i) for i in range(1024)]
    assert _check(ctx, to_xy([par[i] for i in np.random.default_rng(63).permutation(1024)])).size == 1024
    line = [(x, 2 * x + 3) for x in np.random.default_rng(64).integers(0, 100000, 5000).tolist()]
    assert _check(ctx, to_xy(line)).size == 2


def test_convex_polygon_many_vertices(ctx):
    """~24k strict vertices: every queue's arc is thousands of columns long,
    so each queue's chain is built in windows and folded."""
    _say("queues convex polygon m=100")
    poly = convex_lattice_polygon(100)
    rng = np.random.default_rng(65)
    pts = [poly[i] for i in rng.permutation(len(poly))]
    got = _check(ctx, to_xy(pts), labels_too=False)
    assert got.size == len(poly)


@pytest.mark.parametrize("n", [2, 3, 255, 4097, 65537])
@pytest.mark.parametrize("kind", workloads.KINDS)
def test_ragged_sizes(ctx, kind, n):
    _say(f"queues ragged {kind} n={n}")
    _check(ctx, workloads.by_kind(kind, n, 70 + n % 5))


@pytest.mark.parametrize("kind", workloads.KINDS)
def test_unaligned_points(ctx, kind):
    _say(f"queues unaligned {kind}")
    xy = workloads.by_kind(kind, 100_001, 71)
    full = _dev(xy)
    view = full[1:]
    assert view.data_ptr() % 16 == 8
    _check(ctx, xy[1:], view)


@pytest.mark.parametrize("name", list(workloads.SINGLE))
def test_configs_reduced(ctx, name):
    for n in (1_000, 1_000_000):
        _say(f"queues config {name} n={n}")
        _check(ctx, workloads.single(name, n))


def test_annulus_many_survivors(ctx):
    """A thin ring: nearly every point survives the octagon, each queue holds
    a quarter of them, and every column of each arc is occupied."""
    _say("queues thin ring 1e6")
    _check(ctx, workloads.annulus(1_000_000, 72, 0.49999, 0.5))


@pytest.mark.parametrize("bad", [float("nan"), 1.0, 2 ** -21])
def test_domain_errors(ctx, bad):
    _say(f"queues domain {bad}")
    import paper_2209_12310_amd as ch
    xy = workloads.uniform(50_000, 73)
    for pos in (0, 49_999):
        bad_xy = xy.copy()
        bad_xy[pos, pos % 2] = np.float32(bad)
        t = _dev(bad_xy)
        for mode in MODES:
            with pytest.raises(ch.DomainError):
                ctx.gpufilter(t, extremes=mode)
            with pytest.raises(ch.DomainError):
                ctx.hull_queues(t, extremes=mode)
    _check(ctx, xy)  # the context recovers


@pytest.mark.parametrize("name", ["normal_1e8", "annulus_1e8", "uniform_1e8"])
def test_full_size(ctx, name):
    """The 10^8-point configurations: the queue route's hull and queue sizes,
    and the two-kernel octagon, against the oracle."""
    _say(f"queues full {name}: generating")
    xy = workloads.single(name)
    t = _dev(xy)
    _say(f"queues full {name}: oracle")
    kx, ky = oracle.to_grid(xy)
    oct_idx, want_s = oracle.filter_parallel(kx, ky, 0)
    want_h = oracle.chain(kx, ky, want_s)
    _, want_l = oracle.filter(kx, ky, oct_idx)
    want_q = _want_queues(want_l)
    for mode in MODES:
        _say(f"queues full {name}: gpu {mode}")
        got, qc = ctx.hull_queues(t, extremes=mode)
        assert np.array_equal(got, want_h), mode
        assert np.array_equal(qc, want_q), (mode, qc, want_q)
        lab, octd, cnt = ctx.gpufilter(t, extremes=mode)
        assert cnt == want_s.size
        assert np.array_equal(lab.cpu().numpy(), want_l), mode
        assert octd["kx"].tolist() == kx[oct_idx].tolist(), mode
        assert octd["ky"].tolist() == ky[oct_idx].tolist(), mode
        del lab

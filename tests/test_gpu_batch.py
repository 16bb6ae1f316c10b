"""GPU parity of the batched mode: every set's hull from ch_hull_batch equals
the oracle's hull of that set alone (and ch_hull's), bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2209_12310_amd import workloads
from tests._shapes import convex_lattice_polygon, lattice_circle, to_xy

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


def _say(msg):
    print(msg, flush=True)


def _run(ctx, sets):
    import torch
    sizes = [s.shape[0] for s in sets]
    off = np.zeros(len(sets) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    xy = np.concatenate(sets).astype(np.float32) if off[-1] else np.zeros((0, 2), np.float32)
    t = torch.from_numpy(np.ascontiguousarray(xy)).to("cuda:0")
    o = torch.from_numpy(off).to("cuda:0")
    idx, cnt = ctx.hull_batch(t, o)
    return off, idx, cnt


def _check_sets(ctx, sets, expect=None):
    off, idx, cnt = _run(ctx, sets)
    for s, pts in enumerate(sets):
        want = oracle.hull(pts) if expect is None or expect[s] is None else expect[s]
        assert cnt[s] == len(want), (s, pts.shape[0], int(cnt[s]), len(want))
        got = idx[off[s]: off[s] + cnt[s]]
        assert np.array_equal(got, want), s
    return off, idx, cnt


def test_mixed_small_sets(ctx):
    _say("batch mixed small sets")
    rng = np.random.default_rng(50)
    sets = []
    for i in range(97):
        n = int(rng.choice([0, 1, 2, 3, 17, 256, 1000, 4097, 8191, 8193, 30000]))
        kind = workloads.KINDS[i % 3]
        sets.append(workloads.by_kind(kind, n, 100 + i))
    _check_sets(ctx, sets)


@pytest.mark.parametrize("nsets", [1, 255, 256, 257, 513])
def test_set_counts_at_workgroup_boundaries(ctx, nsets):
    """Set counts around multiples of 256 (the plan kernels give each
    workgroup 256 sets and rank them against all the others), with sets
    large enough to get sample polygons and second polygons mixed with
    small and empty ones."""
    _say(f"batch set count {nsets}")
    rng = np.random.default_rng(70 + nsets)
    sets = []
    for i in range(nsets):
        n = int(rng.choice([0, 5, 900, 3000, 9000, 40000]))
        sets.append(workloads.by_kind(("uniform", "normal", "annulus_wide")[i % 3], n, 1000 + i))
    _check_sets(ctx, sets)


def test_batch_equals_solo(ctx):
    _say("batch equals solo")
    import torch
    sets = [workloads.by_kind(k, n, 7 + n) for k in workloads.KINDS for n in (5000, 70000, 250000)]
    off, idx, cnt = _check_sets(ctx, sets)
    for s, pts in enumerate(sets):
        solo = ctx.hull(torch.from_numpy(pts).to("cuda:0"))
        assert np.array_equal(idx[off[s]: off[s] + cnt[s]], solo)


def test_degenerate_sets(ctx):
    _say("batch degenerate sets")
    line = np.array([(x, 3 * x + 1) for x in range(0, 3000, 7)], np.int64)
    sets = [
        to_xy([(5, 5)] * 50),
        to_xy(lattice_circle(5 * 13 * 17 * 29)),
        to_xy(line[np.random.default_rng(1).permutation(len(line))]),
        np.zeros((0, 2), np.float32),
        to_xy([(1, 2), (3, 4)]),
    ]
    _check_sets(ctx, sets)


def test_second_polygon_sets(ctx):
    """Sets with at least 1024 candidates, so each gets a second polygon
    built from its candidates: points on a line, one point repeated, two
    points repeated, a square's whole lattice boundary with interior points
    (points on the polygon's sides), a convex lattice polygon (every point a
    hull vertex), thin and wide rings, a lattice circle with interior
    points, and sets with and without a sample polygon."""
    _say("batch second polygon sets")
    rng = np.random.default_rng(61)
    line = np.array([(x, 2 * x + 5) for x in range(0, 40000, 7)], np.int64)
    side = 3000
    t = np.arange(side)
    edge = np.concatenate([np.stack([10 + t, np.full(side, 10)], 1), np.stack([np.full(side, 10 + side), 10 + t], 1),
                           np.stack([10 + side - t, np.full(side, 10 + side)], 1),
                           np.stack([np.full(side, 10), 10 + side - t], 1)])
    square = np.concatenate([edge, rng.integers(11, 10 + side, (20000, 2))])
    poly = np.asarray(convex_lattice_polygon(25), np.int64) + 100
    circ = np.asarray(lattice_circle(5 * 13 * 17 * 29), np.int64)  # centred at 2^19
    circ_in = np.concatenate([circ, rng.integers(-20000, 20000, (30000, 2)) + (1 << 19)])
    shuf = lambda a: to_xy(a[rng.permutation(len(a))])
    sets = [
        shuf(line),
        to_xy([(77, 99)] * 3000),
        to_xy([(5, 6)] * 1500 + [(900, 4)] * 1500),
        shuf(square),
        shuf(poly),
        workloads.annulus(60_000, 62, 0.4999, 0.5),
        workloads.annulus(9_000, 63, 0.3, 0.5),
        shuf(circ_in),
        workloads.by_kind("uniform", 5000, 64),
    ]
    assert len(poly) > 1024 and len(circ) > 16
    _check_sets(ctx, sets)


def test_domain_error_in_one_set(ctx):
    _say("batch domain error")
    sets = [workloads.uniform(10000, s) for s in range(5)]
    bad = sets[2].copy()
    bad[123, 1] = np.float32(1.5)
    sets[2] = bad
    off, idx, cnt = _run(ctx, sets)
    assert cnt[2] == 0xFFFFFFFF
    for s in (0, 1, 3, 4):
        want = oracle.hull(sets[s])
        assert np.array_equal(idx[off[s]: off[s] + cnt[s]], want)


@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_domain_error_inside_sample_polygon(ctx, where):
    """Off-grid values deep inside large sets (inside their sample polygon's
    inner region, where the single read only runs the grid check) and at
    odd tile ends give those sets a domain error; the other sets keep their
    hulls."""
    _say(f"batch domain error inside the polygon, {where}")
    sets = [workloads.normal(70001 + 3 * s, 40 + s) for s in range(4)]
    for s in (1, 3):
        n = sets[s].shape[0]
        i = {"first": 0, "middle": n // 2, "last": n - 1}[where]
        sets[s] = sets[s].copy()
        sets[s][i] = (np.float32(0.5 + 2.0 ** -23), np.float32(0.5))
    off, idx, cnt = _run(ctx, sets)
    assert cnt[1] == 0xFFFFFFFF and cnt[3] == 0xFFFFFFFF
    for s in (0, 2):
        want = oracle.hull(sets[s])
        assert cnt[s] == len(want)
        assert np.array_equal(idx[off[s]: off[s] + cnt[s]], want)


def test_invalid_offsets(ctx):
    _say("batch invalid offsets")
    import torch
    xy = torch.from_numpy(workloads.uniform(1000, 3)).to("cuda:0")
    off = torch.tensor([0, 600, 400, 1000], dtype=torch.int64, device="cuda:0")
    _, cnt = ctx.hull_batch(xy, off)
    assert (cnt == 0xFFFFFFFD).all()


def test_many_annulus_sets_need_rounds(ctx):
    """Wide-annulus sets keep nearly every point through the octagon, so their
    candidates go through the tile-hull rounds."""
    _say("batch annulus rounds")
    sets = [workloads.by_kind("annulus_wide", n, 60 + i) for i, n in enumerate([20000, 150000, 600000])]
    _check_sets(ctx, sets)


def test_batch_config_scaled(ctx):
    """The batch workload recipe (4096 sets, three kinds, log-uniform sizes),
    every size scaled by 1/20."""
    _say("batch config scaled")
    xy, off, kinds = workloads.batch_sets(4096, 3, scale=0.05)
    sets = [xy[int(off[s]): int(off[s + 1])] for s in range(4096)]
    _check_sets(ctx, sets)


def _mixed_batch(seed, count, hi=80000):
    rng = np.random.default_rng(seed)
    sets = [workloads.by_kind(("uniform", "normal", "annulus_wide")[i % 3], int(n), seed + i)
            for i, n in enumerate(rng.integers(0, hi, count))]
    off = np.zeros(count + 1, np.int64)
    off[1:] = np.cumsum([s.shape[0] for s in sets])
    return sets, off


@pytest.mark.parametrize("params", [
    {"tile_points": 4096, "pass_blocks": 1, "hull_blocks": 1, "sample_min": 0},
    {"tile_points": 65536, "pass_blocks": 7, "hull_blocks": 5, "sample_min": 0xFFFFFFFF},
    {"tile_points": 16384, "pass_blocks": 2048, "hull_blocks": 2048, "sample_min": 40000},
])
def test_launch_parameters_do_not_change_results(ctx, params):
    _say(f"batch params {params}")
    import torch
    sets, off = _mixed_batch(300, 25)
    ctx.set_batch_params(params)
    try:
        assert ctx.batch_params(25, int(off[-1])) == params
        t = torch.from_numpy(np.concatenate(sets)).to("cuda:0")
        idx, cnt = ctx.hull_batch(t, torch.from_numpy(off).to("cuda:0"))
        for s, pts in enumerate(sets):
            assert np.array_equal(idx[off[s]: off[s] + cnt[s]], oracle.hull(pts)), s
    finally:
        ctx.set_batch_params(None)


def test_invalid_launch_parameters(ctx):
    import paper_2209_12310_amd as ch
    for bad in ({"tile_points": 5000, "pass_blocks": 1, "hull_blocks": 1, "sample_min": 0},
                {"tile_points": 2048, "pass_blocks": 1, "hull_blocks": 1, "sample_min": 0},
                {"tile_points": 8192, "pass_blocks": 0, "hull_blocks": 1, "sample_min": 0}):
        with pytest.raises(ch.ConvexHullError):
            ctx.set_batch_params(bad)


def test_tuner_and_cache(tmp_path):
    """The tuner returns valid parameters, leaves the batch's result in the
    outputs, and its cache file gives a new context the same choice."""
    _say("batch tuner")
    import torch
    import paper_2209_12310_amd as ch
    cache = str(tmp_path / "tune.txt")
    sets, off = _mixed_batch(400, 60, 150000)
    n, nsets = int(off[-1]), len(sets)
    t = torch.from_numpy(np.concatenate(sets)).to("cuda:0")
    o = torch.from_numpy(off).to("cuda:0")
    idx = torch.empty(n, dtype=torch.int32, device="cuda:0")
    cnt = torch.empty(nsets, dtype=torch.int32, device="cuda:0")
    c1 = ch.Context(0, tune_cache=cache)
    try:
        best = c1.tune_batch(t, o, idx, cnt)
        torch.cuda.synchronize()
        counts = cnt.cpu().numpy().view(np.uint32)
        hidx = idx.cpu().numpy().view(np.uint32)
        for s, pts in enumerate(sets):
            assert np.array_equal(hidx[off[s]: off[s] + counts[s]], oracle.hull(pts)), s
        assert c1.batch_params(nsets, n) == best
        lines = open(cache).read().split("\n")
        assert any(line.startswith("convhull-tune 1 ") for line in lines)
    finally:
        c1.close()
    c2 = ch.Context(0, tune_cache=cache)
    try:
        assert c2.batch_params(nsets, n) == best
        got_idx, got_cnt = c2.hull_batch(t, o)
        for s, pts in enumerate(sets):
            assert np.array_equal(got_idx[off[s]: off[s] + got_cnt[s]], oracle.hull(pts)), s
    finally:
        c2.close()


def test_batch_4096_full(ctx):
    """The full batch workload (4096 sets, 5.84e8 points): every set's hull
    from one ch_hull_batch call, in the launch configuration the benchmark
    times (tuned parameters), against the oracle set by set."""
    from concurrent.futures import ThreadPoolExecutor

    import torch
    _say("batch_4096 full: generating")
    xy, off, _ = workloads.batch_sets(4096, 3)
    n, nsets = xy.shape[0], off.size - 1
    t = torch.from_numpy(xy).to("cuda:0")
    o = torch.from_numpy(off.astype(np.int64)).to("cuda:0")
    idx = torch.empty(n, dtype=torch.int32, device="cuda:0")
    cnt = torch.empty(nsets, dtype=torch.int32, device="cuda:0")
    ws = ctx.workspace(ctx._lib.ch_hull_batch_workspace_bytes(nsets, n))
    _say("batch_4096 full: tuned call")
    ctx.tune_batch(t, o, idx, cnt, ws)
    idx.fill_(-1)
    ctx.hull_batch_async(t, o, idx, cnt, ws)
    got_c = cnt.cpu().numpy().view(np.uint32)
    got_i = idx.cpu().numpy().view(np.uint32)
    del t, idx
    ctx._ws = None
    torch.cuda.empty_cache()
    _say("batch_4096 full: oracle")

    def one(s):
        a, b = int(off[s]), int(off[s + 1])
        want = oracle.hull(xy[a:b])
        return s, got_c[s] == want.size and np.array_equal(got_i[a: a + want.size], want)

    with ThreadPoolExecutor(max_workers=16) as ex:
        bad = [s for s, ok in ex.map(one, range(nsets)) if not ok]
    assert not bad, bad[:10]

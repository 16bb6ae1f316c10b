"""GPU parity of batch mode on sets whose candidates do not shrink within the
tile-hull rounds (many points in convex position, or close to a smooth
curve): they finish on the device through the per-set column path, and every
set's hull equals the oracle's bit for bit. Also the sampler's chunk counts
(one 2,048-point sample chunk per 131,072 points of a set, up to four) at
their boundaries, and a batch with such sets captured in a HIP graph."""
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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _check(ctx, sets):
    off = np.zeros(len(sets) + 1, np.int64)
    off[1:] = np.cumsum([s.shape[0] for s in sets])
    idx, cnt = ctx.hull_batch(_dev(np.concatenate(sets).astype(np.float32)), _dev(off))
    for s, pts in enumerate(sets):
        want = oracle.hull(pts)
        assert cnt[s] == len(want), (s, pts.shape[0], int(cnt[s]), len(want))
        assert np.array_equal(idx[off[s]: off[s] + cnt[s]], want), s
    return off, idx, cnt


def _shuffled(pts, seed):
    a = np.asarray(pts, np.int64)
    return to_xy(a[np.random.default_rng(seed).permutation(len(a))])


def _parabola(n):
    """n points (48 i, floor(i^2 / 512)): a long convex curve whose hull keeps
    thousands of vertices (the floor makes some of them collinear)."""
    i = np.arange(n, dtype=np.int64)
    return np.stack([48 * i, (i * i) >> 9], 1)


def test_convex_position_sets(ctx):
    _say("batch large: lattice polygon, parabola, lattice circle")
    poly = convex_lattice_polygon(100)          # about 24,000 strict vertices
    assert len(poly) > 20000
    sets = [
        _shuffled(poly, 1),
        _shuffled(_parabola(20000), 2),
        _shuffled(lattice_circle(5 * 13 * 17 * 29), 3),
        workloads.uniform(5000, 4),              # a small set between the large ones
        _shuffled(np.concatenate([np.asarray(poly) + 7, np.asarray(poly) + 7]), 5),  # duplicates
    ]
    _check(ctx, sets)


def test_thin_rings(ctx):
    """Points near a circle (the paper's worst case) in sets of 3*10^5 and
    10^6 points: random tiles of them are nearly all in convex position."""
    _say("batch large: thin rings")
    sets = [workloads.annulus(300_000, 71), workloads.normal(40_000, 72),
            workloads.annulus(1_000_000, 73), workloads.annulus(200_000, 74, 0.2, 0.2001)]
    _check(ctx, sets)


def test_large_sets_with_interior(ctx):
    """A convex polygon with many interior points, and a mix of large and
    small sets, so large sets sit between sets finished in earlier stages."""
    _say("batch large: polygon with interior points, mixed batch")
    rng = np.random.default_rng(9)
    poly = np.asarray(convex_lattice_polygon(70), np.int64) + 1000
    c = (poly.min(0) + poly.max(0)) // 2
    inner = rng.integers(-20000, 20000, (200_000, 2)) + c
    big = _shuffled(np.concatenate([poly, inner]), 10)
    sets = []
    for k in range(12):
        sets.append(workloads.by_kind(workloads.KINDS[k % 3], int(rng.integers(0, 50000)), 300 + k))
        if k % 4 == 1:
            sets.append(big if k != 5 else _shuffled(_parabola(15000), 11))
    _check(ctx, sets)


@pytest.mark.parametrize("n", [262143, 262144, 393215, 393216, 524287, 524288])
def test_sampler_chunk_boundaries(ctx, n):
    """Sets at the sizes where the sampler changes its chunk count (1/2, 2/3,
    3/4 chunks), in each kind, in one batch."""
    _say(f"batch sampler chunks n={n}")
    sets = [workloads.by_kind(k, n, 500 + i) for i, k in enumerate(("uniform", "normal", "annulus_wide"))]
    sets.append(workloads.annulus(n, 504))
    _check(ctx, sets)


def test_large_sets_in_graph_replays(ctx):
    """Batch mode with sets that take the per-set column path, captured in a
    HIP graph; every replay equals the eager result."""
    _say("batch large: graph replays")
    import torch
    sets = [_shuffled(convex_lattice_polygon(80), 20), workloads.annulus(250_000, 21),
            workloads.normal(30_000, 22), _shuffled(_parabola(12000), 23)]
    off = np.zeros(len(sets) + 1, np.int64)
    off[1:] = np.cumsum([s.shape[0] for s in sets])
    xy = _dev(np.concatenate(sets))
    o = _dev(off)
    n, nsets = xy.shape[0], len(sets)
    idx = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    cnt = torch.zeros(nsets, dtype=torch.int32, device="cuda:0")
    ws = ctx.workspace(ctx._lib.ch_hull_batch_workspace_bytes(nsets, n))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ctx.hull_batch_async(xy, o, idx, cnt, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    want_cnt = cnt.cpu().numpy().view(np.uint32).copy()
    want_idx = idx.cpu().numpy().view(np.uint32).copy()
    for s, pts in enumerate(sets):
        assert np.array_equal(want_idx[off[s]: off[s] + want_cnt[s]], oracle.hull(pts)), s
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.hull_batch_async(xy, o, idx, cnt, ws)
    for rep in range(3):
        idx.fill_(-1)
        cnt.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cnt.cpu().numpy().view(np.uint32), want_cnt), rep
        got = idx.cpu().numpy().view(np.uint32)
        for s in range(nsets):
            a = int(off[s])
            assert np.array_equal(got[a: a + want_cnt[s]], want_idx[a: a + want_cnt[s]]), (rep, s)
    del g
    torch.cuda.synchronize()

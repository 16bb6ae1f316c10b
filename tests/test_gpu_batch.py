"""GPU parity of the batched mode: every set's hull from ch_hull_batch equals
the oracle's hull of that set alone (and ch_hull's), bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2209_12310_amd import workloads
from tests._shapes import lattice_circle, to_xy

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

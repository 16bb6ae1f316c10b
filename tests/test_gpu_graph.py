"""ch_hull_batch is a fixed sequence of kernels with no host synchronisation,
so it can be captured in a HIP graph. The captured call is replayed several
times, with eager work and synchronisations in between, and every replay is
checked against the eager result (and the oracle)."""
import numpy as np
import pytest

import oracle
from paper_2209_12310_amd import workloads

pytestmark = pytest.mark.gpu


def test_batch_in_graph_replays():
    print("batch graph capture", flush=True)
    import torch
    import paper_2209_12310_amd as ch
    ctx = ch.Context(0)
    try:
        rng = np.random.default_rng(91)
        sets = [workloads.by_kind(("uniform", "normal", "annulus_wide")[i % 3], int(n), 200 + i)
                for i, n in enumerate(rng.integers(0, 60000, 40))]
        off = np.zeros(len(sets) + 1, np.int64)
        off[1:] = np.cumsum([s.shape[0] for s in sets])
        dev = "cuda:0"
        xy = torch.from_numpy(np.concatenate(sets)).to(dev)
        o = torch.from_numpy(off).to(dev)
        n, nsets = xy.shape[0], len(sets)
        idx = torch.zeros(n, dtype=torch.int32, device=dev)
        cnt = torch.zeros(nsets, dtype=torch.int32, device=dev)
        ws = ctx.workspace(ctx._lib.ch_hull_batch_workspace_bytes(nsets, n))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.hull_batch_async(xy, o, idx, cnt, ws)  # eager, on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        want_cnt = cnt.cpu().numpy().view(np.uint32).copy()
        want_idx = idx.cpu().numpy().view(np.uint32).copy()
        for s, pts in enumerate(sets):
            assert np.array_equal(want_idx[off[s]: off[s] + want_cnt[s]], oracle.hull(pts)), s
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.hull_batch_async(xy, o, idx, cnt, ws)
        for rep in range(4):
            idx.fill_(-1)
            cnt.fill_(-1)
            torch.cuda.synchronize()
            _ = (xy * 2).sum()  # unrelated eager work between replays
            g.replay()
            torch.cuda.synchronize()
            got_cnt = cnt.cpu().numpy().view(np.uint32)
            got_idx = idx.cpu().numpy().view(np.uint32)
            assert np.array_equal(got_cnt, want_cnt), rep
            for s in range(nsets):
                a = int(off[s])
                assert np.array_equal(got_idx[a: a + want_cnt[s]], want_idx[a: a + want_cnt[s]]), (rep, s)
        del g
        torch.cuda.synchronize()
    finally:
        ctx.close()

"""ch_filter_noalloc (the filter for callers that cannot allocate: its scratch
is the library's fixed device array) against ch_filter with a caller
workspace: survivors, count, labels and octagon must be identical, on calls
in a row whose inputs shrink (the scratch keeps the previous call's
contents), at the maximum size, and a size above it is refused."""
import numpy as np
import pytest

from paper_2209_12310_amd import _capi, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _run(ctx, t, noalloc):
    import torch
    n = t.shape[0]
    surv = torch.full((max(n, 1),), -1, dtype=torch.int32, device=t.device)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=t.device)
    lab = torch.full((max(n, 1),), 255, dtype=torch.uint8, device=t.device)
    octd = torch.full((24,), -1, dtype=torch.int32, device=t.device)
    if noalloc:
        ctx.filter_noalloc_async(t, surv, cnt, lab, octd)
    else:
        ctx.filter_async(t, surv, cnt, lab, octd)
    torch.cuda.synchronize()
    c = int(cnt.cpu().numpy().view(np.uint32)[0])
    return (c, surv[:c].cpu().numpy().view(np.uint32).copy(), lab[:n].cpu().numpy().copy(),
            octd.cpu().numpy().copy())


def _same(a, b):
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3], b[3])


def test_noalloc_filter_equals_filter():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2209_12310_amd as ch
    ctx = ch.Context(0)
    try:
        assert ctx._lib.ch_filter_noalloc_scratch_bytes() == \
            ctx._lib.ch_filter_workspace_bytes(_capi.CH_FILTER_NOALLOC_MAX_POINTS)
        cases = [("annulus", 3_000_000, 41), ("normal", 200_003, 42), ("uniform", 4097, 43),
                 ("annulus", 1, 44), ("normal", _capi.CH_FILTER_NOALLOC_MAX_POINTS, 45),
                 ("uniform", 130_001, 46)]
        for kind, n, seed in cases:
            _say(f"noalloc filter: {kind} n={n}")
            xy = workloads.by_kind(kind, n, seed)
            t = torch.from_numpy(xy).to("cuda:0")
            got = _run(ctx, t, True)
            want = _run(ctx, t, False)
            _same(got, want)
            again = _run(ctx, t, True)  # the scratch now holds this call's own leftovers
            _same(again, want)
        _say("noalloc filter: n = 0 and the size limit")
        empty = torch.empty((0, 2), dtype=torch.float32, device="cuda:0")
        assert _run(ctx, empty, True)[0] == 0
        big = torch.zeros((_capi.CH_FILTER_NOALLOC_MAX_POINTS + 1, 2), dtype=torch.float32, device="cuda:0")
        s = torch.empty(1, dtype=torch.int32, device="cuda:0")
        with pytest.raises(ch.ConvexHullError) as ei:
            ctx.filter_noalloc_async(big, s, s)
        assert ei.value.status == _capi.CH_E_INVALID_ARG
        assert "at most" in str(ei.value)
        del big
        torch.cuda.synchronize()
    finally:
        ctx.close()


def test_noalloc_filter_domain_error():
    import torch
    import paper_2209_12310_amd as ch
    ctx = ch.Context(0)
    try:
        xy = workloads.by_kind("normal", 50_000, 47)
        xy[1234, 0] = np.float32(0.3)  # off the 2^-20 grid
        t = torch.from_numpy(xy).to("cuda:0")
        _say("noalloc filter: domain error")
        assert _run(ctx, t, True)[0] == _capi.CH_COUNT_DOMAIN_ERROR
        assert _run(ctx, t, False)[0] == _capi.CH_COUNT_DOMAIN_ERROR
        ok = torch.from_numpy(workloads.by_kind("normal", 50_000, 48)).to("cuda:0")
        _same(_run(ctx, ok, True), _run(ctx, ok, False))
    finally:
        ctx.close()

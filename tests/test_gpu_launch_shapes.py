"""Launch shapes do not change results. The persistent grids of the extreme
reduction (CH_REDUCE_BLOCKS), the ordered filter with its look-back over the
earlier workgroups' counts (CH_FILTER_BLOCKS), the fused single read
(CH_FUSED_BLOCKS) and its narrow grid (CH_NARROW_BLOCKS) are read from the
environment when a context is created. For grid sizes from one workgroup to
the largest allowed, survivors, labels, octagon and hull must equal the
oracle's exactly."""
import os

import numpy as np
import pytest

import oracle
from paper_2209_12310_amd import workloads

pytestmark = pytest.mark.gpu

VARS = {"CH_REDUCE_BLOCKS": 4096, "CH_FILTER_BLOCKS": 1024, "CH_FUSED_BLOCKS": 4096,
        "CH_NARROW_BLOCKS": 4096}


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def inputs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    out = {}
    for kind in workloads.KINDS:
        xy = workloads.by_kind(kind, 1_000_000, 300 + len(out))
        kx, ky = oracle.to_grid(xy)
        surv, lab = oracle.filter(kx, ky)
        out[kind] = (xy, torch.from_numpy(xy).to("cuda:0"), surv, lab, oracle.octagon(xy),
                     oracle.heaphull(kx, ky))
    return out


def _context_with(var, value):
    import paper_2209_12310_amd as ch
    old = os.environ.get(var)
    os.environ[var] = str(value)
    try:
        return ch.Context(0)
    finally:
        if old is None:
            del os.environ[var]
        else:
            os.environ[var] = old


def _check(ctx, item):
    xy, t, surv, lab, octo, hull = item
    fr = ctx.filter(t, labels=True, octagon=True)
    assert np.array_equal(fr.survivors.cpu().numpy().view(np.uint32), surv)
    assert np.array_equal(fr.labels.cpu().numpy(), lab)
    for key in ("kx", "ky", "idx"):
        assert fr.octagon[key].tolist() == octo[key].tolist(), key
    assert np.array_equal(ctx.hull(t), hull)


@pytest.mark.parametrize("value", ["1", "7", "64", "max"])
@pytest.mark.parametrize("var", list(VARS))
def test_grid_size_does_not_change_results(inputs, var, value):
    v = VARS[var] if value == "max" else int(value)
    ctx = _context_with(var, v)
    try:
        for kind, item in inputs.items():
            _say(f"{var}={v} {kind}")
            _check(ctx, item)
    finally:
        ctx.close()


@pytest.mark.parametrize("var,value", [("CH_FUSED_BLOCKS", 7), ("CH_FILTER_BLOCKS", 7),
                                       ("CH_REDUCE_BLOCKS", 4096)])
def test_grid_size_full_size(var, value):
    """One 10^8-point configuration (the ring: most points take the exact
    test and survive) on an unusual grid."""
    import torch
    _say(f"{var}={value} annulus_1e8: generating")
    xy = workloads.single("annulus_1e8")
    kx, ky = oracle.to_grid(xy)
    oct_idx, want_s = oracle.filter_parallel(kx, ky, 0)
    want_h = oracle.chain(kx, ky, want_s)
    t = torch.from_numpy(xy).to("cuda:0")
    ctx = _context_with(var, value)
    try:
        _say(f"{var}={value} annulus_1e8: gpu")
        assert np.array_equal(ctx.hull(t), want_h)
        fr = ctx.filter(t)
        assert np.array_equal(fr.survivors.cpu().numpy().view(np.uint32), want_s)
    finally:
        ctx.close()
    del t
    torch.cuda.synchronize()

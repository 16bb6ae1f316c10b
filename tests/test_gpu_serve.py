"""GPU tests of the request server (ch_serve_*): every request's hull equals
the oracle's hull of that set alone, bit for bit, whatever it was batched
with; admission, back-pressure, time-outs and shutdown behave as declared."""
import threading
import time

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


@pytest.fixture(scope="module")
def arena():
    import torch
    return torch.empty(2 << 30, dtype=torch.uint8, device="cuda:0")


def _say(msg):
    print(msg, flush=True)


def _mixed_sets(seed, count):
    rng = np.random.default_rng(seed)
    sets = []
    for i in range(count):
        n = int(rng.choice([0, 1, 2, 5, 300, 4096, 8193, 20000, 150000, 400000]))
        sets.append(workloads.by_kind(("uniform", "normal", "annulus_wide")[i % 3], n, 1000 + i))
    return sets


def test_requests_match_oracle_in_a_mix(ctx, arena):
    _say("serve mixed requests")
    sets = _mixed_sets(70, 60)
    srv = ctx.serve(arena, n_streams=3)
    try:
        tickets = [srv.submit(s) for s in sets]
        for s, t in zip(sets, tickets):
            got, tns = srv.wait(t)
            assert np.array_equal(got, oracle.hull(s)), s.shape
            assert tns[0] <= tns[1] <= tns[2]
        st = srv.stats()
        assert st["completed"] == len(sets)
        assert 1 <= st["batches"] <= len(sets)
        assert 0 < st["p50_us"] <= st["p99_us"]
        assert st["hulls_per_s"] > 0
    finally:
        srv.stop()


def test_request_alone_equals_in_batch(ctx, arena):
    _say("serve alone vs batched")
    sets = _mixed_sets(71, 12)
    srv = ctx.serve(arena, n_streams=1)
    try:
        alone = []
        for s in sets:
            alone.append(srv.wait(srv.submit(s))[0])
        tickets = [srv.submit(s) for s in sets]
        for a, t in zip(alone, tickets):
            assert np.array_equal(srv.wait(t)[0], a)
        assert srv.stats()["batches"] < 2 * len(sets)
    finally:
        srv.stop()


def test_degenerate_and_convex_position_requests(ctx, arena):
    """A set with ~24K points in convex position overflows the batch's tile
    rounds and is finished by the general path inside the server."""
    _say("serve degenerate and convex-position requests")
    poly = convex_lattice_polygon(100)
    rng = np.random.default_rng(72)
    sets = [
        to_xy([poly[i] for i in rng.permutation(len(poly))]),
        to_xy([(7, 9)] * 33),
        to_xy(lattice_circle(5 * 13 * 17 * 29)),
        np.zeros((0, 2), np.float32),
        workloads.normal(5000, 9),
    ]
    srv = ctx.serve(arena, n_streams=2)
    try:
        tickets = [srv.submit(s) for s in sets]
        for s, t in zip(sets, tickets):
            assert np.array_equal(srv.wait(t)[0], oracle.hull(s))
    finally:
        srv.stop()


def test_domain_error_is_per_request(ctx, arena):
    _say("serve domain error")
    import paper_2209_12310_amd as ch
    good = [workloads.uniform(3000, s) for s in range(3)]
    bad = workloads.uniform(3000, 9)
    bad[17, 0] = np.float32(np.nan)
    srv = ctx.serve(arena, n_streams=1)
    try:
        tg = [srv.submit(g) for g in good[:2]]
        tb = srv.submit(bad)
        tg.append(srv.submit(good[2]))
        with pytest.raises(ch.DomainError):
            srv.wait(tb)
        for g, t in zip(good, tg):
            assert np.array_equal(srv.wait(t)[0], oracle.hull(g))
    finally:
        srv.stop()


def test_pinned_tensor_request(ctx, arena):
    _say("serve pinned request")
    import torch
    xy = workloads.normal(250000, 11)
    pinned = torch.from_numpy(xy).pin_memory()
    srv = ctx.serve(arena)
    try:
        assert np.array_equal(srv.wait(srv.submit(pinned))[0], oracle.hull(xy))
    finally:
        srv.stop()


def test_backpressure_and_timeouts(ctx, arena):
    _say("serve back-pressure")
    import paper_2209_12310_amd as ch
    sets = [workloads.uniform(1000, s) for s in range(5)]
    srv = ctx.serve(arena, n_streams=2, max_inflight=4)
    try:
        tickets = [srv.submit(s) for s in sets[:4]]
        with pytest.raises(ch.BusyError):
            srv.submit(sets[4])
        try:
            got = srv.wait(tickets[0], timeout_us=0)[0]
        except ch.WaitTimeout:
            got = srv.wait(tickets[0])[0]
        assert np.array_equal(got, oracle.hull(sets[0]))
        tickets = tickets[1:] + [srv.submit(sets[4])]
        for s, t in zip(sets[1:], tickets):
            assert np.array_equal(srv.wait(t, timeout_us=30_000_000)[0], oracle.hull(s))
        with pytest.raises(ch.ConvexHullError) as ei:
            srv.wait(tickets[0])
        assert ei.value.status == ch._capi.CH_E_NOT_FOUND
    finally:
        srv.stop()


def test_request_too_large_for_slot_is_rejected(ctx):
    _say("serve request above the slot size")
    import torch
    import paper_2209_12310_amd as ch
    small = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    srv = ctx.serve(small, n_streams=2)
    try:
        m = srv.max_request_points
        assert 0 < m < 10**6
        xy = workloads.uniform(m + 1, 5)
        with pytest.raises(ch.ConvexHullError) as ei:
            srv.submit(xy)
        assert ei.value.status == ch._capi.CH_E_INVALID_ARG
        ok = workloads.uniform(m, 6)
        assert np.array_equal(srv.wait(srv.submit(ok))[0], oracle.hull(ok))
    finally:
        srv.stop()
        torch.cuda.synchronize()


def test_stop_wakes_waiters(ctx, arena):
    """Stop finishes admitted batches and resolves the queued requests with
    CH_E_SHUTDOWN; a waiter blocked inside wait returns its ticket's final
    status."""
    _say("serve stop with a blocked waiter")
    import paper_2209_12310_amd as ch
    xy = workloads.uniform(2_000_000, 41)
    srv = ctx.serve(arena, n_streams=1, max_batch_points=2_000_000)
    tickets = [srv.submit(xy) for _ in range(128)]
    results = {}
    entering = threading.Event()

    def waiter():
        entering.set()
        try:
            results["last"] = ("ok", srv.wait(tickets[-1])[0])
        except ch.ConvexHullError as e:
            results["last"] = ("err", e.status)

    th = threading.Thread(target=waiter)
    th.start()
    first, _ = srv.wait(tickets[0])
    assert entering.wait(10)
    time.sleep(0.05)
    srv.stop()
    th.join(30)
    assert not th.is_alive()
    want = oracle.hull(xy)
    assert np.array_equal(first, want)
    kind, val = results["last"]
    if kind == "ok":
        assert np.array_equal(val, want)
    else:
        assert val == ch._capi.CH_E_SHUTDOWN


def test_request_at_the_top_of_the_size_range(ctx):
    """One request of 10^7 points (the largest request size of the serving
    workload), next to small ones, in an arena sized for it."""
    import torch
    _say("serve 1e7-point request")
    big = workloads.by_kind("annulus_wide", 10_000_000, 77)
    small = [workloads.by_kind("normal", 5000, 78 + i) for i in range(3)]
    arena = torch.empty(6 << 30, dtype=torch.uint8, device="cuda:0")
    srv = ctx.serve(arena, n_streams=2)
    try:
        assert srv.max_request_points >= big.shape[0]
        tickets = [srv.submit(s) for s in [small[0], big] + small[1:]]
        for s, tk in zip([small[0], big] + small[1:], tickets):
            got, _ = srv.wait(tk)
            assert np.array_equal(got, oracle.hull(s)), s.shape
    finally:
        srv.stop()
    del arena
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

"""Benchmark: end-to-end convex hull of 10^8 points on one MI355X.

Workload (the configuration the headline metric is quoted on): 10^8 float32
points, bivariate normal (mean 0.5, sigma 0.1) quantized to the 2^-20 grid in
[0,1), seed 1, resident in HBM before timing starts. One step = one ch_hull
call: domain check, extreme reduction, octagon filter with compaction, device
hull, hull indices back in host memory.

Prints one JSON line (see the design notes for every field). Roofline: the
dominant kernel's algorithmic bytes per launch divided by its mean duration,
timed with HIP events recorded by the library on the launch stream in a
second region of the same steps (the end-to-end figure is taken without
them).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpts/s end-to-end hull at 1e8 pts (% HBM peak); batched hulls/s + p50/p99"
WORKLOAD = "normal_1e8"
# Streaming kernels of the filtering stage and the point bytes each reads.
# From 131072 points ch_hull reads the points once (pass_fused: the extreme
# reduction and the sample-polygon test together) and writes 16 B candidate
# records; below that, or without a usable sample polygon, pass 1 (reduce8)
# and pass 2 (filter_compact) each read 8 B per point.
BYTES_PER_POINT = {"reduce8": 8, "filter_compact": 8, "pass_fused": 8}
STAGE_KERNELS = ("sample_poly", "pass_fused", "reduce8", "oct_build", "cand_filter", "filter_compact")


def stage_bytes(n: int, info: dict) -> dict:
    """Algorithmic HBM bytes of one ch_hull filtering stage, from the call's
    counts: point reads, the sample gather (8 B per sample point), candidate
    records written and read back, survivor records written."""
    cand, surv = info["candidates"], info["survivors"]
    if cand:
        b = {"points": 8 * n, "sample": 8 * 65536, "candidates": 32 * cand, "survivors": 16 * surv}
    else:
        b = {"points": 16 * n, "sample": 0, "candidates": 0, "survivors": 16 * surv}
    b["total"] = sum(b.values())
    b["per_point"] = round(b["total"] / n, 3)
    return b


def kernel_alg_bytes(name: str, n: int, info: dict):
    """Algorithmic HBM bytes of one launch of a ch_hull kernel (None where no
    byte model applies: one-workgroup stages bound by latency)."""
    cand, surv = info.get("candidates", 0), info.get("survivors", 0)
    model = {
        "pass_fused": 8 * n + 16 * cand,          # every point once + candidate records
        "reduce8": 8 * n,                         # pass 1
        "filter_compact": 8 * n + 16 * surv,      # pass 2 + survivor records
        "cand_filter": 16 * cand + 16 * surv,     # candidate records in, survivors out
        # large-hull path (input: the survivor records when no tile round ran)
        "lg_count": 16 * surv,                    # records read, chunk counts in LDS
        "lg_scatter": 32 * surv,                  # records read and written to their chunk
        "lg_chunk": 16 * surv,                    # records read, column table and chains in LDS
    }
    return model.get(name)


def kernel_roofline(stats: dict, n: int, info: dict, read_gbs=None, workload=None) -> dict:
    """Roofline of the dominant kernel among those with a byte model, from
    the library's per-kernel HIP events; also names the kernel that takes the
    most time overall."""
    means = {k: v[1] / v[0] for k, v in stats.items() if v[0]}
    if not means:
        return {}
    overall = max(means, key=lambda k: means[k] * stats[k][0])
    modelled = [k for k in means if kernel_alg_bytes(k, n, info) is not None]
    if not modelled:
        return {"dominant_overall": overall}
    dom = max(modelled, key=lambda k: means[k])
    alg = kernel_alg_bytes(dom, n, info)
    achieved = alg / (means[dom] * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": alg,
         "mean_us": round(means[dom] * 1e3, 2), "dominant_overall": overall,
        "traffic": load_traffic(workload, n, dom) if workload else None}
    if read_gbs:
        r["frac_of_read_stream"] = round(achieved / read_gbs, 4)
    return r


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


KERNEL_SOURCES = ["paper_2209_12310_amd/csrc/ch_filter.hip", "paper_2209_12310_amd/csrc/ch_internal.hpp",
                  "paper_2209_12310_amd/csrc/ch_device.hpp", "paper_2209_12310_amd/csrc/ch_refine.hpp",
                  "paper_2209_12310_amd/csrc/ch_refine.hip", "paper_2209_12310_amd/csrc/ch_hull.hip"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, n: int, kernel: str):
    """HBM bytes per launch of one kernel from the committed rocprofv3 counter
    summary of this workload, or None when it is absent or the kernel source
    changed since."""
    try:
        with open(traffic_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash() or t.get("n") != n:
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(xy, t, ctx, budget_s: float = 6.0):
    """The CPU oracle as it stands, built on this host with -O3 -march=native
    (the planted-mistake switch compiled out), timed on the full headline
    input within a time budget per variant:
      value            the multi-core heaphull of Sec. III taken to the end:
                       grid conversion, then extremes and filter by divide and
                       conquer, labels, the four queues, each hulled with a
                       parallel sort, on every host thread;
      single_thread    the sequential heaphull (extremes, filter, chain);
      paper_architecture  the paper's own split (Sec. III): the label array
                       of Alg. 2 on this GPU (ch_gpufilter with the two-kernel
                       extreme search), copied to pinned host memory, then the
                       four queues and their hulls on the host cores.
    Each variant's hull is checked against ch_hull's."""
    import numpy as np
    import torch

    import oracle
    nat = oracle.native()
    n = xy.shape[0]
    want = ctx.hull(t)

    def timed(fn):
        reps, total, out = 0, 0.0, None
        while reps < 5 and (reps == 0 or total < budget_s):
            t0 = time.perf_counter()
            out = fn()
            total += time.perf_counter() - t0
            reps += 1
        return reps, total, out

    cores = nat.max_threads()
    t0 = time.perf_counter()
    kx, ky = oracle.to_grid(xy)
    grid_s = time.perf_counter() - t0
    reps, total, h = timed(lambda: nat.heaphull_parallel(kx, ky, 0))
    assert np.array_equal(h, want), "multi-core heaphull differs from ch_hull"
    multi_s = grid_s + total / reps
    reps1, total1, h1 = timed(lambda: nat.heaphull(kx, ky))
    assert np.array_equal(h1, want), "sequential heaphull differs from ch_hull"
    single_s = grid_s + total1 / reps1

    # The paper's architecture: GPU labels -> host -> CPU queues and hulls.
    lab_dev = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    oct_dev = torch.empty(24, dtype=torch.int32, device="cuda:0")
    lab_host = torch.empty(n, dtype=torch.uint8).pin_memory()
    oct_host = torch.empty(24, dtype=torch.int32).pin_memory()

    def paper():
        a = time.perf_counter()
        ctx.gpufilter_async(t, lab_dev, oct_dev, None, "two_kernels")
        torch.cuda.synchronize()
        b = time.perf_counter()
        lab_host.copy_(lab_dev, non_blocking=True)
        oct_host.copy_(oct_dev, non_blocking=True)
        torch.cuda.synchronize()
        c = time.perf_counter()
        labels = lab_host.numpy()
        oct_idx = oct_host.numpy()[16:24].view(np.uint32).astype(np.int64)
        hull, _ = nat.heaphull_queues(kx, ky, labels, oct_idx, cores)
        d = time.perf_counter()
        return hull, (b - a, c - b, d - c)

    paper()  # warm the GPU path
    times = []
    for _ in range(3):
        hp, parts = paper()
        times.append(parts)
    assert np.array_equal(hp, want), "paper architecture differs from ch_hull"
    gpu_s, d2h_s, cpu_s = (float(np.median([p[i] for p in times])) for i in range(3))
    return {"value": round(n / multi_s / 1e6, 3), "unit": "Mpts/s", "cores": cores, "kind": "oracle",
            "sample": f"full {WORKLOAD} input ({n} points): grid conversion ({grid_s:.2f} s, one "
                      f"thread), then the four-queue heaphull on {cores} threads, {reps} run(s) in "
                      f"{total:.1f} s; oracle built -O3 -march=native",
            "ms": round(multi_s * 1e3, 1),
            "single_thread_value": round(n / single_s / 1e6, 3),
            "single_thread_sample": f"grid conversion, then {reps1} run(s) in {total1:.1f} s of the "
                                    f"sequential heaphull",
            "paper_architecture": {
                "value": round(n / (gpu_s + d2h_s + cpu_s) / 1e6, 3), "unit": "Mpts/s",
                "ms": round((gpu_s + d2h_s + cpu_s) * 1e3, 2),
                "gpu_labels_ms": round(gpu_s * 1e3, 3), "d2h_labels_ms": round(d2h_s * 1e3, 3),
                "cpu_queues_hull_ms": round(cpu_s * 1e3, 2), "cores": cores,
                "what": "ch_gpufilter (two-kernel extremes, Alg. 2 labels) on the GPU, labels and "
                        "octagon copied to pinned host memory, four queues + hulls on the host "
                        "(kx, ky already on the host); median of 3"}}


def bench_paper_pipeline(ctx, t, steps: int) -> dict:
    """Alg. 1 stage by stage on the device (ch_hull_queues) with each extreme
    search, and the A/B of the extreme searches alone: Sec. III's two
    reductions (axis extremes, then Manhattan corners) against the one-read
    search, from the library's kernel events."""
    import torch
    n = t.shape[0]
    out = {}
    ref = ctx.hull(t)
    for mode in ("two_kernels", "fused"):
        for _ in range(2):
            got, qc = ctx.hull_queues(t, extremes=mode)
        assert (got == ref).all(), f"ch_hull_queues ({mode}) differs from ch_hull"
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.hull_queues(t, extremes=mode)
        ms = (time.perf_counter() - t0) / steps * 1e3
        ctx.profile_reset()
        ctx.profile_enable(True)
        for _ in range(steps):
            ctx.hull_queues(t, extremes=mode)
        ctx.profile_enable(False)
        st = ctx.profile_read()
        out[f"hull_queues_{mode}"] = {
            "ms_per_step": round(ms, 4), "mpts_per_s": round(n / (ms * 1e-3) / 1e6, 1),
            "queue_sizes": [int(v) for v in qc],
            "kernels_us": {k: round(v[1] / v[0] * 1e3, 2) for k, v in st.items() if v[0]}}
    lab = torch.empty(n, dtype=torch.uint8, device=t.device)
    ab = {}
    for mode in ("two_kernels", "fused"):
        ctx.gpufilter_async(t, lab, None, None, mode)
        ctx.profile_reset()
        ctx.profile_enable(True)
        for _ in range(steps):
            ctx.gpufilter_async(t, lab, None, None, mode)
        ctx.profile_enable(False)
        st = ctx.profile_read()
        k = {name: round(v[1] / v[0] * 1e3, 2) for name, v in st.items() if v[0]}
        ext = ("axis_extremes", "corner_extremes") if mode == "two_kernels" else ("reduce8",)
        ab[mode] = {"extremes_us": round(sum(k.get(e, 0.0) for e in ext), 2),
                    "gpufilter_us": round(sum(k.values()), 2), "kernels_us": k,
                    "extremes_read_bytes": (16 if mode == "two_kernels" else 8) * n}
    ab["speedup_extremes"] = round(ab["two_kernels"]["extremes_us"] / ab["fused"]["extremes_us"], 3)
    out["extremes_ab"] = ab
    return out


def measure_read_stream(ctx, buf, reps: int = 10) -> dict:
    """The read bandwidth this device reaches on a plain non-temporal stream
    over the same buffer (ch_diag_read_stream), best over a few grid sizes:
    the reference for the roofline fraction beside the vendor peak."""
    import torch
    by = {}
    nbytes = 0
    for blocks in (256, 512, 1024):
        for _ in range(2):
            nbytes = ctx.read_stream_async(buf, blocks)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            ctx.read_stream_async(buf, blocks)
        b.record()
        torch.cuda.synchronize()
        by[blocks] = round(nbytes / (a.elapsed_time(b) / reps * 1e-3) / 1e9, 1)
    best = max(by, key=by.get)
    return {"gbs": by[best], "blocks": best, "bytes": nbytes, "by_blocks": by,
            "kernel": "ch_diag_read_stream: 16-byte non-temporal loads, 4 per thread per step"}


def bench_single(ctx, name: str, steps: int, warmup: int, read_gbs=None) -> dict:
    """ch_hull end to end on one more single-set configuration."""
    import torch

    from paper_2209_12310_amd import workloads
    log(f"generating {name}")
    xy = workloads.single(name)
    n = xy.shape[0]
    t = torch.from_numpy(xy).to("cuda:0")
    fr = ctx.filter(t)  # octagon survivor count, before the warmup of the timed calls
    survivors = fr.count
    del fr
    for _ in range(warmup):
        hull = ctx.hull(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hull = ctx.hull(t)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    info = ctx.last_hull_info()
    moved = stage_bytes(n, info)["total"] + 16 * info["survivors"]
    # Kernel durations in a second region (library events on the launch stream).
    ctx.profile_reset()
    ctx.profile_enable(True)
    for _ in range(steps):
        ctx.hull(t)
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    stats = ctx.profile_read()
    del t
    return {"workload": name, "n": n, "ms_per_step": round(ms, 4), "mpts_per_s": round(n / (ms * 1e-3) / 1e6, 1),
            "bytes_per_point": round(moved / n, 3),
            "hbm_frac": round(moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "octagon_survivors": survivors, "hull_info": info, "h": int(hull.size),
            "kernels_us": {k: round(v[1] / v[0] * 1e3, 2) for k, v in stats.items() if v[0]},
            "kernel_launches_per_step": {k: round(v[0] / steps, 2) for k, v in stats.items() if v[0]},
            "roofline": kernel_roofline(stats, n, info, read_gbs, name)}


def pct(vals, q):
    import numpy as np
    return float(np.percentile(np.asarray(vals, dtype=np.float64), q))


def bench_batch(ctx, steps: int, warmup: int, params=None, plain_mode: bool = True) -> dict:
    """Batched mode on 4096 sets (log-uniform sizes in [1e3, 1e6], kinds
    uniform / normal / annulus 0.49-0.5, seed 3): parameters from the
    autotuner, then the ch_hull_batch call captured once in a HIP graph and
    the graph replayed once per step, timed with events on the replay
    stream (the headline batch figure); eager calls are timed beside it.
    Every set of a batch completes when the launch sequence does, so the
    per-set latency is the batch latency. Compared with one ch_hull call per
    set on the same device-resident points."""
    import numpy as np
    import torch

    from paper_2209_12310_amd import workloads
    log("generating batch_4096")
    xy, off, kinds = workloads.batch_sets(4096, 3)
    n = xy.shape[0]
    nsets = off.size - 1
    t = torch.from_numpy(xy).to("cuda:0")
    o = torch.from_numpy(off.astype(np.int64)).to("cuda:0")
    idx = torch.empty(n, dtype=torch.int32, device="cuda:0")
    cnt = torch.empty(nsets, dtype=torch.int32, device="cuda:0")
    ws = ctx.workspace(ctx._lib.ch_hull_batch_workspace_bytes(nsets, n))
    t0 = time.perf_counter()
    if params is None:
        log("tuning batch parameters")
        params = ctx.tune_batch(t, o, idx, cnt, ws)
    else:
        log(f"batch parameters fixed: {params}")
        ctx.set_batch_params(params)
    tune_s = time.perf_counter() - t0
    for _ in range(warmup):
        ctx.hull_batch_async(t, o, idx, cnt, ws)
    torch.cuda.synchronize()
    counts = cnt.cpu().numpy().view(np.uint32).copy()
    assert (counts < 0xFFFFFFF0).all(), "batch returned an error code"
    hull_idx_eager = idx.cpu().numpy().view(np.uint32).copy()

    def timed(launch):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for a, b in ev:
            a.record()
            launch()
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev], (time.perf_counter() - w0) / steps

    lat_eager, wall_eager = timed(lambda: ctx.hull_batch_async(t, o, idx, cnt, ws))
    # One capture, replayed per step (the launch sequence holds no host
    # synchronisation and no memset node).
    log("batch: graph capture and replays")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ctx.hull_batch_async(t, o, idx, cnt, ws)
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    lat, wall = timed(g.replay)
    same = (np.array_equal(cnt.cpu().numpy().view(np.uint32), counts) and
            np.array_equal(idx.cpu().numpy().view(np.uint32), hull_idx_eager))
    assert same, "graph replay differs from the eager call"
    del g
    # Per-kernel durations (library events around each launch, eager calls).
    ctx.profile_reset()
    ctx.profile_enable(True)
    for _ in range(steps):
        ctx.hull_batch_async(t, o, idx, cnt, ws)
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    stats = ctx.profile_read()
    kernels = {k: {"launches_per_batch": round(v[0] / steps, 2), "ms_per_batch": round(v[1] / steps, 4)}
               for k, v in stats.items() if v[0]}
    # Roofline of the single read over all sets (k_batch_pass): 8 B per point
    # (candidate records written are not counted: a lower bound).
    pass_ms = stats.get("batch_pass", (0, 0.0))[1] / max(stats.get("batch_pass", (1, 0))[0], 1)
    roof = None
    if pass_ms > 0:
        ach = 8 * n / (pass_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "batch_pass", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": 8 * n,
                "mean_us": round(pass_ms * 1e3, 2),
                "note": "8 B per point read; candidate records written are left out (lower bound)",
                "traffic": load_traffic("batch_4096", n, "batch_pass")}
    # Plain mode: one synchronous ch_hull per set.
    plain = float("nan")
    if plain_mode:
        log("plain mode: one ch_hull per set")
        for s in range(min(64, nsets)):
            ctx.hull(t[int(off[s]): int(off[s + 1])])
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for s in range(nsets):
            ctx.hull(t[int(off[s]): int(off[s + 1])])
        torch.cuda.synchronize()
        plain = time.perf_counter() - tp
    ms = float(np.mean(lat))
    return {"workload": "batch_4096", "sets": nsets, "points": n, "steps": steps,
            "timing": "one HIP graph replay of the captured ch_hull_batch call per step",
            "ms_per_batch": round(ms, 3), "wall_ms_per_batch": round(wall * 1e3, 3),
            "hulls_per_s": round(nsets / (ms * 1e-3), 1),
            "mpts_per_s": round(n / (ms * 1e-3) / 1e6, 1),
            "hbm_frac_8B_per_point": round(8 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "batch_latency_p50_ms": round(pct(lat, 50), 3), "batch_latency_p99_ms": round(pct(lat, 99), 3),
            "eager_ms_per_batch": round(float(np.mean(lat_eager)), 3),
            "eager_wall_ms_per_batch": round(wall_eager * 1e3, 3),
            "plain_ms": round(plain * 1e3, 1) if plain_mode else None,
            "plain_hulls_per_s": round(nsets / plain, 1) if plain_mode else None,
            "speedup_vs_plain": round(plain / (ms * 1e-3), 2) if plain_mode else None,
            "params": params, "tune_s": round(tune_s, 2), "kernels": kernels, "roofline": roof,
            "kinds": {k: kinds.count(k) for k in sorted(set(kinds))}}


def _serve_views(pools, sizes, kinds, seeds):
    """Request payloads: windows of the pinned per-kind pools (offset drawn
    from the request's seed), so no request data is generated while timing."""
    views = []
    for n, k, sd in zip(sizes, kinds, seeds):
        pool = pools[k]
        o = int(sd) % (pool.shape[0] - int(n) + 1)
        views.append(pool[o: o + int(n)])
    return views


def bench_serve(ctx, duration_s: float = 60.0, arena_gb: int = 64, streams: int = 4,
                plain_s: float = 15.0, max_batch_points: int = 0, rate=None) -> dict:
    """Serving: Poisson arrivals of host-resident requests (sizes log-uniform
    in [1e2, 1e7], kinds uniform / normal / wide annulus, seed 4) through the
    ch_serve server; latency = completion - scheduled arrival, including
    queueing and the host-to-device copy. The rate is 0.7 x the capacity
    measured on a saturated burst. Compared with plain mode: the first
    plain_s seconds of the same trace solved one request at a time (copy,
    then ch_hull) on one stream; plain mode's capacity is below the arrival
    rate, so its queue only grows after that."""
    import queue
    import threading

    import numpy as np
    import torch

    from paper_2209_12310_amd import workloads
    pool_n = 10_000_000
    log("serve: pinned request pools")
    pools = {k: torch.from_numpy(workloads.by_kind(k, pool_n, 90 + i)).pin_memory()
             for i, k in enumerate(("uniform", "normal", "annulus_wide"))}
    arena = torch.empty(arena_gb << 30, dtype=torch.uint8, device="cuda:0")
    srv = ctx.serve(arena, n_streams=streams, max_batch_points=max_batch_points)
    try:
        # Capacity on a saturated burst.
        _, bs, bk, bseed = workloads.serve_trace(1e9, 1e9, seed=5, max_requests=1500)
        burst = _serve_views(pools, bs, bk, bseed)
        log(f"serve: saturated burst of {len(burst)} requests")
        t0 = time.monotonic_ns()
        tick = [srv.submit(v) for v in burst]
        last = max(int(srv.wait(t)[1][2]) for t in tick)
        capacity = len(burst) / ((last - t0) * 1e-9)
        if rate is None:
            rate = 0.7 * capacity
        times, sizes, kinds, seeds = workloads.serve_trace(rate, duration_s, seed=4)
        views = _serve_views(pools, sizes, kinds, seeds)
        log(f"serve: {len(views)} requests at {rate:.0f}/s for {duration_s} s")
        q: "queue.Queue" = queue.Queue()
        start = time.monotonic_ns() + 50_000_000
        sched = start + (np.asarray(times) * 1e9).astype(np.int64)

        def submitter():
            for i, v in enumerate(views):
                d = (int(sched[i]) - time.monotonic_ns()) * 1e-9
                if d > 0:
                    time.sleep(d)
                q.put(srv.submit(v))

        th = threading.Thread(target=submitter)
        th.start()
        lat, done_max = [], 0
        parts = np.zeros((len(views), 3))  # submit lag, queueing, service (us)
        for i in range(len(views)):
            _, tns = srv.wait(q.get())
            a, m, d = (int(v) for v in tns)
            lat.append((d - int(sched[i])) * 1e-3)
            parts[i] = ((a - int(sched[i])) * 1e-3, (m - a) * 1e-3, (d - m) * 1e-3)
            done_max = max(done_max, d)
        th.join()
        st = srv.stats()
    finally:
        srv.stop()
    del arena
    # Where the latency goes: per component, and the tail by request size.
    lat_a = np.asarray(lat)
    sz = np.asarray(sizes, dtype=np.float64)
    tail = lat_a >= np.percentile(lat_a, 99)
    breakdown = {
        "submit_lag_us": {"p50": round(pct(parts[:, 0], 50), 1), "p99": round(pct(parts[:, 0], 99), 1)},
        "queue_us": {"p50": round(pct(parts[:, 1], 50), 1), "p99": round(pct(parts[:, 1], 99), 1)},
        "service_us": {"p50": round(pct(parts[:, 2], 50), 1), "p99": round(pct(parts[:, 2], 99), 1),
                       "what": "admission to completion: host-to-device copy, batch kernels, hull copy back"},
        "p99_tail": {"requests": int(tail.sum()),
                     "median_points": int(np.median(sz[tail])),
                     "mean_queue_us": round(float(parts[tail, 1].mean()), 1),
                     "mean_service_us": round(float(parts[tail, 2].mean()), 1)},
        "by_size_p99_us": {label: round(pct(lat_a[m], 99), 1) for label, m in
                           (("lt_1e5", sz < 1e5), ("1e5_1e6", (sz >= 1e5) & (sz < 1e6)),
                            ("ge_1e6", sz >= 1e6)) if m.any()},
    }
    # Plain mode on the same trace: one request at a time.
    log("serve: plain mode")
    dev = torch.empty((int(max(sizes)), 2), dtype=torch.float32, device="cuda:0")
    plat = []
    pstart = time.monotonic_ns() + 50_000_000
    psched = pstart + (np.asarray(times) * 1e9).astype(np.int64)
    for i, v in enumerate(views):
        if times[i] > plain_s:
            break
        d = (int(psched[i]) - time.monotonic_ns()) * 1e-9
        if d > 0:
            time.sleep(d)
        n = v.shape[0]
        dev[:n].copy_(v, non_blocking=True)
        ctx.hull(dev[:n])
        plat.append((time.monotonic_ns() - int(psched[i])) * 1e-3)
    pend = time.monotonic_ns()
    return {"workload": "serve_poisson", "requests": len(views), "rate_hz": round(rate, 1),
            "duration_s": duration_s, "streams": streams, "arena_gb": arena_gb,
            "max_batch_points": max_batch_points,
            "mean_points": round(float(np.mean(sizes)), 1),
            "capacity_hulls_per_s": round(capacity, 1),
            "hulls_per_s": round(len(views) / ((done_max - start) * 1e-9), 1),
            "p50_us": round(pct(lat, 50), 1), "p99_us": round(pct(lat, 99), 1),
            "batches": st["batches"],
            "latency_breakdown": breakdown,
            "h2d_gbs": round(len(views) / ((done_max - start) * 1e-9) * float(np.mean(sizes)) * 8 / 1e9, 2),
            "plain_requests": len(plat),
            "plain_hulls_per_s": round(len(plat) / ((pend - pstart) * 1e-9), 1),
            "plain_p50_us": round(pct(plat, 50), 1) if plat else None,
            "plain_p99_us": round(pct(plat, 99), 1) if plat else None,
            "plain_trace_s": plain_s,
            "input": "pinned host memory, copied to the device inside the measured latency"}


def copy_calibration(nbytes: int = 800_000_000, reps: int = 3) -> None:
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-mode measurement")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-extra", action="store_true", help="skip the other single-set configurations")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-pipeline measurements")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="single-set workload of the headline line (profiling runs of other configs)")
    ap.add_argument("--only-batch", action="store_true",
                    help="measure batch mode alone (profiling runs of batch_4096)")
    ap.add_argument("--batch-params", default=None,
                    help="JSON batch parameters to use instead of tuning (profiling runs)")
    ap.add_argument("--no-plain", action="store_true", help="skip batch plain mode (profiling runs)")
    ap.add_argument("--only-serve", action="store_true", help="measure serving alone")
    ap.add_argument("--serve-duration", type=float, default=60.0)
    ap.add_argument("--serve-plain-s", type=float, default=15.0)
    ap.add_argument("--serve-max-batch-points", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "design is described, not built.", file=sys.stderr)
        return 2
    if args.copy_calibration:
        copy_calibration()
        return 0
    if args.only_batch:
        import torch

        import paper_2209_12310_amd as ch
        ctx = ch.Context(0)
        bp = json.loads(args.batch_params) if args.batch_params else None
        print(json.dumps({"batch": bench_batch(ctx, max(5, min(args.steps, 20)), args.warmup, bp,
                                               not args.no_plain)}), flush=True)
        ctx.close()
        return 0
    if args.only_serve:
        import torch

        import paper_2209_12310_amd as ch
        torch.zeros(1, device="cuda:0")  # torch's device runtime first, then the library's context
        ctx = ch.Context(0)
        print(json.dumps({"serve": bench_serve(ctx, args.serve_duration, plain_s=args.serve_plain_s,
                                               max_batch_points=args.serve_max_batch_points)}), flush=True)
        ctx.close()
        return 0
    workload = args.workload

    import numpy as np
    import torch

    import paper_2209_12310_amd as ch
    from paper_2209_12310_amd import workloads

    log(f"generating {workload}")
    xy = workloads.single(workload)
    n = xy.shape[0]
    dev = torch.device("cuda:0")
    t = torch.from_numpy(xy).to(dev)
    torch.cuda.synchronize()
    ctx = ch.Context(0)
    log(f"warmup {args.warmup}")
    hull = None
    for _ in range(args.warmup):
        hull = ctx.hull(t)
    fr = ctx.filter(t)
    survivors = fr.count
    del fr
    torch.cuda.synchronize()

    log(f"timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    for _ in range(args.steps):
        hull = ctx.hull(t)  # synchronous: returns with the hull in host memory
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed / args.steps * 1e3
    value = n / (ms * 1e-3) / 1e6
    step_ms = np.diff(np.array([t0] + marks)) * 1e3
    step_stats = {"mean": round(float(step_ms.mean()), 4), "median": round(float(np.median(step_ms)), 4),
                  "p99": round(float(np.percentile(step_ms, 99)), 4), "min": round(float(step_ms.min()), 4)}

    # Kernel durations: a second region of the same steps with the library's
    # HIP events recorded on the launch stream around every kernel (they add
    # their own gaps, so the end-to-end figure above is taken without them).
    log(f"kernel timing {args.steps} steps")
    ctx.profile_reset()
    ctx.profile_enable(True)
    for _ in range(args.steps):
        ctx.hull(t)
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    stats = ctx.profile_read()

    info = ctx.last_hull_info()
    kernels = {k: {"launches": v[0], "mean_us": round(v[1] / max(v[0], 1) * 1e3, 2)}
               for k, v in stats.items() if v[0]}
    read_stream = measure_read_stream(ctx, t)
    dom = max((k for k in BYTES_PER_POINT if k in stats), key=lambda k: stats[k][1])
    launches, total_ms = stats[dom]
    mean_s = total_ms / launches * 1e-3
    if dom == "pass_fused":
        alg_bytes = 8 * n + 16 * info["candidates"]
    elif dom == "filter_compact":
        alg_bytes = 8 * n + 16 * info["survivors"]
    else:
        alg_bytes = 8 * n
    achieved = alg_bytes / mean_s / 1e9
    traffic = load_traffic(workload, n, dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": alg_bytes,
                "mean_us": round(mean_s * 1e6, 2),
                "frac_of_read_stream": round(achieved / read_stream["gbs"], 4)}
    sb = stage_bytes(n, info)
    filt_ms = sum(stats[k][1] / stats[k][0] for k in STAGE_KERNELS if k in stats and stats[k][0])
    filter_stage = {"bytes_per_point": sb["per_point"], "bytes": sb, "mean_us": round(filt_ms * 1e3, 2),
                    "gbs": round(sb["total"] / (filt_ms * 1e-3) / 1e9, 1),
                    "frac_of_peak": round(sb["total"] / (filt_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "kernels": [k for k in STAGE_KERNELS if k in stats]}
    moved = sb["total"] + 16 * info["survivors"]  # plus the hull pass reading the survivors

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "step_ms": step_stats,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "input_dtype": "f32",
        "arithmetic": "float32 (x, y) on the 2^-20 grid in; every predicate exact in fp64 / int64",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "distribution": workloads.describe(workload),
                   "seed": workloads.seed_of(workload), "survivors": survivors,
                   "h": int(hull.size)},
        "bytes_per_point_end_to_end": round(moved / n, 3),
        "hbm_frac_end_to_end": round(moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "hull_info": info,
        "filter_stage": filter_stage,
        "roofline": roofline,
        "read_stream": read_stream,
        "kernels": kernels,
    }
    if not args.no_paper:
        log("paper pipeline: ch_hull_queues and the extreme-search A/B")
        out["paper_pipeline"] = bench_paper_pipeline(ctx, t, max(3, min(args.steps, 10)))
    del t
    torch.cuda.synchronize()
    out["single_sets"] = {workload: {"workload": workload, "n": n, "ms_per_step": round(ms, 4),
                                     "mpts_per_s": round(value, 1),
                                     "bytes_per_point": out["bytes_per_point_end_to_end"],
                                     "hbm_frac": out["hbm_frac_end_to_end"],
                                     "octagon_survivors": survivors, "hull_info": info,
                                     "h": int(hull.size), "kernels_us": {k: v["mean_us"] for k, v in kernels.items()},
                                     "roofline": kernel_roofline(stats, n, info, read_stream["gbs"],
                                                                 workload)}}
    if not args.no_extra:
        for name in ("uniform_1e8", "annulus_1e8", "uniform_1e6"):
            if name == workload:
                continue
            out["single_sets"][name] = bench_single(ctx, name, max(3, min(args.steps, 20)), 5,
                                                    read_stream["gbs"])
            torch.cuda.synchronize()
    if not args.no_batch:
        out["batch"] = bench_batch(ctx, max(5, min(args.steps, 20)), 1)
        torch.cuda.synchronize()
    if not args.no_serve:
        out["serve"] = bench_serve(ctx, args.serve_duration, plain_s=args.serve_plain_s,
                                   max_batch_points=args.serve_max_batch_points)

    if not args.no_cpu:
        log("cpu baseline (oracle) and the paper's architecture")
        t = torch.from_numpy(xy).to(dev)
        out["cpu_baseline"] = cpu_baseline(xy, t, ctx)
        del t
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

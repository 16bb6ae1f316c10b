"""MI355X-native convex hull: the heaphull-style octagon filter and a device
hull pass (Keith, Ferrada, Navarro, arXiv 2209.12310), as HIP kernels for
gfx950 behind the C ABI in include/convhull.h.

This package is a thin binding: it checks tensor arguments, allocates device
buffers with torch, and passes pointers and the current HIP stream to the
library. It never computes any part of the hull itself.
"""
from __future__ import annotations

import ctypes
import threading
from dataclasses import dataclass

import numpy as np

from . import _capi
from ._capi import CH_COUNT_DOMAIN_ERROR, KernelStat, Octagon, load

__all__ = ["Context", "ConvexHullError", "DomainError", "CapacityError", "FilterResult", "Server",
           "default_context", "filter", "hull", "load"]


class ConvexHullError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_capi.STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


class DomainError(ConvexHullError, ValueError):
    pass


class CapacityError(ConvexHullError):
    pass


class BusyError(ConvexHullError):
    pass


class WaitTimeout(ConvexHullError):
    pass


def _torch():
    import torch
    return torch


def _check_points(xy):
    torch = _torch()
    if not isinstance(xy, torch.Tensor) or not xy.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if xy.dtype != torch.float32 or xy.dim() != 2 or xy.shape[1] != 2:
        raise TypeError("points must be float32 of shape (n, 2)")
    if not xy.is_contiguous():
        raise ValueError("points must be contiguous (interleaved x, y)")
    n = xy.shape[0]
    if n > _capi.CH_MAX_POINTS:
        raise ValueError("too many points")
    return n


@dataclass
class FilterResult:
    survivors: "object"      # torch uint32-valued int64 tensor on the device, ascending
    count: int
    labels: "object | None"  # torch uint8 tensor (n,) or None
    octagon: "dict | None"   # {'kx','ky','idx'} numpy arrays in slot order E..SE


class Context:
    """A library context bound to one HIP device, with a cached workspace."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        self._lib = load()
        self.device = device
        h = ctypes.c_void_p()
        st = self._lib.ch_ctx_create(device, tune_cache.encode() if tune_cache else None, ctypes.byref(h))
        if st != _capi.CH_OK:
            raise ConvexHullError(st, "ch_ctx_create failed")
        self._h = h
        self._ws = None

    # -- plumbing ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.ch_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st: int):
        detail = self._lib.ch_last_error(self._h).decode(errors="replace")
        if st == _capi.CH_E_DOMAIN:
            raise DomainError(st, detail)
        if st == _capi.CH_E_CAPACITY:
            raise CapacityError(st, detail)
        raise ConvexHullError(st, detail)

    def workspace(self, nbytes: int):
        """A device byte buffer of at least nbytes (reused across calls)."""
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def stream_handle(self):
        torch = _torch()
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # -- entry points -----------------------------------------------------
    def filter_async(self, xy, survivors, count, labels=None, octagon_dev=None):
        """ch_filter on caller-provided device buffers (uint32 views as int32
        tensors); enqueues on the current stream and returns immediately."""
        n = _check_points(xy)
        ws_bytes = self._lib.ch_filter_workspace_bytes(n)
        ws = self.workspace(ws_bytes)
        st = self._lib.ch_filter(
            self._h, ctypes.c_void_p(xy.data_ptr()), n, ctypes.c_void_p(survivors.data_ptr()),
            ctypes.c_void_p(count.data_ptr()),
            ctypes.c_void_p(labels.data_ptr()) if labels is not None else None,
            ctypes.c_void_p(octagon_dev.data_ptr()) if octagon_dev is not None else None,
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)

    def filter_noalloc_async(self, xy, survivors, count, labels=None, octagon_dev=None):
        """ch_filter_noalloc: as filter_async, with the library's fixed
        device scratch instead of a workspace (at most
        CH_FILTER_NOALLOC_MAX_POINTS points; nothing is allocated)."""
        n = _check_points(xy)
        st = self._lib.ch_filter_noalloc(
            self._h, ctypes.c_void_p(xy.data_ptr()), n, ctypes.c_void_p(survivors.data_ptr()),
            ctypes.c_void_p(count.data_ptr()),
            ctypes.c_void_p(labels.data_ptr()) if labels is not None else None,
            ctypes.c_void_p(octagon_dev.data_ptr()) if octagon_dev is not None else None,
            self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)

    def filter(self, xy, labels: bool = False, octagon: bool = False) -> FilterResult:
        torch = _torch()
        n = _check_points(xy)
        dev = xy.device
        surv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        cnt = torch.empty(1, dtype=torch.int32, device=dev)
        lab = torch.empty(max(n, 1), dtype=torch.uint8, device=dev) if labels else None
        octd = torch.empty(24, dtype=torch.int32, device=dev) if octagon else None
        self.filter_async(xy, surv, cnt, lab, octd)
        c = int(cnt.cpu().numpy().view(np.uint32)[0])
        if c == CH_COUNT_DOMAIN_ERROR:
            raise DomainError(_capi.CH_E_DOMAIN, "input outside the 2^-20 grid on [0,1)")
        oct_np = None
        if octagon and n:
            o = octd.cpu().numpy()
            oct_np = {"kx": o[0:8].copy(), "ky": o[8:16].copy(), "idx": o[16:24].view(np.uint32).copy()}
        return FilterResult(survivors=surv[:c], count=c, labels=lab[:n] if labels else None,
                            octagon=oct_np)

    def hull(self, xy, cap: int | None = None) -> np.ndarray:
        """Counter-clockwise hull vertex indices (uint32 numpy array)."""
        n = _check_points(xy)
        ws_bytes = self._lib.ch_hull_workspace_bytes(n)
        ws = self.workspace(ws_bytes)
        if cap is None:
            cap = max(min(n, 1 << 21), 1)
        out = np.empty(cap, np.uint32)
        h = ctypes.c_uint32(0)
        st = self._lib.ch_hull(self._h, ctypes.c_void_p(xy.data_ptr()), n,
                               out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(h),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)
        return out[: h.value].copy()

    @staticmethod
    def _extremes_mode(extremes: str) -> int:
        modes = {"fused": _capi.CH_EXTREMES_FUSED, "two_kernels": _capi.CH_EXTREMES_TWO_KERNELS}
        if extremes not in modes:
            raise ValueError(f"extremes must be one of {sorted(modes)}")
        return modes[extremes]

    def gpufilter_async(self, xy, labels, octagon_dev=None, count=None, extremes: str = "two_kernels"):
        """ch_gpufilter (Alg. 2) on caller-provided device buffers: labels
        (n,) uint8, optional octagon (24,) int32 and count (1,) int32;
        enqueues on the current stream and returns immediately."""
        n = _check_points(xy)
        mode = self._extremes_mode(extremes)
        ws = self.workspace(self._lib.ch_gpufilter_workspace_bytes(n))
        st = self._lib.ch_gpufilter(
            self._h, ctypes.c_void_p(xy.data_ptr()), n, mode, ctypes.c_void_p(labels.data_ptr()),
            ctypes.c_void_p(octagon_dev.data_ptr()) if octagon_dev is not None else None,
            ctypes.c_void_p(count.data_ptr()) if count is not None else None,
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)

    def gpufilter(self, xy, extremes: str = "two_kernels"):
        """Alg. 2: (labels as a device uint8 tensor, octagon dict, survivor
        count)."""
        torch = _torch()
        n = _check_points(xy)
        dev = xy.device
        lab = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        octd = torch.empty(24, dtype=torch.int32, device=dev)
        cnt = torch.empty(1, dtype=torch.int32, device=dev)
        self.gpufilter_async(xy, lab, octd, cnt, extremes)
        c = int(cnt.cpu().numpy().view(np.uint32)[0])
        if c == CH_COUNT_DOMAIN_ERROR:
            raise DomainError(_capi.CH_E_DOMAIN, "input outside the 2^-20 grid on [0,1)")
        oct_np = None
        if n:
            o = octd.cpu().numpy()
            oct_np = {"kx": o[0:8].copy(), "ky": o[8:16].copy(), "idx": o[16:24].view(np.uint32).copy()}
        return lab[:n], oct_np, c

    def hull_queues(self, xy, extremes: str = "fused", cap: int | None = None):
        """ch_hull_queues (Alg. 1 with its four queues): returns (hull
        indices, queue sizes) as numpy uint32 arrays."""
        n = _check_points(xy)
        mode = self._extremes_mode(extremes)
        ws = self.workspace(self._lib.ch_hull_queues_workspace_bytes(n))
        if cap is None:
            cap = max(min(n, 1 << 21), 1)
        out = np.empty(cap, np.uint32)
        qc = np.zeros(4, np.uint32)
        h = ctypes.c_uint32(0)
        st = self._lib.ch_hull_queues(self._h, ctypes.c_void_p(xy.data_ptr()), n, mode,
                                      out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(h),
                                      qc.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel(), self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)
        return out[: h.value].copy(), qc

    def read_stream_async(self, buf, blocks: int = 0):
        """ch_diag_read_stream over a contiguous device tensor (its bytes,
        rounded down to a multiple of 16), on the current stream."""
        nbytes = (buf.numel() * buf.element_size()) & ~15
        st = self._lib.ch_diag_read_stream(self._h, ctypes.c_void_p(buf.data_ptr()), nbytes, blocks,
                                           self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)
        return nbytes

    def last_hull_info(self) -> dict:
        """Counts of the last successful hull() on this context."""
        info = _capi.HullInfo()
        self._lib.ch_last_hull_info(self._h, ctypes.byref(info))
        return {f: getattr(info, f) for f, _ in _capi.HullInfo._fields_}

    def hull_batch_async(self, xy, off, hull_idx, hull_count, ws=None):
        """ch_hull_batch on device tensors: xy (N,2) float32, off (nsets+1)
        int64 (uint64 offsets), hull_idx (N,) int32, hull_count (nsets,) int32.
        Enqueues on the current stream and returns."""
        torch = _torch()
        n = _check_points(xy)
        if off.dtype != torch.int64 or not off.is_cuda or off.dim() != 1:
            raise TypeError("offsets must be a 1-D int64 CUDA tensor")
        nsets = off.numel() - 1
        nbytes = self._lib.ch_hull_batch_workspace_bytes(nsets, n)
        if ws is None:
            ws = self.workspace(nbytes)
        st = self._lib.ch_hull_batch(
            self._h, ctypes.c_void_p(xy.data_ptr()), ctypes.c_void_p(off.data_ptr()), nsets, n,
            ctypes.c_void_p(hull_idx.data_ptr()), ctypes.c_void_p(hull_count.data_ptr()),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), self.stream_handle())
        if st != _capi.CH_OK:
            self._raise(st)

    def hull_batch(self, xy, off):
        """Hulls of the sets [off[s], off[s+1]) of xy: returns (hull_idx,
        counts) as numpy uint32 arrays; set s's local indices are
        hull_idx[off[s] : off[s] + counts[s]] when counts[s] is a count."""
        torch = _torch()
        n = _check_points(xy)
        nsets = off.numel() - 1
        idx = torch.empty(max(n, 1), dtype=torch.int32, device=xy.device)
        cnt = torch.empty(max(nsets, 1), dtype=torch.int32, device=xy.device)
        self.hull_batch_async(xy, off, idx, cnt)
        return idx.cpu().numpy().view(np.uint32)[:n], cnt.cpu().numpy().view(np.uint32)[:nsets]

    @staticmethod
    def _params_dict(p) -> dict:
        return {"tile_points": p.tile_points, "pass_blocks": p.pass_blocks,
                "hull_blocks": p.hull_blocks, "sample_min": p.sample_min}

    def batch_params(self, nsets: int = 1, total_points: int = 1) -> dict:
        """The batch parameters a call of this shape would use."""
        p = _capi.BatchParams()
        st = self._lib.ch_batch_params_get(self._h, nsets, total_points, ctypes.byref(p))
        if st != _capi.CH_OK:
            self._raise(st)
        return self._params_dict(p)

    def set_batch_params(self, params: dict | None):
        """Fix the batch parameters (None: back to tuned / default ones)."""
        if params is None:
            st = self._lib.ch_batch_params_set(self._h, None)
        else:
            p = _capi.BatchParams(params["tile_points"], params["pass_blocks"], params["hull_blocks"],
                                  params["sample_min"])
            st = self._lib.ch_batch_params_set(self._h, ctypes.byref(p))
        if st != _capi.CH_OK:
            self._raise(st)

    def tune_batch(self, xy, off, hull_idx, hull_count, ws=None) -> dict:
        """ch_tune_batch on device tensors (as hull_batch_async); returns the
        chosen parameters. Synchronous."""
        torch = _torch()
        n = _check_points(xy)
        if off.dtype != torch.int64 or not off.is_cuda or off.dim() != 1:
            raise TypeError("offsets must be a 1-D int64 CUDA tensor")
        nsets = off.numel() - 1
        if ws is None:
            ws = self.workspace(self._lib.ch_hull_batch_workspace_bytes(nsets, n))
        best = _capi.BatchParams()
        st = self._lib.ch_tune_batch(
            self._h, ctypes.c_void_p(xy.data_ptr()), ctypes.c_void_p(off.data_ptr()), nsets, n,
            ctypes.c_void_p(hull_idx.data_ptr()), ctypes.c_void_p(hull_count.data_ptr()),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), self.stream_handle(), ctypes.byref(best))
        if st != _capi.CH_OK:
            self._raise(st)
        return self._params_dict(best)

    def serve(self, arena, n_streams: int = 4, max_inflight: int = 0,
              max_batch_points: int = 0) -> "Server":
        """Start a request server on this context's device (ch_serve_start)."""
        return Server(self, arena, n_streams, max_inflight, max_batch_points)

    # -- profiling --------------------------------------------------------
    def profile_enable(self, on: bool = True):
        self._lib.ch_profile_enable(self._h, 1 if on else 0)

    def profile_reset(self):
        self._lib.ch_profile_reset(self._h)

    def profile_read(self) -> dict:
        arr = (KernelStat * 64)()
        n = ctypes.c_int(0)
        self._lib.ch_profile_read(self._h, ctypes.cast(arr, ctypes.c_void_p), 64, ctypes.byref(n))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms))
                for i in range(min(n.value, 64))}


def _host_points(xy):
    """(pointer, n, keep-alive object) for a host float32 (n, 2) array: a
    numpy array or a CPU torch tensor (pinned memory is copied by DMA)."""
    if isinstance(xy, np.ndarray):
        if xy.dtype != np.float32 or xy.ndim != 2 or xy.shape[1] != 2 or not xy.flags.c_contiguous:
            raise TypeError("points must be a C-contiguous float32 array of shape (n, 2)")
        return xy.ctypes.data, xy.shape[0], xy
    torch = _torch()
    if isinstance(xy, torch.Tensor):
        if xy.is_cuda:
            raise TypeError("serve requests are host arrays")
        if xy.dtype != torch.float32 or xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_contiguous():
            raise TypeError("points must be a contiguous float32 tensor of shape (n, 2)")
        return xy.data_ptr(), xy.shape[0], xy
    raise TypeError("points must be a numpy array or a CPU torch tensor")


class Server:
    """A running ch_serve server: submit host point sets, wait for their hulls.

    The arena (a device uint8 tensor) is the admission budget; the server
    splits it into one slot per stream and never allocates device memory.
    Submitted arrays are kept referenced until their ticket is collected."""

    def __init__(self, ctx: Context, arena, n_streams: int = 4, max_inflight: int = 0,
                 max_batch_points: int = 0):
        torch = _torch()
        if not isinstance(arena, torch.Tensor) or not arena.is_cuda or arena.dtype != torch.uint8:
            raise TypeError("arena must be a CUDA uint8 tensor")
        self._lib = ctx._lib
        self._ctx = ctx
        self._arena = arena
        self._cfg = _capi.ServeConfig(arena.data_ptr(), arena.numel(), max_inflight, n_streams,
                                      max_batch_points)
        h = ctypes.c_void_p()
        st = self._lib.ch_serve_start(ctx._h, ctypes.byref(self._cfg), ctypes.byref(h))
        if st != _capi.CH_OK:
            raise ConvexHullError(st, "ch_serve_start failed")
        self._h = h
        self._keep = {}
        self._mu = threading.Lock()

    @property
    def max_request_points(self) -> int:
        return int(self._lib.ch_serve_max_request_points(ctypes.byref(self._cfg)))

    def submit(self, xy) -> int:
        """Queue one request; returns its ticket. Raises BusyError when
        max_inflight requests are outstanding."""
        ptr, n, keep = _host_points(xy)
        t = ctypes.c_uint64(0)
        st = self._lib.ch_serve_submit(self._h, ctypes.c_void_p(ptr), n, ctypes.byref(t))
        if st == _capi.CH_E_BUSY:
            raise BusyError(st, "too many requests in flight")
        if st != _capi.CH_OK:
            raise ConvexHullError(st, "ch_serve_submit failed")
        with self._mu:
            self._keep[t.value] = (keep, n)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        """(hull indices uint32, [arrive, admit, done] ns) of a ticket.
        Raises WaitTimeout (ticket kept), DomainError, or ConvexHullError."""
        with self._mu:
            n = self._keep[ticket][1] if ticket in self._keep else 0
        cap = max(min(n, 1 << 21), 1)
        out = np.empty(cap, np.uint32)
        h = ctypes.c_uint32(0)
        tns = np.zeros(3, np.uint64)
        st = self._lib.ch_serve_wait(self._h, ticket, timeout_us, out.ctypes.data_as(ctypes.c_void_p), cap,
                                     ctypes.byref(h), tns.ctypes.data_as(ctypes.c_void_p))
        if st == _capi.CH_E_TIMEOUT:
            raise WaitTimeout(st, f"ticket {ticket} not done")
        if st not in (_capi.CH_E_NOT_FOUND, _capi.CH_E_CAPACITY):
            with self._mu:
                self._keep.pop(ticket, None)
        if st == _capi.CH_E_DOMAIN:
            raise DomainError(st, f"ticket {ticket}: input outside the 2^-20 grid on [0,1)")
        if st != _capi.CH_OK:
            raise ConvexHullError(st, f"ticket {ticket}")
        return out[: h.value].copy(), tns

    def stats(self) -> dict:
        c, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
        r, p50, p99 = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        self._lib.ch_serve_stats(self._h, ctypes.byref(c), ctypes.byref(b), ctypes.byref(r),
                                 ctypes.byref(p50), ctypes.byref(p99))
        return {"completed": c.value, "batches": b.value, "hulls_per_s": r.value,
                "p50_us": p50.value, "p99_us": p99.value}

    def stop(self):
        if getattr(self, "_h", None):
            self._lib.ch_serve_stop(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


_default = None


def default_context() -> Context:
    global _default
    if _default is None:
        _default = Context(0)
    return _default


def filter(xy, labels: bool = False, octagon: bool = False) -> FilterResult:  # noqa: A001
    return default_context().filter(xy, labels=labels, octagon=octagon)


def hull(xy, cap: int | None = None) -> np.ndarray:
    return default_context().hull(xy, cap)

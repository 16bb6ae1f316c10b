"""CPU oracle for the heaphull-style convex hull.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_2209_12310_amd``) never imports it, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, exact int64 predicates); this
module only marshals numpy arrays.  Each function names the passage of the
paper (Keith, Ferrada, Navarro, arXiv 2209.12310) it follows:

* ``to_grid``      -- the input of Alg. 1/2 ("n points in 2D"), read as float32
                      on the 2^-20 grid in [0, 1).
* ``extremes``     -- findExtremes as Sec. III does it on the GPU: axis extremes
                      N, S, E, W, then the Manhattan-closest point to each box
                      corner.
* ``filter``       -- the outside test of Alg. 1 and the labels of Alg. 2, with
                      the boundary rule of Sec. I (stage 1).
* ``chain``        -- Andrew's monotone chain (Table I) over a candidate set.
* ``heaphull``     -- the pipeline of Alg. 1 with the four queues merged into
                      one candidate set (the hull of the union is unique).
* ``filter_parallel`` -- the divide-and-conquer CPU variant of Sec. III.
* ``heaphull_queues`` -- Alg. 1, stages (2)-(4): the four queues built from
                      Alg. 2's label array, a hull per queue, their union.
* ``heaphull_parallel`` / ``chain_parallel`` -- the same on every host core
                      (the CPU baseline of the measurements).

Parity unpinned by the paper: the queue label rule (the paper gives no
findQueue rule).  Everything else is pinned by the tests in
``tests/test_oracle.py`` against brute force, closed forms and invariants.

``build()`` compiles a portable library (with the planted-mistake switch the
tests use); ``native()`` compiles, on the host that runs it, an ``-O3
-march=native`` copy with that switch compiled out, for timing the CPU
baseline.  Both are the same source and arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SLOTS = ("E", "NE", "N", "NW", "W", "SW", "S", "SE")


class DomainError(ValueError):
    """A coordinate is not k * 2^-20 with integer k in [0, 2^20)."""

    def __init__(self, index: int):
        super().__init__(f"point {index} is outside the 2^-20 grid on [0,1)")
        self.index = index


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no -march flags, so
    the library runs on any x86-64 host)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(lib):
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.or_to_grid.argtypes = [P, I64, P, P]
    lib.or_to_grid.restype = I64
    lib.or_extremes.argtypes = [P, P, I64, P]
    lib.or_extremes.restype = None
    lib.or_filter.argtypes = [P, P, I64, P, P, P]
    lib.or_filter.restype = I64
    lib.or_filter_parallel.argtypes = [P, P, I64, P, P, ctypes.c_int]
    lib.or_filter_parallel.restype = I64
    lib.or_chain.argtypes = [P, P, I64, P, I64, P]
    lib.or_chain.restype = I64
    lib.or_heaphull.argtypes = [P, P, I64, P, P]
    lib.or_heaphull.restype = I64
    lib.or_set_mutation.argtypes = [ctypes.c_int]
    lib.or_set_mutation.restype = None
    lib.or_max_threads.restype = ctypes.c_int
    lib.or_chain_parallel.argtypes = [P, P, I64, P, I64, P, ctypes.c_int]
    lib.or_chain_parallel.restype = I64
    lib.or_heaphull_queues.argtypes = [P, P, I64, P, P, P, P, ctypes.c_int]
    lib.or_heaphull_queues.restype = I64
    lib.or_heaphull_parallel.argtypes = [P, P, I64, P, ctypes.c_int]
    lib.or_heaphull_parallel.restype = I64
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


_native = None


def native():
    """The oracle compiled on this host with ``-O3 -march=native`` and the
    planted-mistake switch compiled out (a private temporary copy). Returns an
    object with the same functions as this module's ``heaphull``,
    ``heaphull_parallel`` and ``heaphull_queues``."""
    global _native
    if _native is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="oracle_native_")
        path = os.path.join(d, "liboracle_native.so")
        subprocess.check_call(["gcc", "-O3", "-march=native", "-DOR_NO_MUTATION", "-std=c11",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", path, "-lm"])
        _native = _Oracle(_bind(ctypes.CDLL(path)))
    return _native


class _Oracle:
    """Entry points bound to one compiled copy of the oracle."""

    def __init__(self, lib):
        self.lib = lib

    def heaphull(self, kx, ky):
        return heaphull(kx, ky, lib=self.lib)

    def heaphull_parallel(self, kx, ky, nthreads=0):
        return heaphull_parallel(kx, ky, nthreads, lib=self.lib)

    def heaphull_queues(self, kx, ky, labels, oct_idx=None, nthreads=1):
        return heaphull_queues(kx, ky, labels, oct_idx, nthreads, lib=self.lib)

    def max_threads(self):
        return int(self.lib.or_max_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_mutation(m: int) -> None:
    """Plant a known mistake in the oracle (0 restores it). Used only by the
    test showing that the pins catch such mistakes."""
    _load().or_set_mutation(int(m))


def max_threads() -> int:
    return int(_load().or_max_threads())


def to_grid(xy) -> tuple[np.ndarray, np.ndarray]:
    """(n,2) float32 -> (kx, ky) int32 grid coordinates; raises DomainError."""
    xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)
    n = xy.shape[0]
    kx = np.empty(n, np.int32)
    ky = np.empty(n, np.int32)
    bad = _load().or_to_grid(_ptr(xy), n, _ptr(kx), _ptr(ky))
    if bad >= 0:
        raise DomainError(int(bad))
    return kx, ky


def _k(kx, ky):
    return np.ascontiguousarray(kx, np.int32), np.ascontiguousarray(ky, np.int32)


def extremes(kx, ky) -> np.ndarray:
    """Indices of the 8 octagon vertices in slot order E, NE, N, NW, W, SW, S, SE."""
    kx, ky = _k(kx, ky)
    if kx.size == 0:
        raise ValueError("extremes of an empty set")
    out = np.empty(8, np.int64)
    _load().or_extremes(_ptr(kx), _ptr(ky), kx.size, _ptr(out))
    return out


def filter(kx, ky, oct_idx=None):  # noqa: A001 - the paper's name for the stage
    """Survivors (ascending uint32 indices) and per-point labels (uint8)."""
    kx, ky = _k(kx, ky)
    n = kx.size
    if n == 0:
        return np.empty(0, np.uint32), np.empty(0, np.uint8)
    if oct_idx is None:
        oct_idx = extremes(kx, ky)
    oct_idx = np.ascontiguousarray(oct_idx, np.int64)
    surv = np.empty(n, np.uint32)
    lab = np.empty(n, np.uint8)
    m = _load().or_filter(_ptr(kx), _ptr(ky), n, _ptr(oct_idx), _ptr(surv), _ptr(lab))
    return surv[:m].copy(), lab


def filter_parallel(kx, ky, nthreads: int = 0):
    """Divide-and-conquer multi-core filter; returns (octagon indices, survivors)."""
    kx, ky = _k(kx, ky)
    n = kx.size
    oct_idx = np.empty(8, np.int64)
    surv = np.empty(max(n, 1), np.uint32)
    if n == 0:
        return oct_idx[:0], surv[:0]
    m = _load().or_filter_parallel(_ptr(kx), _ptr(ky), n, _ptr(oct_idx), _ptr(surv), int(nthreads))
    return oct_idx, surv[:m].copy()


def chain(kx, ky, cand=None) -> np.ndarray:
    """Andrew's monotone chain over ``cand`` (all points when None)."""
    kx, ky = _k(kx, ky)
    n = kx.size
    if cand is None:
        m = n
        hull = np.empty(max(m, 1), np.uint32)
        h = _load().or_chain(_ptr(kx), _ptr(ky), n, None, 0, _ptr(hull))
    else:
        cand = np.ascontiguousarray(cand, np.uint32)
        m = cand.size
        hull = np.empty(max(m, 1), np.uint32)
        h = _load().or_chain(_ptr(kx), _ptr(ky), n, _ptr(cand), m, _ptr(hull))
    return hull[:h].copy()


def heaphull(kx, ky, lib=None) -> np.ndarray:
    """Alg. 1: extremes, octagon filter, chain over the survivors."""
    kx, ky = _k(kx, ky)
    n = kx.size
    surv = np.empty(max(n, 1), np.uint32)
    hull = np.empty(max(n, 1), np.uint32)
    h = (lib or _load()).or_heaphull(_ptr(kx), _ptr(ky), n, _ptr(surv), _ptr(hull))
    return hull[:h].copy()


def chain_parallel(kx, ky, cand=None, nthreads: int = 0) -> np.ndarray:
    """``chain`` with the sort on ``nthreads`` threads (0: all)."""
    kx, ky = _k(kx, ky)
    n = kx.size
    m = n if cand is None else len(cand)
    hull = np.empty(max(m, 1), np.uint32)
    if cand is None:
        h = _load().or_chain_parallel(_ptr(kx), _ptr(ky), n, None, 0, _ptr(hull), int(nthreads))
    else:
        cand = np.ascontiguousarray(cand, np.uint32)
        h = _load().or_chain_parallel(_ptr(kx), _ptr(ky), n, _ptr(cand), m, _ptr(hull), int(nthreads))
    return hull[:h].copy()


def heaphull_queues(kx, ky, labels, oct_idx=None, nthreads: int = 1, lib=None):
    """Alg. 1, stages (2)-(4), from Alg. 2's label array: returns (hull,
    queue sizes). ``oct_idx`` defaults to the octagon of ``extremes``."""
    kx, ky = _k(kx, ky)
    n = kx.size
    if n == 0:
        return np.empty(0, np.uint32), np.zeros(4, np.int64)
    if oct_idx is None:
        oct_idx = extremes(kx, ky)
    oct_idx = np.ascontiguousarray(oct_idx, np.int64)
    labels = np.ascontiguousarray(labels, np.uint8)
    if labels.size != n:
        raise ValueError("one label per point")
    hull = np.empty(n + 4, np.uint32)
    qc = np.zeros(4, np.int64)
    h = (lib or _load()).or_heaphull_queues(_ptr(kx), _ptr(ky), n, _ptr(oct_idx), _ptr(labels),
                                            _ptr(hull), _ptr(qc), int(nthreads))
    return hull[:h].copy(), qc


def heaphull_parallel(kx, ky, nthreads: int = 0, lib=None) -> np.ndarray:
    """The full heaphull on ``nthreads`` host threads (0: all): parallel
    extremes and filter, labels, four queues, each hulled in parallel."""
    kx, ky = _k(kx, ky)
    n = kx.size
    hull = np.empty(max(n, 1), np.uint32)
    h = (lib or _load()).or_heaphull_parallel(_ptr(kx), _ptr(ky), n, _ptr(hull), int(nthreads))
    return hull[:h].copy()


def hull(xy) -> np.ndarray:
    """Counter-clockwise hull vertex indices of float32 points on the grid."""
    kx, ky = to_grid(xy)
    return heaphull(kx, ky)


def octagon(xy) -> dict:
    """The octagon as the GPU library reports it: grid coordinates and the
    smallest index holding each vertex, in slot order."""
    kx, ky = to_grid(xy)
    idx = extremes(kx, ky)
    vx = kx[idx].astype(np.int32)
    vy = ky[idx].astype(np.int32)
    first = np.empty(8, np.uint32)
    for k in range(8):
        first[k] = np.flatnonzero((kx == vx[k]) & (ky == vy[k]))[0]
    return {"kx": vx, "ky": vy, "idx": first}

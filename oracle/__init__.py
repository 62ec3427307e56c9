"""CPU oracle for the Wedge pull-only frontier method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it, and the
two share no code: the only inputs both sides see come from the seeded
generators in ``gen``.

The arithmetic lives in ``oracle.c`` (plain C, FP64 where floating point is
involved); this module only marshals numpy arrays. Every result here is pinned
by tests against brute force, closed forms or independent library routines
(see ``tests/test_oracle_pins.py``); nothing is "parity unpinned".

Graphs are CSR: ``row_off`` uint64[n+1], ``col`` uint32[m] (out-neighbours).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# WEDGE_ORACLE_LIB selects another build (the address/undefined-behaviour sanitizer
# build, liboracle_asan.so, in the host sanitizer test)
_SO = os.environ.get("WEDGE_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SO_ASAN = os.path.join(_HERE, "liboracle_asan.so")
_lib = None

INF = 0xFFFFFFFF
APP = {"bfs": 1, "cc": 2, "sssp": 3}


SANITIZE = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
            "-fno-sanitize-recover=undefined"]


def build(sanitize: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc -O2, OpenMP); with sanitize, into
    liboracle_asan.so under AddressSanitizer and UBSan (host code only)."""
    src = os.path.join(_HERE, "oracle.c")
    out = _SO_ASAN if sanitize else os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    flags = SANITIZE if sanitize else ["-O2"]
    subprocess.check_call(["gcc", *flags, "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    c = ctypes
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
    vp = c.c_void_p
    lib.or_csc_from_csr.argtypes = [c.c_uint32, u64p, u32p, vp, u64p, u32p, vp]
    lib.or_symmetrize.argtypes = [c.c_uint32, u64p, u32p, u64p, u32p]
    lib.or_symmetrize.restype = c.c_uint64
    lib.or_bfs_levels.argtypes = [c.c_uint32, u64p, u32p, c.c_uint32, u32p]
    lib.or_wcc_labels.argtypes = [c.c_uint32, u64p, u32p, u32p]
    lib.or_sssp_dist.argtypes = [c.c_uint32, u64p, u32p, u32p, c.c_uint32, u32p]
    lib.or_sssp_dist.restype = c.c_int
    lib.or_pagerank.argtypes = [c.c_uint32, u64p, u32p, c.c_uint32, c.c_double, f64p, c.c_int]
    lib.or_wedge_frontier.argtypes = [c.c_uint64, u32p, u8p, c.c_uint32, u8p]
    lib.or_wedge_frontier.restype = c.c_uint64
    lib.or_pull_engine.argtypes = [c.c_int, c.c_uint32, u64p, u32p, vp, c.c_uint32, c.c_uint64,
                                   c.c_uint32, c.c_uint32, u32p, vp, vp, vp, vp, vp, vp, c.c_int]
    lib.or_pull_engine.restype = c.c_int64
    lib.or_push_engine.argtypes = [c.c_int, c.c_uint32, u64p, u32p, vp, c.c_uint32, c.c_uint32,
                                   u32p, vp]
    lib.or_push_engine.restype = c.c_int64
    lib.or_threads.restype = c.c_int
    _lib = lib
    return lib


def _csr(row_off, col):
    return (np.ascontiguousarray(row_off, dtype=np.uint64),
            np.ascontiguousarray(col if len(col) else np.zeros(1, np.uint32), dtype=np.uint32))


def threads() -> int:
    return int(_load().or_threads())


def csc(row_off, col, w=None):
    """(col_off uint64[n+1], in_src uint32[m], in_w uint32[m] or None); sources ascend per vertex."""
    lib = _load()
    n = len(row_off) - 1
    m = int(row_off[-1])
    ro, cl = _csr(row_off, col)
    col_off = np.zeros(n + 1, np.uint64)
    in_src = np.zeros(max(m, 1), np.uint32)
    in_w = np.zeros(max(m, 1), np.uint32) if w is not None else None
    wa = np.ascontiguousarray(w, np.uint32) if w is not None else None
    lib.or_csc_from_csr(n, ro, cl, wa.ctypes.data if wa is not None else None, col_off, in_src,
                        in_w.ctypes.data if in_w is not None else None)
    return col_off, in_src[:m], (in_w[:m] if in_w is not None else None)


def symmetrize(row_off, col):
    """Undirected view as a CSR (both directions, no self-loops, no duplicates)."""
    lib = _load()
    n = len(row_off) - 1
    m = int(row_off[-1])
    ro, cl = _csr(row_off, col)
    out_ro = np.zeros(n + 1, np.uint64)
    out_col = np.zeros(max(2 * m, 1), np.uint32)
    k = lib.or_symmetrize(n, ro, cl, out_ro, out_col)
    return out_ro, out_col[:k].copy()


def bfs(row_off, col, src):
    n = len(row_off) - 1
    out = np.empty(max(n, 1), np.uint32)
    _load().or_bfs_levels(n, *_csr(row_off, col), src, out)
    return out[:n]


def cc(row_off, col):
    """Min-id label of each weakly connected component."""
    n = len(row_off) - 1
    out = np.empty(max(n, 1), np.uint32)
    _load().or_wcc_labels(n, *_csr(row_off, col), out)
    return out[:n]


def sssp(row_off, col, w, src):
    n = len(row_off) - 1
    out = np.empty(max(n, 1), np.uint32)
    wa = np.ascontiguousarray(w if len(w) else np.zeros(1, np.uint32), np.uint32)
    rc = _load().or_sssp_dist(n, *_csr(row_off, col), wa, src, out)
    if rc != 0:
        raise OverflowError("a shortest-path distance does not fit in 32 bits")
    return out[:n]


def pagerank(row_off, col, iters=20, damping=0.85, threads=0):
    n = len(row_off) - 1
    out = np.empty(max(n, 1), np.float64)
    _load().or_pagerank(n, *_csr(row_off, col), iters, damping, out, threads)
    return out[:n]


def wedge_frontier(in_src, frontier, chunk):
    """Marked edge groups (uint8 per group) of a vertex frontier (uint8 per vertex)."""
    m = len(in_src)
    groups = (m + chunk - 1) // chunk
    bits = np.zeros(max(groups, 1), np.uint8)
    src = np.ascontiguousarray(in_src if m else np.zeros(1, np.uint32), np.uint32)
    fr = np.ascontiguousarray(frontier if len(frontier) else np.zeros(1, np.uint8), np.uint8)
    k = _load().or_wedge_frontier(m, src, fr, chunk, bits)
    return bits[:groups], int(k)


def threshold_edges(theta_ppm: int, m: int) -> int:
    """Fullness threshold in edges: floor(theta * m) with theta in parts per million."""
    return (int(theta_ppm) * int(m)) // 1_000_000


class PullTrace:
    """Result of the pull engine: final values and one row per iteration."""

    def __init__(self, values, iters, F, A, mode, K, edges, frontiers):
        self.values, self.iters = values, iters
        self.F, self.A, self.mode, self.K, self.edges = F, A, mode, K, edges
        self.frontiers = frontiers


def pull_engine(app, row_off, col, w=None, src=0, theta_ppm=10_000, chunk=32, max_iters=100000,
                keep_frontiers=False, threads=0):
    """Synchronous pull with the fullness decision; for "cc" pass the undirected view."""
    lib = _load()
    n = len(row_off) - 1
    m = int(row_off[-1])
    thr = threshold_edges(theta_ppm, m)
    cap = max_iters
    # the trace arrays need one slot per iteration; n+1 bounds BFS, CC and SSSP with
    # positive weights is bounded by n as well, so cap at n + 2 to keep memory small
    cap = min(cap, n + 2)
    val = np.empty(max(n, 1), np.uint32)
    F = np.zeros(cap, np.uint64)
    A = np.zeros(cap, np.uint64)
    mode = np.zeros(cap, np.uint8)
    K = np.zeros(cap, np.uint64)
    E = np.zeros(cap, np.uint64)
    frs = np.zeros((cap, n), np.uint8) if keep_frontiers else None
    wa = np.ascontiguousarray(w, np.uint32) if w is not None else None
    it = lib.or_pull_engine(APP[app], n, *_csr(row_off, col),
                            wa.ctypes.data if wa is not None else None, src, thr, chunk,
                            cap, val, F.ctypes.data, A.ctypes.data, mode.ctypes.data,
                            K.ctypes.data, E.ctypes.data,
                            frs.ctypes.data if frs is not None else None, threads)
    if it < 0:
        raise RuntimeError("pull engine did not converge within max_iters")
    return PullTrace(val[:n], int(it), F[:it], A[:it], mode[:it], K[:it], E[:it],
                     frs[:it] if frs is not None else None)


def push_engine(app, row_off, col, w=None, src=0, max_iters=100000):
    lib = _load()
    n = len(row_off) - 1
    cap = min(max_iters, n + 2)
    val = np.empty(max(n, 1), np.uint32)
    F = np.zeros(cap, np.uint64)
    wa = np.ascontiguousarray(w, np.uint32) if w is not None else None
    it = lib.or_push_engine(APP[app], n, *_csr(row_off, col),
                            wa.ctypes.data if wa is not None else None, src, cap, val,
                            F.ctypes.data)
    if it < 0:
        raise RuntimeError("push engine did not converge within max_iters")
    return val[:n], int(it), F[:it]

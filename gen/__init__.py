"""Seeded synthetic graph inputs (R-MAT, Erdos-Renyi, weights, sources).

Input generation only: nothing here computes any part of the graph-processing
method. Both the GPU library's tests/benchmarks and the CPU oracle take their
graphs from this module. All randomness is counter based (see gen.c), so every
output is a pure function of its seed and sizes.

Graphs come back as a sorted, de-duplicated CSR without self-loops:
``row_off`` (uint64, n+1) and ``col`` (uint32, m), out-neighbours ascending.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# WEDGE_GEN_LIB selects another build (the address/undefined-behaviour sanitizer
# build, libwedgegen_asan.so, in the host sanitizer test)
_SO = os.environ.get("WEDGE_GEN_LIB") or os.path.join(_HERE, "libwedgegen.so")
_SO_ASAN = os.path.join(_HERE, "libwedgegen_asan.so")
_lib = None

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(sanitize: bool = False) -> str:
    """Compile gen.c into libwedgegen.so (gcc, OpenMP); with sanitize, into
    libwedgegen_asan.so under AddressSanitizer and UBSan."""
    src = os.path.join(_HERE, "gen.c")
    out = _SO_ASAN if sanitize else os.path.join(_HERE, "libwedgegen.so")
    tmp = out + ".tmp"
    flags = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
              "-fno-sanitize-recover=undefined"] if sanitize else ["-O3", "-march=x86-64-v2"])
    subprocess.check_call(["gcc", *flags, "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    c = ctypes
    lib.gen_rmat_edges.argtypes = [c.c_int, c.c_uint64, c.c_double, c.c_double, c.c_double,
                                   c.c_uint64, u32p, u32p]
    lib.gen_uniform_edges.argtypes = [c.c_uint32, c.c_uint64, c.c_uint64, c.c_uint64, u32p, u32p]
    lib.gen_permutation.argtypes = [c.c_uint32, c.c_uint64, u32p]
    lib.gen_apply_permutation.argtypes = [c.c_uint64, u32p, u32p, u32p]
    lib.gen_build_csr.argtypes = [c.c_uint32, c.c_uint64, u32p, u32p, c.c_void_p, u64p, u32p,
                                  c.c_void_p]
    lib.gen_build_csr.restype = c.c_uint64
    lib.gen_filter_tag_below.argtypes = [c.c_uint32, u64p, u32p, u32p, c.c_uint32]
    lib.gen_filter_tag_below.restype = c.c_uint64
    lib.gen_edge_weights.argtypes = [c.c_uint32, u64p, u32p, c.c_uint64, c.c_uint32, c.c_uint32,
                                     u32p]
    lib.gen_pick_sources.argtypes = [c.c_uint32, u64p, c.c_uint32, c.c_uint64, u32p]
    lib.gen_pick_sources.restype = c.c_int
    lib.gen_draw.argtypes = [c.c_uint64, c.c_uint64]
    lib.gen_draw.restype = c.c_uint64
    lib.gen_threads.restype = c.c_int
    _lib = lib
    return lib


def threads() -> int:
    return int(_load().gen_threads())


def draw(seed: int, counter: int) -> int:
    """The raw 64-bit counter-based draw (exposed for tests)."""
    return int(_load().gen_draw(seed, counter))


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray):
    """Sorted, de-duplicated CSR without self-loops from an edge list."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    row_off = np.zeros(n + 1, dtype=np.uint64)
    col = np.empty(max(len(src), 1), dtype=np.uint32)
    m = lib.gen_build_csr(n, len(src), src, dst, None, row_off, col, None)
    return row_off, col[:m].copy()


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, abcd=RMAT_ABCD, permute: bool = True):
    """Directed R-MAT graph with 2**scale vertices and edge_factor * 2**scale draws.

    Vertex ids are relabelled by a seeded random permutation (seed + 0x5EED) so
    that ids carry no degree information; self-loops and duplicate pairs are
    removed.
    """
    lib = _load()
    n = 1 << scale
    m0 = edge_factor * n
    a, b, c, _ = abcd
    src = np.empty(m0, dtype=np.uint32)
    dst = np.empty(m0, dtype=np.uint32)
    lib.gen_rmat_edges(scale, m0, a, b, c, seed, src, dst)
    if permute:
        perm = np.empty(n, dtype=np.uint32)
        lib.gen_permutation(n, seed + 0x5EED, perm)
        lib.gen_apply_permutation(m0, perm, src, dst)
        del perm
    row_off = np.zeros(n + 1, dtype=np.uint64)
    col = np.empty(m0, dtype=np.uint32)
    m = lib.gen_build_csr(n, m0, src, dst, None, row_off, col, None)
    del src, dst
    return row_off, col[:m].copy()


def erdos_renyi(n: int, m: int, seed: int = 2):
    """Directed G(n, m): the first m distinct non-loop pairs in draw order."""
    lib = _load()
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of possible directed edges")
    slack = 1024 + m // 256
    while True:
        cand = m + slack
        if cand >= 2**32:
            raise ValueError("graph too large for 32-bit draw tags")
        src = np.empty(cand, dtype=np.uint32)
        dst = np.empty(cand, dtype=np.uint32)
        lib.gen_uniform_edges(n, cand, seed, 0, src, dst)
        tag = np.arange(cand, dtype=np.uint32)
        row_off = np.zeros(n + 1, dtype=np.uint64)
        col = np.empty(cand, dtype=np.uint32)
        tag_out = np.empty(cand, dtype=np.uint32)
        kept = lib.gen_build_csr(n, cand, src, dst, tag.ctypes.data, row_off, col,
                                 tag_out.ctypes.data)
        del src, dst, tag
        if kept >= m:
            t = tag_out[:kept]
            cutoff = int(np.partition(t, m - 1)[m - 1]) + 1 if m > 0 else 0
            got = lib.gen_filter_tag_below(n, row_off, col, tag_out, cutoff)
            assert got == m
            return row_off, col[:m].copy()
        slack *= 4


def edge_weights(row_off: np.ndarray, col: np.ndarray, seed: int = 4, lo: int = 1, hi: int = 255):
    """uint32 weight per CSR edge, a hash of (u, v, seed) mapped into [lo, hi]."""
    lib = _load()
    n = len(row_off) - 1
    w = np.empty(max(len(col), 1), dtype=np.uint32)
    lib.gen_edge_weights(n, np.ascontiguousarray(row_off, np.uint64),
                         np.ascontiguousarray(col, np.uint32), seed, lo, hi, w)
    return w[:len(col)]


def pick_sources(row_off: np.ndarray, count: int, seed: int = 2):
    """`count` seeded uniform vertices with out-degree >= 1 (repeats allowed)."""
    lib = _load()
    n = len(row_off) - 1
    out = np.empty(max(count, 1), dtype=np.uint32)
    if lib.gen_pick_sources(n, np.ascontiguousarray(row_off, np.uint64), count, seed, out) != 0:
        raise ValueError("graph has no vertex with an out-edge")
    return out[:count]


def batch_scales(count: int = 256, lo: int = 10, hi: int = 16, seed: int = 7):
    """Scales drawn uniformly from [lo, hi] for a many-graph batch."""
    return [lo + int((draw(seed, j) * (hi - lo + 1)) >> 64) for j in range(count)]


def random_graph(n: int, m: int, seed: int):
    """Small uniform test graph (self-loops and duplicates removed, so <= m edges)."""
    lib = _load()
    src = np.empty(max(m, 1), dtype=np.uint32)
    dst = np.empty(max(m, 1), dtype=np.uint32)
    if m:
        lib.gen_uniform_edges(max(n, 1), m, seed, 0, src, dst)
    return csr_from_edges(n, src[:m], dst[:m])


def grid2d(rows: int, cols: int):
    """Directed 4-neighbour grid in both directions (a high-diameter test graph)."""
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    pairs = []
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        pairs.append((a.ravel(), b.ravel()))
        pairs.append((b.ravel(), a.ravel()))
    src = np.concatenate([p[0] for p in pairs]).astype(np.uint32)
    dst = np.concatenate([p[1] for p in pairs]).astype(np.uint32)
    return csr_from_edges(rows * cols, src, dst)

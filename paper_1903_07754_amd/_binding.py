"""ctypes binding of libwedge.so (include/wedge.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels. Device buffers are torch tensors on a ROCm device (PyTorch is used
for device memory and streams only). Importing this module does not touch the
GPU; loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# WEDGE_LIB selects another build of the library (e.g. libwedge_debug.so, with
# device checks compiled in)
LIB_PATH = os.environ.get("WEDGE_LIB") or os.path.join(HERE, "libwedge.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "wedge.h")

OK = 0
STATUS = {0: "WEDGE_OK", -1: "WEDGE_ERR_INVALID_ARG", -2: "WEDGE_ERR_BAD_GRAPH",
          -3: "WEDGE_ERR_NO_WEIGHTS", -4: "WEDGE_ERR_OOM", -5: "WEDGE_ERR_HIP",
          -6: "WEDGE_ERR_UNSUPPORTED", -7: "WEDGE_ERR_MODEL", -8: "WEDGE_ERR_NOT_CONVERGED",
          -9: "WEDGE_ERR_BUSY"}

INPUT_DEVICE, SYMMETRIZE, HOST_ONLY, KEEP_IDS = 0x1, 0x2, 0x4, 0x8
GATE = {"threshold": 0, "wedge": 1, "full": 2, "learned": 3, "push": 4, "hybrid": 5}
RUN_TIME_PULL, RUN_TIME_ITERS, RUN_PERSISTENT, RUN_INPLACE = 0x1, 0x2, 0x4, 0x8
TUNE = {"single": 0, "multisource": 1, "batch": 2}
LAYOUT = {"col_off": 0, "in_src": 1, "in_w": 2, "row_off": 3, "pos": 4, "rowmask": 5,
          "rowseg": 6, "nzdst": 7, "pr_spans": 8, "perm": 9, "xs_src": 10, "xs_w": 11,
          "xs_rowmask": 12, "xs_rowseg": 13, "xs_nzdst": 14, "xs_bounds": 15,
          "xs_pr_span_v": 16, "xs_pr_span_off": 17, "xs_pr_span_tiles": 18}


class WedgeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64), ("nonempty", C.c_uint32),
                ("rows", C.c_uint64), ("flags", C.c_uint32), ("weighted", C.c_uint32),
                ("dangling", C.c_uint32), ("pr_tile_edges", C.c_uint32),
                ("pr_spans", C.c_uint64), ("device_bytes", C.c_uint64),
                ("pr_short_spans", C.c_uint64), ("relabeled", C.c_uint32),
                ("xs_rows", C.c_uint64), ("xs_segments", C.c_uint64),
                ("xs_pr_spans", C.c_uint64), ("xs_pr_short_spans", C.c_uint64),
                ("xs_pr_span_pairs", C.c_uint64), ("xs_packed", C.c_uint32),
                ("xs_slices", C.c_uint32)]


class IterRecord(C.Structure):
    _fields_ = [("iter", C.c_uint32), ("mode", C.c_uint32), ("chunk_edges", C.c_uint32),
                ("reserved", C.c_uint32), ("frontier", C.c_uint64), ("active_edges", C.c_uint64),
                ("marked_chunks", C.c_uint64), ("ms", C.c_float), ("reserved2", C.c_float)]


class TraceSample(C.Structure):
    _fields_ = [("app", C.c_uint32), ("iter", C.c_uint32), ("prev_mode", C.c_uint32),
                ("threshold_mode", C.c_uint32), ("n", C.c_uint64), ("m", C.c_uint64),
                ("frontier", C.c_uint64), ("active", C.c_uint64), ("prev_us", C.c_float),
                ("t_us", C.c_float * 4), ("reserved", C.c_float)]


APP = {"bfs": 1, "cc": 2, "sssp": 3}
MLP_PARAMS = 1476


class Opts(C.Structure):
    _fields_ = [("gate", C.c_uint32), ("threshold_ppm", C.c_uint32), ("chunk_edges", C.c_uint32),
                ("max_iters", C.c_uint32), ("flags", C.c_uint32), ("trace_cap", C.c_uint32),
                ("trace", C.POINTER(IterRecord)), ("model", C.c_void_p),
                ("blocks_per_cu", C.c_uint32), ("rows_per_wave", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_uint32), ("wedge_iters", C.c_uint32),
                ("full_iters", C.c_uint32), ("pull_launches", C.c_uint32),
                ("edges_scanned", C.c_uint64), ("ms", C.c_double), ("pull_ms", C.c_double),
                ("full_pull_ms", C.c_double), ("full_pull_launches", C.c_uint32),
                ("push_iters", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libwedge.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    # the library must share PyTorch's HIP runtime (same streams and allocations):
    # load torch first so that libamdhip64.so.7 resolves to the copy it ships
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
    L.wedge_graph_create_csr.argtypes = [u32, u64, vp, vp, vp, u32, vp, C.POINTER(vp)]
    L.wedge_graph_create_csc.argtypes = [u32, u64, vp, vp, vp, u32, vp, C.POINTER(vp)]
    L.wedge_graph_destroy.argtypes = [vp]
    L.wedge_graph_get_info.argtypes = [vp, C.POINTER(GraphInfo)]
    L.wedge_graph_layout.argtypes = [vp, C.c_int, vp, u64]
    L.wedge_bfs.argtypes = [vp, u32, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_bfs_noalloc.argtypes = [vp, u32, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_cc.argtypes = [vp, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_sssp.argtypes = [vp, u32, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_pagerank.argtypes = [vp, u32, C.c_float, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_frontier_translate.argtypes = [vp, vp, u32, u32, vp, vp, C.POINTER(u64), vp]
    L.wedge_bfs_multisource.argtypes = [vp, vp, u32, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_graph_create_batch_csr.argtypes = [u32, vp, vp, vp, u32, vp, C.POINTER(vp)]
    L.wedge_graph_batch_parts.argtypes = [vp, vp, u32, C.POINTER(u32)]
    L.wedge_bfs_batch.argtypes = [vp, vp, vp, C.POINTER(Opts), vp, C.POINTER(Stats)]
    L.wedge_tune_bfs.argtypes = [vp, u32, vp, u32, vp, vp, C.POINTER(Opts), C.POINTER(C.c_double)]
    L.wedge_tune_lookup.argtypes = [u32, u32, u64, C.POINTER(Opts)]
    L.wedge_model_create.argtypes = [u64, C.POINTER(vp)]
    L.wedge_model_create_ensemble.argtypes = [u64, u32, C.POINTER(vp)]
    L.wedge_model_members.argtypes = [vp, C.POINTER(u32)]
    L.wedge_model_free.argtypes = [vp]
    L.wedge_model_load.argtypes = [C.c_char_p, C.POINTER(vp)]
    L.wedge_model_save.argtypes = [vp, C.c_char_p]
    L.wedge_model_params.argtypes = [vp, vp, u32, C.c_int]
    L.wedge_model_envelope.argtypes = [vp, vp, vp, C.c_int]
    L.wedge_model_margin.argtypes = [vp, C.POINTER(C.c_float), C.c_int]
    L.wedge_model_features.argtypes = [vp, u32, vp]
    L.wedge_model_predict.argtypes = [vp, vp, u32, vp, vp]
    L.wedge_model_grad.argtypes = [vp, vp, vp, vp, u32, vp, vp, vp]
    L.wedge_model_train.argtypes = [vp, vp, u32, u32, C.c_float, vp, C.POINTER(C.c_float)]
    L.wedge_trace_counterfactual.argtypes = [vp, u32, u32, C.POINTER(Opts), vp, u32,
                                             C.POINTER(u32), vp]
    L.wedge_status_string.argtypes = [C.c_int]
    L.wedge_status_string.restype = C.c_char_p
    L.wedge_last_error.restype = C.c_char_p
    L.wedge_version.restype = C.c_char_p
    for name in ("wedge_graph_create_csr", "wedge_graph_create_csc", "wedge_graph_destroy",
                 "wedge_graph_get_info", "wedge_graph_layout", "wedge_bfs", "wedge_bfs_noalloc", "wedge_cc",
                 "wedge_sssp", "wedge_pagerank", "wedge_frontier_translate",
                 "wedge_bfs_multisource", "wedge_graph_create_batch_csr", "wedge_graph_batch_parts",
                 "wedge_bfs_batch", "wedge_tune_bfs", "wedge_tune_lookup", "wedge_model_create",
                 "wedge_model_create_ensemble", "wedge_model_members",
                 "wedge_model_free", "wedge_model_load", "wedge_model_save", "wedge_model_params",
                 "wedge_model_envelope", "wedge_model_margin", "wedge_model_features", "wedge_model_predict",
                 "wedge_model_grad", "wedge_model_train", "wedge_trace_counterfactual"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status):
    if status != OK:
        raise WedgeError(status, lib().wedge_last_error().decode())


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(x):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


class Graph:
    """A graph held by the library (layout on the device unless host_only)."""

    def __init__(self, handle, keep=None):
        self._h = C.c_void_p(handle)
        self._keep = keep
        info = self.info
        self.n, self.m = info["n"], info["m"]

    @property
    def info(self):
        """wedge_graph_info, read afresh (device_bytes grows as workspaces are made)."""
        info = GraphInfo()
        check(lib().wedge_graph_get_info(self._h, C.byref(info)))
        return {k: getattr(info, k) for k, _ in GraphInfo._fields_}

    @staticmethod
    def _make(fn, n, off, ids, w, symmetrize, host_only, stream, keep_ids=False):
        flags = ((SYMMETRIZE if symmetrize else 0) | (HOST_ONLY if host_only else 0)
                 | (KEEP_IDS if keep_ids else 0))
        arrs = [off, ids, w]
        if not all(a is None or isinstance(a, np.ndarray) for a in arrs):
            flags |= INPUT_DEVICE
        else:
            off = np.ascontiguousarray(off, np.uint64)
            ids = np.ascontiguousarray(ids, np.uint32)
            w = None if w is None else np.ascontiguousarray(w, np.uint32)
        m = int(off[-1]) if isinstance(off, np.ndarray) else int(off[-1].item())
        h = C.c_void_p()
        st = fn(n, m, _ptr(off), _ptr(ids) if m else None, _ptr(w), flags,
                None if host_only else _stream_handle(stream), C.byref(h))
        check(st)
        return Graph(h.value)

    @classmethod
    def from_csr(cls, row_off, col, w=None, symmetrize=False, host_only=False, stream=None,
                 keep_ids=False):
        return cls._make(lib().wedge_graph_create_csr, len(row_off) - 1, row_off, col, w,
                         symmetrize, host_only, stream, keep_ids)

    @classmethod
    def from_csc(cls, col_off, src, w=None, symmetrize=False, host_only=False, stream=None,
                 keep_ids=False):
        return cls._make(lib().wedge_graph_create_csc, len(col_off) - 1, col_off, src, w,
                         symmetrize, host_only, stream, keep_ids)

    @classmethod
    def from_batch_csr(cls, parts, host_only=False, stream=None, keep_ids=False):
        """Disjoint union of [(row_off, col), ...] (host arrays, part-local ids)."""
        count = len(parts)
        keep = [(np.ascontiguousarray(r, np.uint64), np.ascontiguousarray(c, np.uint32)) for r, c in parts]
        n_each = np.array([len(r) - 1 for r, _ in keep], np.uint32)
        ros = (C.c_void_p * count)(*[r.ctypes.data for r, _ in keep])
        cols = (C.c_void_p * count)(*[c.ctypes.data if len(c) else None for _, c in keep])
        flags = (HOST_ONLY if host_only else 0) | (KEEP_IDS if keep_ids else 0)
        h = C.c_void_p()
        check(lib().wedge_graph_create_batch_csr(count, n_each.ctypes.data, ros, cols, flags,
                                                 None if host_only else _stream_handle(stream),
                                                 C.byref(h)))
        return Graph(h.value)

    def parts(self):
        cnt = C.c_uint32()
        check(lib().wedge_graph_batch_parts(self._h, None, 0, C.byref(cnt)))
        first = np.zeros(cnt.value + 1, np.uint64)
        check(lib().wedge_graph_batch_parts(self._h, first.ctypes.data, cnt.value + 1, C.byref(cnt)))
        return first

    def layout(self, name):
        dt = np.uint64 if name in ("rowmask", "xs_rowmask") else np.uint32
        info = self.info
        sizes = {"col_off": self.n + 1, "in_src": self.m, "in_w": self.m, "row_off": self.n + 1,
                 "pos": self.m, "rowmask": info["rows"], "rowseg": info["rows"],
                 "nzdst": info["nonempty"], "pr_spans": 3 * info["pr_spans"],
                 "perm": self.n, "xs_src": 64 * info["xs_rows"], "xs_w": 64 * info["xs_rows"],
                 "xs_rowmask": info["xs_rows"], "xs_rowseg": info["xs_rows"],
                 "xs_nzdst": info["xs_segments"], "xs_bounds": 2 * info["xs_slices"] + 1,
                 "xs_pr_span_v": info["xs_pr_spans"],
                 "xs_pr_span_off": info["xs_pr_spans"] + 1 if info["xs_pr_spans"] else 0,
                 "xs_pr_span_tiles": 2 * info["xs_pr_span_pairs"]}
        out = np.zeros(max(int(sizes[name]), 1), dt)
        nbytes = int(sizes[name]) * out.itemsize
        check(lib().wedge_graph_layout(self._h, LAYOUT[name], out.ctypes.data, nbytes))
        return out[:int(sizes[name])]

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().wedge_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(gate="threshold", theta_ppm=0, chunk=0, max_iters=0, time_pull=False,
              time_iters=False, trace_cap=0, model=None, persistent=False, blocks_per_cu=0,
              rows_per_wave=0, inplace=False):
    o = Opts()
    o.gate = GATE[gate] if isinstance(gate, str) else int(gate)
    o.threshold_ppm, o.chunk_edges, o.max_iters = theta_ppm, chunk, max_iters
    o.flags = ((RUN_TIME_PULL if time_pull else 0) | (RUN_TIME_ITERS if time_iters else 0)
               | (RUN_PERSISTENT if persistent else 0) | (RUN_INPLACE if inplace else 0))
    o.blocks_per_cu = blocks_per_cu
    o.rows_per_wave = rows_per_wave
    trace = (IterRecord * trace_cap)() if trace_cap else None
    o.trace_cap = trace_cap
    o.trace = C.cast(trace, C.POINTER(IterRecord)) if trace is not None else None
    o.model = model
    return o, trace


def _trace_list(trace, iters):
    if trace is None:
        return None
    return [{k: getattr(trace[i], k) for k, _ in IterRecord._fields_ if not k.startswith("reserved")}
            for i in range(min(iters, len(trace)))]


def _out_u32(n, out):
    import torch
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    return out


def _run_int(fn, g, args, out, stream, trace_cap, **kw):
    o, trace = make_opts(trace_cap=trace_cap, **kw)
    out = _out_u32(g.n, out)
    st = Stats()
    check(fn(g.handle, *args, _ptr(out), C.byref(o), _stream_handle(stream), C.byref(st)))
    return out[:g.n], st.as_dict(), _trace_list(trace, st.iterations)


def bfs(g, src, out=None, stream=None, trace_cap=0, **kw):
    """Levels (int32 tensor viewed as uint32; 0xFFFFFFFF = unreachable), stats, trace."""
    return _run_int(lib().wedge_bfs, g, (src,), out, stream, trace_cap, **kw)


def bfs_noalloc(g, src, out=None, stream=None, trace_cap=0, **kw):
    """BFS with the library's fixed device scratch as its workspace (no allocation in
    the library; pass `out` to keep the call itself allocation-free)."""
    return _run_int(lib().wedge_bfs_noalloc, g, (src,), out, stream, trace_cap, **kw)


def cc(g, out=None, stream=None, trace_cap=0, **kw):
    return _run_int(lib().wedge_cc, g, (), out, stream, trace_cap, **kw)


def sssp(g, src, out=None, stream=None, trace_cap=0, **kw):
    return _run_int(lib().wedge_sssp, g, (src,), out, stream, trace_cap, **kw)


def pagerank(g, iters=20, damping=0.85, out=None, stream=None, time_pull=False, rows_per_wave=0,
             **kw):
    import torch
    o, _ = make_opts(time_pull=time_pull, rows_per_wave=rows_per_wave, **kw)
    if out is None:
        out = torch.empty(max(g.n, 1), dtype=torch.float32, device="cuda")
    st = Stats()
    check(lib().wedge_pagerank(g.handle, iters, damping, _ptr(out), C.byref(o),
                               _stream_handle(stream), C.byref(st)))
    return out[:g.n], st.as_dict()


def bfs_multisource(g, srcs, out=None, stream=None, trace_cap=0, **kw):
    """Levels [len(srcs), n] (int32 tensor viewed as uint32), stats, trace."""
    import torch
    srcs = np.ascontiguousarray(srcs, np.uint32)
    k = len(srcs)
    if out is None:
        out = torch.empty(max(k * g.n, 1), dtype=torch.int32, device="cuda")
    o, trace = make_opts(trace_cap=trace_cap, **kw)
    st = Stats()
    check(lib().wedge_bfs_multisource(g.handle, srcs.ctypes.data, k, _ptr(out), C.byref(o),
                                      _stream_handle(stream), C.byref(st)))
    return out[:k * g.n].view(k, g.n), st.as_dict(), _trace_list(trace, st.iterations)


def bfs_batch(g, srcs, out=None, stream=None, trace_cap=0, **kw):
    """Union-order levels of one BFS per part (srcs: part-local sources)."""
    srcs = np.ascontiguousarray(srcs, np.uint32)
    o, trace = make_opts(trace_cap=trace_cap, **kw)
    out = _out_u32(g.n, out)
    st = Stats()
    check(lib().wedge_bfs_batch(g.handle, srcs.ctypes.data, _ptr(out), C.byref(o),
                                _stream_handle(stream), C.byref(st)))
    return out[:g.n], st.as_dict(), _trace_list(trace, st.iterations)


def tune_bfs(g, kind, srcs, out, stream=None, gate="threshold", theta_ppm=0):
    """Autotune a BFS kind; returns (best options dict, best ms)."""
    srcs = np.ascontiguousarray(srcs, np.uint32)
    o, _ = make_opts(gate=gate, theta_ppm=theta_ppm)
    ms = C.c_double()
    check(lib().wedge_tune_bfs(g.handle, TUNE[kind], srcs.ctypes.data, len(srcs), _ptr(out),
                               _stream_handle(stream), C.byref(o), C.byref(ms)))
    best = {"chunk": o.chunk_edges, "persistent": bool(o.flags & RUN_PERSISTENT),
            "blocks_per_cu": o.blocks_per_cu, "rows_per_wave": o.rows_per_wave, "gate": o.gate,
            "theta_ppm": o.threshold_ppm}
    return best, ms.value


def tune_lookup(kind, count, m):
    o, _ = make_opts()
    st = lib().wedge_tune_lookup(TUNE[kind], count, m, C.byref(o))
    if st != OK:
        return None
    return {"chunk": o.chunk_edges, "persistent": bool(o.flags & RUN_PERSISTENT),
            "blocks_per_cu": o.blocks_per_cu, "rows_per_wave": o.rows_per_wave}


def frontier_translate(g, frontier, chunk, stream=None):
    """(Wedge bitmap as uint64 tensor, marked chunk ids tensor[:K]) for a device frontier."""
    import torch
    nchunks = (g.m + chunk - 1) // chunk
    words = (nchunks + 63) // 64
    wbits = torch.zeros(max(words, 1), dtype=torch.int64, device="cuda")
    lst = torch.zeros(max(nchunks, 1), dtype=torch.int32, device="cuda")
    marked = C.c_uint64()
    check(lib().wedge_frontier_translate(g.handle, _ptr(frontier), int(frontier.numel()), chunk,
                                         _ptr(wbits), _ptr(lst), C.byref(marked),
                                         _stream_handle(stream)))
    return wbits[:words], lst[:marked.value]


class Model:
    """Learned-gate model (FP32 MLP 8 -> 32 -> 32 -> 4) held by the library."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    @classmethod
    def create(cls, seed=0, members=1):
        """New model; members > 1 gives an ensemble whose prediction is the mean."""
        h = C.c_void_p()
        if members == 1:
            check(lib().wedge_model_create(seed, C.byref(h)))
        else:
            check(lib().wedge_model_create_ensemble(seed, members, C.byref(h)))
        return cls(h.value)

    @property
    def members(self):
        n = C.c_uint32()
        check(lib().wedge_model_members(self._h, C.byref(n)))
        return n.value

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        check(lib().wedge_model_load(os.fsencode(path), C.byref(h)))
        return cls(h.value)

    def save(self, path):
        check(lib().wedge_model_save(self._h, os.fsencode(path)))

    @property
    def handle(self):
        return self._h

    def params(self, new=None):
        """All members' parameters, members one after another (1476 each)."""
        count = MLP_PARAMS * self.members
        p = np.zeros(count, np.float32)
        if new is not None:
            p[:] = np.asarray(new, np.float32).ravel()
            check(lib().wedge_model_params(self._h, p.ctypes.data, count, 1))
        else:
            check(lib().wedge_model_params(self._h, p.ctypes.data, count, 0))
        return p

    def envelope(self, lo=None, hi=None):
        a = np.zeros(8, np.float32)
        b = np.zeros(8, np.float32)
        if lo is not None:
            a[:] = lo
            b[:] = hi
            check(lib().wedge_model_envelope(self._h, a.ctypes.data, b.ctypes.data, 1))
        else:
            check(lib().wedge_model_envelope(self._h, a.ctypes.data, b.ctypes.data, 0))
        return a, b

    def margin(self, value=None):
        """The decision margin over the threshold rule (set it when value is given)."""
        v = C.c_float(0.0 if value is None else value)
        check(lib().wedge_model_margin(self._h, C.byref(v), 0 if value is None else 1))
        return v.value

    def predict(self, x, stream=None):
        x = np.ascontiguousarray(x, np.float32)
        y = np.zeros((len(x), 4), np.float32)
        check(lib().wedge_model_predict(self._h, x.ctypes.data, len(x), y.ctypes.data,
                                        _stream_handle(stream)))
        return y

    def grad(self, x, t, mask, stream=None):
        x = np.ascontiguousarray(x, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        mask = np.ascontiguousarray(mask, np.float32)
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = C.c_float()
        check(lib().wedge_model_grad(self._h, x.ctypes.data, t.ctypes.data, mask.ctypes.data,
                                     len(x), g.ctypes.data, C.byref(loss),
                                     _stream_handle(stream)))
        return g, loss.value

    def train(self, samples, epochs=2000, lr=1e-3, stream=None):
        loss = C.c_float()
        check(lib().wedge_model_train(self._h, samples, len(samples), epochs, lr,
                                      _stream_handle(stream), C.byref(loss)))
        return loss.value

    def close(self):
        if self._h is not None and self._h.value:
            lib().wedge_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(samples):
    """Gate features (host formula) of a TraceSample array: float32 [count, 8]."""
    x = np.zeros((len(samples), 8), np.float32)
    if len(samples):
        check(lib().wedge_model_features(samples, len(samples), x.ctypes.data))
    return x


def trace_counterfactual(g, app, src=0, cap=4096, stream=None, theta_ppm=0, chunk=0):
    """Per-iteration times of all four modes from each iteration's state (TraceSample array)."""
    o, _ = make_opts(theta_ppm=theta_ppm, chunk=chunk)
    out = (TraceSample * cap)()
    cnt = C.c_uint32()
    check(lib().wedge_trace_counterfactual(g.handle, APP[app], src, C.byref(o), out, cap,
                                           C.byref(cnt), _stream_handle(stream)))
    res = (TraceSample * cnt.value)()
    C.memmove(res, out, C.sizeof(TraceSample) * cnt.value)
    return res


def samples_to_dicts(samples):
    return [{"app": s.app, "iter": s.iter, "prev_mode": s.prev_mode,
             "threshold_mode": s.threshold_mode, "n": s.n, "m": s.m, "frontier": s.frontier,
             "active": s.active, "prev_us": s.prev_us, "t_us": list(s.t_us)} for s in samples]


def u32(t):
    """Host numpy uint32 view of an int32 device tensor."""
    return t.cpu().numpy().view(np.uint32)


def header_functions():
    """Names of the functions include/wedge.h declares."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:wedge_status|const char\*)\s+(wedge_\w+)\s*\(", txt, re.M)))

"""CPU-side checks of the C-ABI library: it loads without a GPU, exports every
function include/wedge.h declares, builds the layout on the host exactly as the
method defines it, and rejects malformed input before any device work."""
import ctypes as C

import numpy as np
import pytest

import gen
import oracle
import paper_1903_07754_amd as W
from paper_1903_07754_amd import _binding as B
from helpers import relabel


def test_library_exports_every_header_function():
    names = W.header_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(W.lib(), n), n
    assert W.lib().wedge_version() == b"0.1.0"
    assert W.lib().wedge_status_string(-4) == b"out of memory"


def host_graph(ro, col, w=None, symmetrize=False, keep_ids=True):
    return W.Graph.from_csr(ro, col, w, symmetrize=symmetrize, host_only=True, keep_ids=keep_ids)


@pytest.mark.parametrize("seed,scale", [(1, 9), (2, 11)])
def test_relabelled_layout_is_degree_order(seed, scale):
    """Default layout: internal id = rank by decreasing out-degree (ties by id), and
    every array is the canonical layout of the renamed graph."""
    ro, col = gen.rmat(scale, 16, seed=seed)
    w = gen.edge_weights(ro, col, seed=seed)
    g = host_graph(ro, col, w, keep_ids=False)
    assert g.info["relabeled"] == 1
    perm = g.layout("perm")
    n = len(ro) - 1
    deg = np.diff(ro.astype(np.int64))
    want_inv = np.lexsort((np.arange(n), -deg))
    np.testing.assert_array_equal(np.argsort(perm), want_inv)
    rro, rcol, rw = relabel(ro, col, perm, w)
    ref = host_graph(rro, rcol, rw, keep_ids=True)
    for name in ("col_off", "in_src", "in_w", "row_off", "pos", "rowmask", "rowseg", "nzdst",
                 "pr_spans"):
        np.testing.assert_array_equal(g.layout(name), ref.layout(name))


@pytest.mark.parametrize("seed,scale", [(1, 8), (2, 10), (3, 12)])
def test_layout_matches_oracle_csc_and_edge_index(seed, scale):
    ro, col = gen.rmat(scale, 16, seed=seed)
    w = gen.edge_weights(ro, col, seed=seed)
    g = host_graph(ro, col, w)
    n, m = len(ro) - 1, len(col)
    co, src, iw = oracle.csc(ro, col, w)
    np.testing.assert_array_equal(g.layout("col_off"), co.astype(np.uint32))
    np.testing.assert_array_equal(g.layout("in_src"), src)
    np.testing.assert_array_equal(g.layout("in_w"), iw)
    np.testing.assert_array_equal(g.layout("row_off"), ro.astype(np.uint32))
    # edge index: CSR edge q = (u -> v) sits at in-edge position pos[q]
    pos = g.layout("pos").astype(np.int64)
    assert np.array_equal(np.sort(pos), np.arange(m))             # a permutation
    u = np.repeat(np.arange(n), np.diff(ro.astype(np.int64)))
    assert np.array_equal(src[pos], u)                             # same source
    assert np.all(co[col] <= pos) and np.all(pos < co[col.astype(np.int64) + 1])  # same destination
    # one vertex's entries ascend (out-neighbours ascend)
    same = u[1:] == u[:-1]
    assert np.all(np.diff(pos)[same] > 0)


@pytest.mark.parametrize("seed,scale", [(4, 9), (5, 11)])
def test_row_layout_names_every_position_destination(seed, scale):
    ro, col = gen.rmat(scale, 8, seed=seed)
    g = host_graph(ro, col)
    n, m = len(ro) - 1, len(col)
    co, src, _ = oracle.csc(ro, col)
    dst_of_pos = np.repeat(np.arange(n), np.diff(co.astype(np.int64)))
    mask = g.layout("rowmask")
    seg = g.layout("rowseg").astype(np.int64)
    nz = g.layout("nzdst")
    assert np.array_equal(nz, np.flatnonzero(np.diff(co.astype(np.int64)) > 0))
    p = np.arange(m)
    r, b = p >> 6, p & 63
    bits = (mask[r] >> b.astype(np.uint64)) & np.uint64(1)
    starts = np.zeros(m, bool)
    starts[co[nz].astype(np.int64)] = True
    assert np.array_equal(bits.astype(bool), starts)
    # destination = nz[seg[row] + number of segment starts in (row start, p]]
    cum = np.cumsum(starts)
    row_first = r * 64
    got = nz[seg[r] + (cum - cum[row_first])]
    assert np.array_equal(got, dst_of_pos)
    assert g.info["rows"] == (m + 63) // 64
    assert g.info["dangling"] == int((np.diff(ro.astype(np.int64)) == 0).sum())


def test_pagerank_tile_spans():
    ro, col = gen.rmat(12, 16, seed=9)
    g = host_graph(ro, col)
    co, _, _ = oracle.csc(ro, col)
    T = g.info["pr_tile_edges"]
    sp = g.layout("pr_spans").reshape(-1, 3).astype(np.int64)
    short, long_ = [], []
    for v in range(len(ro) - 1):
        a, b = int(co[v]), int(co[v + 1]) - 1
        if b >= a and a // T != b // T:
            (short if b // T - a // T <= 8 else long_).append((v, a // T, b // T))
    assert [tuple(x) for x in sp] == short + long_
    assert g.info["pr_short_spans"] == len(short)


def test_symmetrized_layout_is_oracle_undirected_view():
    ro, col = gen.random_graph(300, 1500, 3)
    g = host_graph(ro, col, symmetrize=True)
    sro, scol = oracle.symmetrize(ro, col)
    assert g.m == len(scol)
    np.testing.assert_array_equal(g.layout("row_off"), sro.astype(np.uint32))
    co, src, _ = oracle.csc(sro, scol)
    np.testing.assert_array_equal(g.layout("in_src"), src)


def test_from_csc_equals_from_csr():
    ro, col = gen.rmat(9, 16, seed=7)
    w = gen.edge_weights(ro, col, seed=3)
    co, src, iw = oracle.csc(ro, col, w)
    a = host_graph(ro, col, w, keep_ids=False)
    b = W.Graph.from_csc(co, src, iw, host_only=True)
    for name in ("col_off", "in_src", "in_w", "row_off", "pos", "rowmask", "rowseg", "nzdst",
                 "perm"):
        np.testing.assert_array_equal(a.layout(name), b.layout(name))


def test_degenerate_graphs_build():
    for ro, col in [(np.zeros(1, np.uint64), np.zeros(0, np.uint32)),          # n = 0
                    (np.zeros(2, np.uint64), np.zeros(0, np.uint32)),          # one vertex
                    (np.array([0, 1], np.uint64), np.array([0], np.uint32))]:  # self-loop only
        g = host_graph(ro, col)
        assert g.n == len(ro) - 1 and g.m == len(col)


def status_of(fn):
    with pytest.raises(W.WedgeError) as e:
        fn()
    return e.value.name


def test_malformed_input_is_rejected():
    ro, col = gen.random_graph(20, 60, 1)
    bad = ro.copy(); bad[3] = bad[4] + 1
    assert status_of(lambda: host_graph(bad, col)) == "WEDGE_ERR_BAD_GRAPH"
    bad = ro.copy(); bad[0] = 1
    assert status_of(lambda: host_graph(bad, col)) == "WEDGE_ERR_BAD_GRAPH"
    bad = col.copy(); bad[5] = 20
    assert status_of(lambda: host_graph(ro, bad)) == "WEDGE_ERR_BAD_GRAPH"
    w = gen.edge_weights(ro, col)
    assert status_of(lambda: host_graph(ro, col, w, symmetrize=True)) == "WEDGE_ERR_INVALID_ARG"
    L = W.lib()
    h = C.c_void_p()
    # m >= 2^32, null pointers, unknown flags, host-only with device input
    assert L.wedge_graph_create_csr(4, 1 << 32, ro.ctypes.data, col.ctypes.data, None,
                                    B.HOST_ONLY, None, C.byref(h)) == -2
    assert L.wedge_graph_create_csr(4, 0, None, None, None, B.HOST_ONLY, None, C.byref(h)) == -1
    assert L.wedge_graph_create_csr(20, len(col), ro.ctypes.data, None, None, B.HOST_ONLY, None,
                                    C.byref(h)) == -1
    assert L.wedge_graph_create_csr(20, len(col), ro.ctypes.data, col.ctypes.data, None, 0x80,
                                    None, C.byref(h)) == -1
    assert L.wedge_graph_create_csr(20, len(col), ro.ctypes.data, col.ctypes.data, None,
                                    B.HOST_ONLY | B.INPUT_DEVICE, None, C.byref(h)) == -1
    assert L.wedge_graph_create_csr(1 << 31, 0, ro.ctypes.data, None, None, B.HOST_ONLY, None,
                                    C.byref(h)) == -2
    assert h.value is None
    assert L.wedge_last_error()


def test_runs_on_host_only_graph_are_refused():
    ro, col = gen.random_graph(10, 30, 2)
    g = host_graph(ro, col)
    L = W.lib()
    st = B.Stats()
    o, _ = B.make_opts()
    out = np.zeros(10, np.uint32)
    assert L.wedge_bfs(g.handle, 0, out.ctypes.data, C.byref(o), None, C.byref(st)) == -6
    assert L.wedge_pagerank(g.handle, 20, 0.85, out.ctypes.data, C.byref(o), None, C.byref(st)) == -6
    assert L.wedge_graph_layout(g.handle, B.LAYOUT["pos"], out.ctypes.data, 3) == -1
    assert L.wedge_graph_layout(g.handle, 99, out.ctypes.data, 4) == -1
    assert L.wedge_graph_destroy(None) == 0


def test_batch_union_is_the_concatenation():
    parts = [gen.rmat(s, 16, seed=70 + s) for s in (3, 6, 5, 2)]
    g = W.Graph.from_batch_csr(parts, host_only=True, keep_ids=True)
    first = g.parts()
    assert list(first) == list(np.cumsum([0] + [len(r) - 1 for r, _ in parts]))
    ro = np.concatenate([[0]] + [r[1:] + sum(int(p[0][-1]) for p in parts[:i])
                                 for i, (r, _) in enumerate(parts)]).astype(np.uint64)
    col = np.concatenate([c + first[i] for i, (_, c) in enumerate(parts)]).astype(np.uint32)
    co, src, _ = oracle.csc(ro, col)
    np.testing.assert_array_equal(g.layout("row_off"), ro.astype(np.uint32))
    np.testing.assert_array_equal(g.layout("in_src"), src)
    with pytest.raises(W.WedgeError):
        bad = [(parts[0][0], parts[0][1] + 100)]
        W.Graph.from_batch_csr(bad, host_only=True)


def _slice_of(u, S):
    """Source slice of internal id u: 1024-id groups dealt to S slices in snake order."""
    g = u.astype(np.int64) >> 10
    return np.where((g // S) & 1, S - 1 - (g % S), g % S)


@pytest.mark.parametrize("seed,scale,weighted,sym,keep,slices", [
    (6, 12, True, False, True, 8), (7, 13, False, True, False, 8), (8, 14, True, False, False, 8),
    (9, 12, "heavy", False, False, 8), (10, 13, True, False, False, 16), (11, 14, False, True, False, 32),
    (12, 13, "heavy", False, True, 64)])
def test_source_sliced_copy(monkeypatch, seed, scale, weighted, sym, keep, slices):
    """The source-sliced in-edge copy holds every in-edge once, in the slice of
    its source, each slice grouped by destination with sources ascending (the
    canonical order restricted to the slice), starting on a row boundary; its
    row layout names every real position's destination."""
    monkeypatch.setenv("WEDGE_SLICED_PULL", "1")
    monkeypatch.setenv("WEDGE_XS_SLICES", str(slices))
    ro, col = gen.rmat(scale, 16, seed=seed)
    w = None
    if weighted:
        # weights up to 255 are packed with the slice-local source; heavier not
        w = gen.edge_weights(ro, col, seed=seed, hi=100_000 if weighted == "heavy" else 255)
    g = host_graph(ro, col, w, symmetrize=sym, keep_ids=keep)
    info = g.info
    assert info["xs_rows"] > 0
    assert info["xs_packed"] == (weighted is True)
    S = slices
    assert info["xs_slices"] == S
    co = g.layout("col_off").astype(np.int64)
    src = g.layout("in_src")
    n, m = len(co) - 1, len(src)
    dst_c = np.repeat(np.arange(n), np.diff(co))
    b = g.layout("xs_bounds").astype(np.int64)
    assert len(b) == 2 * S + 1
    row_begin, edge_end = b[:S + 1], b[S + 1:]
    assert row_begin[0] == 0 and np.all(np.diff(row_begin) >= 0)
    assert row_begin[S] == info["xs_rows"]
    assert np.all(edge_end <= row_begin[1:] * 64) and np.all(edge_end >= row_begin[:S] * 64)
    xsrc = g.layout("xs_src")
    xw = None
    if weighted and info["xs_packed"]:
        # one word per position: (slice-local source << 8) | weight
        xw = xsrc & np.uint32(255)
        loc = (xsrc >> np.uint32(8)).astype(np.int64)
        b_ = loc >> 10
        xsrc = np.zeros(len(loc), np.uint32)
        for j in range(S):
            lo, hi = row_begin[j] * 64, row_begin[j + 1] * 64
            gidx = b_[lo:hi] * S + np.where(b_[lo:hi] & 1, S - 1 - j, j)
            xsrc[lo:hi] = ((gidx << 10) | (loc[lo:hi] & 1023)).astype(np.uint32)
        with pytest.raises(W.WedgeError):
            g.layout("xs_w")
    elif weighted:
        assert not info["xs_packed"]
        xw = g.layout("xs_w")
    else:
        assert not info["xs_packed"]
    mask = g.layout("xs_rowmask")
    seg = g.layout("xs_rowseg").astype(np.int64)
    nz = g.layout("xs_nzdst").astype(np.int64)
    sl = _slice_of(src, S)
    P = 64 * info["xs_rows"]
    p = np.arange(P)
    r, bb = p >> 6, p & 63
    bits = ((mask[r] >> bb.astype(np.uint64)) & np.uint64(1)).astype(bool)
    cum = np.cumsum(bits)
    dst_x = nz[seg[r] + (cum - cum[r * 64])]  # the row-layout destination of every position
    total = 0
    for j in range(S):
        lo, hi = row_begin[j] * 64, edge_end[j]
        want = np.flatnonzero(sl == j)                      # canonical order, slice j only
        assert hi - lo == len(want), j
        np.testing.assert_array_equal(xsrc[lo:hi], src[want])
        np.testing.assert_array_equal(dst_x[lo:hi], dst_c[want])
        if weighted:
            np.testing.assert_array_equal(xw[lo:hi], g.layout("in_w")[want])
        if hi > lo:
            assert bits[lo]                                 # a slice starts a segment
        # segment starts inside the slice are exactly the destination changes
        d = dst_c[want]
        starts = np.ones(len(d), bool)
        starts[1:] = d[1:] != d[:-1]
        np.testing.assert_array_equal(bits[lo:hi], starts)
        assert not bits[hi:row_begin[j + 1] * 64].any()     # padding starts nothing
        total += hi - lo
    assert total == m
    assert info["xs_segments"] == int(bits.sum())
    # PageRank tiles (8 rows) never straddle two slices
    T = info["pr_tile_edges"]
    assert np.all(row_begin * 64 % T == 0)
    # fix-up lists: every slice segment whose positions cross a tile boundary,
    # grouped by destination in slice order; destinations whose segments cover
    # at most 8 extra tiles in all come first
    per_v = {}
    for j in range(S):
        lo, hi = int(row_begin[j] * 64), int(edge_end[j])
        if hi == lo:
            continue
        d = dst_x[lo:hi]
        cut = np.flatnonzero(np.diff(d)) + 1
        for a, b in zip(np.r_[0, cut] + lo, np.r_[cut, hi - lo] + lo - 1):
            if a // T != b // T:
                per_v.setdefault(int(dst_x[a]), []).append((a // T, b // T))
    order = sorted(per_v)
    short = [v for v in order if sum(b - a for a, b in per_v[v]) <= 8]
    long_ = [v for v in order if sum(b - a for a, b in per_v[v]) > 8]
    assert info["xs_pr_spans"] == len(order)
    assert info["xs_pr_short_spans"] == len(short)
    np.testing.assert_array_equal(g.layout("xs_pr_span_v"), np.array(short + long_, np.uint32))
    off = g.layout("xs_pr_span_off").astype(np.int64)
    tiles = g.layout("xs_pr_span_tiles").reshape(-1, 2).astype(np.int64)
    for k, v in enumerate(short + long_):
        assert [tuple(x) for x in tiles[off[k]:off[k + 1]]] == per_v[v]
    assert (len(off) == 0 and len(tiles) == 0) or off[-1] == len(tiles)


def test_source_sliced_copy_threshold(monkeypatch):
    ro, col = gen.rmat(10, 8, seed=3)
    monkeypatch.delenv("WEDGE_SLICED_PULL", raising=False)
    assert host_graph(ro, col).info["xs_rows"] == 0        # small graphs: not built
    monkeypatch.setenv("WEDGE_SLICED_PULL", "0")
    assert host_graph(ro, col).info["xs_rows"] == 0
    monkeypatch.setenv("WEDGE_SLICED_PULL", "1")
    assert host_graph(ro, col).info["xs_rows"] > 0
    # few sources: the fewest slices (the count grows with the sources' values)
    assert host_graph(ro, col).info["xs_slices"] == 8
    monkeypatch.setenv("WEDGE_XS_SLICES", "32")
    assert host_graph(ro, col).info["xs_slices"] == 32
    monkeypatch.setenv("WEDGE_XS_SLICES", "12")  # not a power of two: the default
    assert host_graph(ro, col).info["xs_slices"] == 8

"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer results (BFS levels, CC labels, SSSP distances) must be bit-exact, and
so must every per-iteration record (frontier size, out-degree sum A, gate
decision, marked chunks). PageRank (FP32) must be within 1e-5 relative L1 of
the FP64 oracle. Sizes span many wave tiles and end in ragged tails.
"""
import numpy as np
import pytest

import gen
import oracle
from helpers import relabel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1903_07754_amd as W  # noqa: E402

THETA = {"bfs": 10_000, "cc": 200_000, "sssp": 200_000}
CHUNK = {"bfs": 32, "cc": 16, "sssp": 16}


def run_app(app, g, src, **kw):
    print(f"  [{app} n={g.n} m={g.m} src={src} {kw}]", flush=True)
    if app == "bfs":
        out, st, tr = W.bfs(g, src, trace_cap=g.n + 2, **kw)
    elif app == "cc":
        out, st, tr = W.cc(g, trace_cap=g.n + 2, **kw)
    else:
        out, st, tr = W.sssp(g, src, trace_cap=g.n + 2, **kw)
    torch.cuda.synchronize()
    return W.u32(out), st, tr


def internal_marked(g, gro, gcol, frontiers, chunk):
    """Wedge Frontier sizes of the oracle's frontiers, on the library's internal
    vertex order (the canonical in-edge array of the renamed graph)."""
    n = len(gro) - 1
    perm = g.layout("perm") if g.info["relabeled"] else np.arange(n, dtype=np.uint32)
    rro, rcol, _ = relabel(gro, gcol, perm)
    _, isrc, _ = oracle.csc(rro, rcol)
    out = []
    for fr in frontiers:
        fi = np.empty(n, np.uint8)
        fi[perm] = fr
        out.append(oracle.wedge_frontier(isrc, fi, chunk)[1])
    return out


def check_trace(tr, ref, chunk, K):
    assert len(tr) == ref.iters
    for k, r in enumerate(tr):
        assert r["frontier"] == ref.F[k], k
        assert r["active_edges"] == ref.A[k], k
        if r["mode"] == 1:
            assert r["chunk_edges"] == chunk
            assert r["marked_chunks"] == K[k], k


def parity(app, ro, col, w=None, src=0, gate="threshold", theta=None, chunk=None, keep_ids=False):
    theta = THETA[app] if theta is None else theta
    chunk = CHUNK[app] if chunk is None else chunk
    if app == "cc":
        gro, gcol = oracle.symmetrize(ro, col)
        g = W.Graph.from_csr(ro, col, symmetrize=True, keep_ids=keep_ids)
        ref = oracle.pull_engine("cc", gro, gcol, theta_ppm=theta, chunk=chunk, keep_frontiers=True)
        want = oracle.cc(ro, col)
    else:
        gro, gcol = ro, col
        g = W.Graph.from_csr(ro, col, w, keep_ids=keep_ids)
        ref = oracle.pull_engine(app, ro, col, w, src, theta_ppm=theta, chunk=chunk,
                                 keep_frontiers=True)
        want = oracle.bfs(ro, col, src) if app == "bfs" else oracle.sssp(ro, col, w, src)
    K = internal_marked(g, gro, gcol, ref.frontiers, chunk)
    if keep_ids:
        np.testing.assert_array_equal(K, ref.K)
    np.testing.assert_array_equal(ref.values, want)
    got, st, tr = run_app(app, g, src, gate=gate, theta_ppm=theta, chunk=chunk)
    np.testing.assert_array_equal(got, want)
    assert st["iterations"] == ref.iters
    check_trace(tr, ref, chunk, K)
    if gate == "threshold":
        assert [r["mode"] for r in tr] == list(ref.mode)
    elif gate == "wedge":
        assert all(r["mode"] == 1 for r in tr)
    else:
        assert all(r["mode"] == 0 for r in tr)
    g.close()
    return tr


GRAPHS = {
    "er_small": lambda: gen.random_graph(1000, 6000, 11),
    "er_ragged": lambda: gen.random_graph(4099, 37001, 12),
    "rmat12": lambda: gen.rmat(12, 16, seed=13),
    "rmat14": lambda: gen.rmat(14, 16, seed=14),
    "grid": lambda: gen.grid2d(37, 53),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("app", ["bfs", "cc", "sssp"])
def test_parity_threshold_gate(app, name):
    ro, col = GRAPHS[name]()
    w = gen.edge_weights(ro, col, seed=4) if app == "sssp" else None
    srcs = gen.pick_sources(ro, 2, seed=5) if app != "cc" else [0]
    for s in srcs:
        parity(app, ro, col, w, int(s))
        parity(app, ro, col, w, int(s), keep_ids=True)


@pytest.mark.parametrize("gate", ["wedge", "full"])
@pytest.mark.parametrize("chunk", [1, 4, 16, 32, 64, 128, 1024])
@pytest.mark.parametrize("app", ["bfs", "cc", "sssp"])
def test_mode_and_granularity_invariance(app, chunk, gate):
    """Any chunk size and either forced mode gives the same values and the same
    per-iteration frontiers (Frontier Transformation, Frontier Precision)."""
    ro, col = gen.rmat(11, 16, seed=21)
    w = gen.edge_weights(ro, col, seed=6) if app == "sssp" else None
    s = int(gen.pick_sources(ro, 1, seed=7)[0])
    parity(app, ro, col, w, s, gate=gate, chunk=chunk)


@pytest.mark.parametrize("slices", ["8", "64"])
@pytest.mark.parametrize("name", ["er_ragged", "rmat14", "grid", "rmat14_heavy"])
@pytest.mark.parametrize("gate", ["threshold", "full"])
@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_parity_source_sliced_full_pull(monkeypatch, app, gate, name, slices):
    """CC and SSSP with the full pulls over the source-sliced copy (forced on
    small graphs): values and every per-iteration record equal the oracle, as
    with the canonical pull, in the synchronous and the in-place forms. SSSP
    weights up to 255 run on the packed copy (one word per in-edge), heavier
    ones on separate source and weight arrays."""
    monkeypatch.setenv("WEDGE_SLICED_PULL", "1")
    monkeypatch.setenv("WEDGE_XS_SLICES", slices)  # 64: most slices of these graphs are empty
    heavy = name.endswith("_heavy")
    ro, col = GRAPHS[name.replace("_heavy", "")]()
    w = gen.edge_weights(ro, col, seed=4, hi=100_000 if heavy else 255) if app == "sssp" else None
    src = int(gen.pick_sources(ro, 1, seed=6)[0]) if app != "cc" else 0
    tr = parity(app, ro, col, w, src, gate=gate)
    assert tr is not None
    g = (W.Graph.from_csr(ro, col, symmetrize=True) if app == "cc" else W.Graph.from_csr(ro, col, w))
    assert g.info["xs_rows"] > 0
    assert g.info["xs_packed"] == (app == "sssp" and not heavy)
    assert g.info["xs_slices"] == int(slices)
    want = oracle.cc(ro, col) if app == "cc" else oracle.sssp(ro, col, w, src)
    out, _, _ = run_app(app, g, src, gate=gate, inplace=True)
    np.testing.assert_array_equal(out, want)
    g.close()


@pytest.mark.parametrize("gate", ["threshold", "wedge", "full"])
@pytest.mark.parametrize("app", ["bfs", "sssp", "cc"])
def test_per_iteration_frontier_sets(app, gate):
    """The frontier of every iteration as a set, not only its size: a run cut
    off after k iterations (max_iters = k) leaves the values of iteration k in
    the caller's buffer, and the vertices whose value changed in iteration k-1
    must be exactly the oracle's frontier F_k (Background, Push vs. Pull: a
    vertex is active when its value was updated). After a full pull the next
    frontier is taken from the values, after a chunk pull from the bits the
    pull set: both must give F_k."""
    check_frontier_sets(app, gate)


@pytest.mark.parametrize("gate", ["threshold", "full"])
@pytest.mark.parametrize("app", ["sssp", "cc"])
def test_per_iteration_frontier_sets_sliced(monkeypatch, app, gate):
    """The same with the CC/SSSP full pulls over the source-sliced copy
    (forced on this small graph), one launch per slice before the frontier is
    taken from the values."""
    monkeypatch.setenv("WEDGE_SLICED_PULL", "1")
    check_frontier_sets(app, gate, sliced=True)


def check_frontier_sets(app, gate, sliced=False):
    ro, col = gen.rmat(12, 16, seed=13)
    n = len(ro) - 1
    w = gen.edge_weights(ro, col, seed=6) if app == "sssp" else None
    src = int(gen.pick_sources(ro, 1, seed=7)[0])
    if app == "cc":
        gro, gcol = oracle.symmetrize(ro, col)
        g = W.Graph.from_csr(ro, col, symmetrize=True, keep_ids=True)
        ref = oracle.pull_engine("cc", gro, gcol, keep_frontiers=True)
        prev = np.arange(n, dtype=np.uint32)
    else:
        g = W.Graph.from_csr(ro, col, w, keep_ids=True)
        ref = oracle.pull_engine(app, ro, col, w, src, keep_frontiers=True)
        prev = np.full(n, 0xFFFFFFFF, np.uint32)
        prev[src] = 0
    assert (g.info["xs_rows"] > 0) == sliced
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    run = {"bfs": lambda k: W.bfs(g, src, out=out, gate=gate, max_iters=k),
           "sssp": lambda k: W.sssp(g, src, out=out, gate=gate, max_iters=k),
           "cc": lambda k: W.cc(g, out=out, gate=gate, max_iters=k)}[app]
    print(f"  [{app} gate={gate} iterations={ref.iters}]", flush=True)
    for k in range(1, ref.iters + 1):
        try:
            run(k)
            converged = True
        except W.WedgeError as e:
            assert e.name == "WEDGE_ERR_NOT_CONVERGED"
            converged = False
        torch.cuda.synchronize()
        cur = W.u32(out).copy()
        changed = cur != prev
        if k < ref.iters:
            assert not converged, k
            np.testing.assert_array_equal(changed, ref.frontiers[k].astype(bool), err_msg=f"F_{k}")
        else:
            assert converged and not changed.any()
            np.testing.assert_array_equal(cur, ref.values)
        prev = cur
    g.close()


def test_theta_extremes():
    ro, col = gen.rmat(12, 8, seed=31)
    w = gen.edge_weights(ro, col, seed=8)
    s = int(gen.pick_sources(ro, 1, seed=9)[0])
    for theta in (1, 50_000, 480_000, 1_000_000):
        parity("sssp", ro, col, w, s, theta=theta)


def test_wedge_frontier_bitmap_is_the_definition():
    """The translated bitmap equals the full-scan definition bit for bit."""
    ro, col = gen.rmat(13, 16, seed=41)
    g = W.Graph.from_csr(ro, col, keep_ids=True)
    co, src, _ = oracle.csc(ro, col)
    n = len(ro) - 1
    rng = np.random.default_rng(3)
    for chunk in (1, 2, 16, 32, 64, 256):
        for frac in (0.0005, 0.01, 0.3, 1.0):
            fr = np.flatnonzero(rng.random(n) < frac).astype(np.uint32)
            dev = torch.from_numpy(fr.view(np.int32)).cuda()
            wbits, lst = W.frontier_translate(g, dev, chunk)
            mask = np.zeros(n, np.uint8)
            mask[fr] = 1
            want, k = oracle.wedge_frontier(src, mask, chunk)
            words = wbits.cpu().numpy().view(np.uint64)
            got = np.unpackbits(words.view(np.uint8), bitorder="little")[:len(want)]
            np.testing.assert_array_equal(got, want)
            assert lst.numel() == k
            assert np.array_equal(np.sort(lst.cpu().numpy().view(np.uint32)), np.flatnonzero(want))


def test_wedge_frontier_bitmap_relabelled_layout():
    """Frontier given in caller ids; the bitmap is over the internal in-edge order."""
    ro, col = gen.rmat(12, 16, seed=42)
    g = W.Graph.from_csr(ro, col)
    assert g.info["relabeled"] == 1
    n = len(ro) - 1
    perm = g.layout("perm")
    rro, rcol, _ = relabel(ro, col, perm)
    _, isrc, _ = oracle.csc(rro, rcol)
    rng = np.random.default_rng(5)
    for chunk in (1, 16, 64):
        fr = np.flatnonzero(rng.random(n) < 0.02).astype(np.uint32)
        wbits, lst = W.frontier_translate(g, torch.from_numpy(fr.view(np.int32)).cuda(), chunk)
        mask = np.zeros(n, np.uint8)
        mask[perm[fr]] = 1
        want, k = oracle.wedge_frontier(isrc, mask, chunk)
        got = np.unpackbits(wbits.cpu().numpy().view(np.uint8), bitorder="little")[:len(want)]
        np.testing.assert_array_equal(got, want)
        assert lst.numel() == k


def test_worked_example_on_gpu():
    """Design Requirements example: frontier {2, 4} marks exactly its 4 edges at
    one edge per group and 3 groups at two edges per group."""
    pairs = [(2, 4), (2, 6), (4, 8), (4, 9), (1, 6), (3, 8), (5, 9)]
    ro, col = gen.csr_from_edges(10, np.array([p[0] for p in pairs], np.uint32),
                                 np.array([p[1] for p in pairs], np.uint32))
    g = W.Graph.from_csr(ro, col, keep_ids=True)
    fr = torch.tensor([2, 4], dtype=torch.int32, device="cuda")
    _, l1 = W.frontier_translate(g, fr, 1)
    _, l2 = W.frontier_translate(g, fr, 2)
    assert sorted(l1.cpu().tolist()) == [0, 2, 4, 5]
    assert sorted(l2.cpu().tolist()) == [0, 1, 2]


def test_edge_cases():
    # single vertex, no edges
    ro, col = np.zeros(2, np.uint64), np.zeros(0, np.uint32)
    g = W.Graph.from_csr(ro, col, np.zeros(0, np.uint32))
    assert W.u32(W.bfs(g, 0)[0]).tolist() == [0]
    assert W.u32(W.sssp(g, 0)[0]).tolist() == [0]
    r, _ = W.pagerank(g, 20, 0.85)
    assert abs(float(r.cpu()[0]) - 1.0) < 1e-6
    gs = W.Graph.from_csr(ro, col, symmetrize=True)
    assert W.u32(W.cc(gs)[0]).tolist() == [0]
    # source without out-edges, isolated vertices, self-loops and duplicates in input
    src = np.array([0, 0, 1, 2, 3, 3, 5], np.uint32)
    dst = np.array([1, 1, 2, 2, 3, 4, 5], np.uint32)
    order = np.argsort(src, kind="stable")
    ro = np.zeros(8, np.uint64)
    np.add.at(ro, src.astype(np.int64) + 1, 1)
    ro = np.cumsum(ro).astype(np.uint64)
    col = dst[order]
    g = W.Graph.from_csr(ro, col, np.ones(len(col), np.uint32))
    np.testing.assert_array_equal(W.u32(W.bfs(g, 4)[0]), oracle.bfs(ro, col, 4))
    np.testing.assert_array_equal(W.u32(W.bfs(g, 0)[0]), oracle.bfs(ro, col, 0))
    np.testing.assert_array_equal(W.u32(W.sssp(g, 0)[0]),
                                  oracle.sssp(ro, col, np.ones(len(col), np.uint32), 0))
    rk, _ = W.pagerank(g, 20, 0.85)
    ref = oracle.pagerank(ro, col, 20, 0.85)
    assert np.abs(rk.cpu().numpy() - ref).sum() / ref.sum() < 1e-6
    # errors reported through the ABI, before any device work
    with pytest.raises(W.WedgeError) as e:
        W.bfs(g, 99)
    assert e.value.name == "WEDGE_ERR_INVALID_ARG"
    gu = W.Graph.from_csr(ro, col)
    with pytest.raises(W.WedgeError) as e:
        W.sssp(gu, 0)
    assert e.value.name == "WEDGE_ERR_NO_WEIGHTS"
    with pytest.raises(W.WedgeError) as e:
        W.cc(gu)
    assert e.value.name == "WEDGE_ERR_UNSUPPORTED"
    with pytest.raises(W.WedgeError) as e:
        W.bfs(gu, 0, chunk=3)
    assert e.value.name == "WEDGE_ERR_INVALID_ARG"
    with pytest.raises(W.WedgeError) as e:
        W.pagerank(gu, 20, 1.5)
    assert e.value.name == "WEDGE_ERR_INVALID_ARG"


def test_max_iters_reports_not_converged():
    ro, col = gen.grid2d(30, 30)
    g = W.Graph.from_csr(ro, col)
    with pytest.raises(W.WedgeError) as e:
        W.bfs(g, 0, max_iters=5)
    assert e.value.name == "WEDGE_ERR_NOT_CONVERGED"
    out, st, _ = W.bfs(g, 0, max_iters=60)
    np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, 0))


def rel_l1(got, ref):
    return float(np.abs(got.astype(np.float64) - ref).sum() / np.abs(ref).sum())


@pytest.mark.parametrize("keep_ids", [False, True])
@pytest.mark.parametrize("name", ["er_ragged", "rmat12", "rmat14", "grid"])
def test_pagerank_parity(name, keep_ids):
    ro, col = GRAPHS[name]()
    g = W.Graph.from_csr(ro, col, keep_ids=keep_ids)
    r, st = W.pagerank(g, 20, 0.85)
    ref = oracle.pagerank(ro, col, 20, 0.85)
    got = r.cpu().numpy()
    assert rel_l1(got, ref) <= 1e-5
    assert abs(got.astype(np.float64).sum() - 1.0) < 1e-5
    # deterministic: a second run is bitwise identical
    r2, _ = W.pagerank(g, 20, 0.85)
    assert torch.equal(r, r2)


@pytest.mark.parametrize("sliced", ["0", "1"])
@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_pagerank_large_graph_lds_pull(monkeypatch, kind, sliced):
    """Scale 20 is large enough for the pulls that keep the highest-degree
    vertices' contributions in LDS and stride over the tiles (at least four
    tiles per resident wave on 256 CUs), over the canonical in-edge order and
    over the source-sliced copy (one launch per slice, adding into S, then the
    crossing segments' fix-up); results must be the oracle's and
    deterministic."""
    monkeypatch.setenv("WEDGE_SLICED_PULL", sliced)
    ro, col = gen.rmat(20, 16, seed=81)
    if kind == "er":
        ro, col = gen.erdos_renyi(1 << 20, len(col), seed=81)
    g = W.Graph.from_csr(ro, col)
    assert (g.info["rows"] + 7) // 8 >= 4 * 2 * 256 * 12
    assert (g.info["xs_rows"] > 0) == (sliced == "1")
    r, _ = W.pagerank(g, 20, 0.85)
    ref = oracle.pagerank(ro, col, 20, 0.85)
    got = r.cpu().numpy()
    assert rel_l1(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref) / ref) <= 1e-4
    r2, _ = W.pagerank(g, 20, 0.85)
    assert torch.equal(r, r2)


@pytest.mark.parametrize("slices", ["8", "32"])
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("name", ["er_ragged", "rmat12", "rmat14", "grid", "hub"])
def test_pagerank_source_sliced_small(monkeypatch, name, weighted, slices):
    """The sliced PageRank pull forced on small graphs (slices of a few tiles,
    empty slices, a hub whose in-edges cross many tiles in every slice), over
    the plain copy and over the packed copy of a weighted graph (PageRank
    ignores the weights)."""
    monkeypatch.setenv("WEDGE_SLICED_PULL", "1")
    monkeypatch.setenv("WEDGE_XS_SLICES", slices)
    if name == "hub":
        n = 70000
        rng = np.random.default_rng(1)
        src = np.concatenate([np.arange(1, n), rng.integers(0, n, 200000)]).astype(np.uint32)
        dst = np.concatenate([np.zeros(n - 1), rng.integers(1, n, 200000)]).astype(np.uint32)
        ro, col = gen.csr_from_edges(n, src, dst)
    else:
        ro, col = GRAPHS[name]()
    g = W.Graph.from_csr(ro, col, gen.edge_weights(ro, col, seed=5) if weighted else None)
    assert g.info["xs_rows"] > 0
    assert g.info["xs_packed"] == weighted
    if name == "hub":
        assert g.info["xs_pr_spans"] > g.info["xs_pr_short_spans"] > 0
    r, _ = W.pagerank(g, 20, 0.85)
    ref = oracle.pagerank(ro, col, 20, 0.85)
    got = r.cpu().numpy()
    assert rel_l1(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref) / ref) <= 1e-4
    r2, _ = W.pagerank(g, 20, 0.85)
    assert torch.equal(r, r2)
    g.close()


def test_pagerank_closed_forms():
    n = 1000
    cyc = gen.csr_from_edges(n, np.arange(n, dtype=np.uint32),
                             ((np.arange(n) + 1) % n).astype(np.uint32))
    g = W.Graph.from_csr(*cyc)
    r, _ = W.pagerank(g, 20, 0.85)
    assert np.allclose(r.cpu().numpy(), 1.0 / n, rtol=1e-6, atol=0)
    star = gen.csr_from_edges(40, np.arange(1, 40, dtype=np.uint32), np.zeros(39, np.uint32))
    g = W.Graph.from_csr(*star)
    r, _ = W.pagerank(g, 400, 0.85)
    x = (1 + 39 * 0.85) / (40 + 39 * 0.85)
    assert abs(float(r.cpu()[0]) - x) < 1e-6


def test_pagerank_hub_spans_many_tiles():
    """A destination with tens of thousands of in-edges crosses many tiles."""
    n = 70000
    src = np.arange(1, n, dtype=np.uint32)
    dst = np.zeros(n - 1, np.uint32)
    extra_s = np.random.default_rng(1).integers(0, n, 200000).astype(np.uint32)
    extra_d = np.random.default_rng(2).integers(1, n, 200000).astype(np.uint32)
    ro, col = gen.csr_from_edges(n, np.concatenate([src, extra_s]), np.concatenate([dst, extra_d]))
    g = W.Graph.from_csr(ro, col)
    assert g.info["pr_spans"] > 0
    r, _ = W.pagerank(g, 20, 0.85)
    ref = oracle.pagerank(ro, col, 20, 0.85)
    assert rel_l1(r.cpu().numpy(), ref) <= 1e-5


def test_repeated_runs_reuse_workspace():
    ro, col = gen.rmat(12, 16, seed=51)
    w = gen.edge_weights(ro, col, seed=1)
    g = W.Graph.from_csr(ro, col, w)
    srcs = gen.pick_sources(ro, 4, seed=3)
    for s in srcs:
        for chunk in (64, 16, 1, 32):
            np.testing.assert_array_equal(W.u32(W.bfs(g, int(s), chunk=chunk)[0]),
                                          oracle.bfs(ro, col, int(s)))
            np.testing.assert_array_equal(W.u32(W.sssp(g, int(s), chunk=chunk)[0]),
                                          oracle.sssp(ro, col, w, int(s)))


def device_bytes(g):
    info = W._binding.GraphInfo()
    W._binding.check(W._binding.lib().wedge_graph_get_info(g.handle, W._binding.C.byref(info)))
    return info.device_bytes


def test_device_memory_cap_fails_cleanly_and_recovers(monkeypatch):
    """The per-graph device cap refuses creation, and a run whose workspace
    stops part-way; once lifted, the same graph completes its workspace and
    every result still equals the oracle."""
    ro, col = gen.rmat(12, 16, seed=61)
    w = gen.edge_weights(ro, col, seed=2)
    n = len(ro) - 1
    probe = W.Graph.from_csr(ro, col, w)
    layout = device_bytes(probe)
    probe.close()
    print(f"  [cap: layout {layout} bytes, n={n}]", flush=True)
    monkeypatch.setenv("WEDGE_MAX_DEVICE_BYTES", str(layout // 2))
    with pytest.raises(W.WedgeError) as e:
        W.Graph.from_csr(ro, col, w)
    assert e.value.name == "WEDGE_ERR_OOM"
    # room for the layout and the first few workspace buffers only
    monkeypatch.setenv("WEDGE_MAX_DEVICE_BYTES", str(layout + 4 * n + 4096))
    g = W.Graph.from_csr(ro, col, w)
    assert device_bytes(g) == layout
    for run in (lambda: W.bfs(g, 0, chunk=16), lambda: W.sssp(g, 0, chunk=16)):
        with pytest.raises(W.WedgeError) as e:
            run()
        assert e.value.name == "WEDGE_ERR_OOM"
    partial = device_bytes(g)
    assert layout < partial <= layout + 4 * n + 4096
    monkeypatch.delenv("WEDGE_MAX_DEVICE_BYTES")
    np.testing.assert_array_equal(W.u32(W.bfs(g, 0, chunk=16)[0]), oracle.bfs(ro, col, 0))
    np.testing.assert_array_equal(W.u32(W.sssp(g, 0, chunk=16)[0]), oracle.sssp(ro, col, w, 0))
    # the multi-source buffers: the visited masks fit, the second frontier mask does not
    full = device_bytes(g)
    srcs = gen.pick_sources(ro, 8, seed=5)
    monkeypatch.setenv("WEDGE_MAX_DEVICE_BYTES", str(full + 2 * 8 * n + 256))
    with pytest.raises(W.WedgeError) as e:
        W.bfs_multisource(g, srcs, chunk=16)
    assert e.value.name == "WEDGE_ERR_OOM"
    assert device_bytes(g) > full
    monkeypatch.delenv("WEDGE_MAX_DEVICE_BYTES")
    lv, _, _ = W.bfs_multisource(g, srcs, chunk=16)
    lv = W.u32(lv).reshape(len(srcs), n)
    for i, s in enumerate(srcs):
        np.testing.assert_array_equal(lv[i], oracle.bfs(ro, col, int(s)))
    # PageRank's buffers: the sums fit, the contributions do not
    full = device_bytes(g)
    monkeypatch.setenv("WEDGE_MAX_DEVICE_BYTES", str(full + 4 * n + 256))
    with pytest.raises(W.WedgeError) as e:
        W.pagerank(g, iters=5)
    assert e.value.name == "WEDGE_ERR_OOM"
    assert device_bytes(g) > full
    monkeypatch.delenv("WEDGE_MAX_DEVICE_BYTES")
    r, _ = W.pagerank(g, iters=5)
    assert rel_l1(r.cpu().numpy(), oracle.pagerank(ro, col, 5, 0.85)) <= 1e-5
    g.close()

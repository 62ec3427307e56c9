"""GPU parity at the benchmark's full sizes and launch configuration.

R-MAT scale 16 (BFS, 8 sources) and the scale-24 R-MAT and Erdos-Renyi graphs
(BFS, SSSP, CC, PageRank) are checked against the CPU oracle computed in full:
bit-exact for integers, per-iteration frontier size, out-degree sum and gate
decision for every BFS and SSSP source the benchmark times, and <= 1e-5
relative L1 for PageRank.
The scale-26 PageRank case (1.06B edges) runs too, printing its progress.
"""
import time

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1903_07754_amd as W  # noqa: E402


def say(msg):
    print(f"  [fullsize] {msg}", flush=True)


def rel_l1(got, ref):
    return float(np.abs(got.astype(np.float64) - ref).sum() / np.abs(ref).sum())


@pytest.mark.timeout(600)
def test_config1_rmat16_bfs_eight_sources():
    ro, col = gen.rmat(16, 16, seed=1)
    g = W.Graph.from_csr(ro, col)
    for s in gen.pick_sources(ro, 8, seed=2):
        s = int(s)
        out, st, tr = W.bfs(g, s, theta_ppm=10_000, chunk=32, trace_cap=64)
        np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, s))
        ref = oracle.pull_engine("bfs", ro, col, None, s, theta_ppm=10_000, chunk=0)
        assert [r["frontier"] for r in tr] == list(ref.F)
        assert [r["active_edges"] for r in tr] == list(ref.A)
        assert [r["mode"] for r in tr] == list(ref.mode)


class Big:
    """One scale-24 graph held for the tests of its kind."""

    def __init__(self, kind):
        t = time.time()
        if kind == "rmat":
            self.ro, self.col = gen.rmat(24, 16, seed=1)
        else:
            m = _m_rmat24.get("m") or int(gen.rmat(24, 16, seed=1)[0][-1])
            self.ro, self.col = gen.erdos_renyi(1 << 24, m, seed=2)
        if kind == "rmat":
            _m_rmat24["m"] = len(self.col)
        self.w = gen.edge_weights(self.ro, self.col, seed=4)
        self.srcs = [int(s) for s in gen.pick_sources(self.ro, 4, seed=3)]
        say(f"{kind} n={len(self.ro) - 1} m={len(self.col)} generated in {time.time() - t:.1f}s")
        t = time.time()
        self.g = W.Graph.from_csr(self.ro, self.col, self.w)
        say(f"{kind} directed layout in {time.time() - t:.1f}s")
        self._gs = None

    @property
    def gs(self):
        if self._gs is None:
            t = time.time()
            self._gs = W.Graph.from_csr(self.ro, self.col, symmetrize=True)
            say(f"undirected layout in {time.time() - t:.1f}s")
        return self._gs


_cache = {}
_m_rmat24 = {}


def big(kind):
    if kind not in _cache:
        _cache.clear()
        _cache[kind] = Big(kind)
    return _cache[kind]


def level_trace(levels, outdeg, thr):
    """Per-iteration |F_k|, A_k and gate decision of a synchronous BFS, read off
    its final levels: the frontier consumed by iteration k is exactly the set
    of vertices at level k."""
    lv = np.asarray(levels)
    reached = lv[lv != oracle.INF]
    depth = int(reached.max()) + 1 if reached.size else 0
    F = np.bincount(reached, minlength=depth).astype(np.int64)
    A = np.bincount(reached, weights=outdeg[lv != oracle.INF], minlength=depth).astype(np.int64)
    return list(F), list(A), [1 if a < thr else 0 for a in A]


def check_bfs_sssp(kind):
    """Every source the benchmark times (4 per graph), each with its
    per-iteration records: BFS against the level sets of the oracle's BFS (and,
    for the first source, against the oracle's pull engine as well), SSSP
    against the oracle's pull engine."""
    b = big(kind)
    m = len(b.col)
    outdeg = np.diff(b.ro.astype(np.int64))
    for i, s in enumerate(b.srcs):
        out, st, tr = W.bfs(b.g, s, trace_cap=256)
        want = oracle.bfs(b.ro, b.col, s)
        np.testing.assert_array_equal(W.u32(out), want)
        F, A, mode = level_trace(want, outdeg, oracle.threshold_edges(10_000, m))
        assert [r["frontier"] for r in tr] == F
        assert [r["active_edges"] for r in tr] == A
        assert [r["mode"] for r in tr] == mode
        if i == 0:
            ref = oracle.pull_engine("bfs", b.ro, b.col, None, s, theta_ppm=10_000, chunk=0)
            assert (list(ref.F), list(ref.A), list(ref.mode)) == (F, A, mode)
        say(f"{kind} bfs src={s} ok with its trace ({st['iterations']} iters, {st['ms']:.2f} ms)")
        d, st, trs = W.sssp(b.g, s, trace_cap=4096)
        np.testing.assert_array_equal(W.u32(d), oracle.sssp(b.ro, b.col, b.w, s))
        ref = oracle.pull_engine("sssp", b.ro, b.col, b.w, s, theta_ppm=50_000, chunk=0)
        assert [r["frontier"] for r in trs] == list(ref.F)
        assert [r["active_edges"] for r in trs] == list(ref.A)
        assert [r["mode"] for r in trs] == list(ref.mode)
        say(f"{kind} sssp src={s} ok with its trace ({st['iterations']} iters, {st['ms']:.2f} ms)")


def check_cc(kind):
    b = big(kind)
    out, st, _ = W.cc(b.gs)
    np.testing.assert_array_equal(W.u32(out), oracle.cc(b.ro, b.col))
    say(f"{kind} cc ok ({st['iterations']} iters, {st['ms']:.2f} ms)")


@pytest.mark.timeout(1200)
def test_config2_rmat24_bfs_sssp():
    check_bfs_sssp("rmat")


@pytest.mark.timeout(900)
def test_config2_rmat24_cc():
    check_cc("rmat")


@pytest.mark.timeout(900)
def test_rmat24_every_iteration_wedge():
    """Every iteration on the Wedge Frontier, at each group size the learned
    gate can pick: at scale 24 the chunk pulls stride over millions of marked
    chunks per launch, which the default gate only reaches in a few sparse
    iterations. Results must still be the oracle's."""
    b = big("rmat")
    s = b.srcs[1]
    want_bfs = oracle.bfs(b.ro, b.col, s)
    want_sssp = oracle.sssp(b.ro, b.col, b.w, s)
    want_cc = oracle.cc(b.ro, b.col)
    for chunk in (16, 32, 64):
        out, st, _ = W.bfs(b.g, s, gate="wedge", chunk=chunk)
        np.testing.assert_array_equal(W.u32(out), want_bfs)
        assert st["full_iters"] == 0
        out, st, _ = W.sssp(b.g, s, gate="wedge", chunk=chunk)
        np.testing.assert_array_equal(W.u32(out), want_sssp)
        out, st, _ = W.cc(b.gs, gate="wedge", chunk=chunk)
        np.testing.assert_array_equal(W.u32(out), want_cc)
        say(f"rmat wedge-only chunk={chunk} bfs/sssp/cc ok")


@pytest.mark.timeout(900)
def test_rmat24_pagerank():
    b = big("rmat")
    r, st = W.pagerank(b.g, 20, 0.85)
    ref = oracle.pagerank(b.ro, b.col, 20, 0.85)
    e = rel_l1(r.cpu().numpy(), ref)
    say(f"pagerank s24 rel L1 {e:.3e} ({st['ms']:.1f} ms)")
    assert e <= 1e-5


@pytest.mark.timeout(900)
def test_config4_learned_gate_rmat24_exact():
    """The shipped learned gate at scale 24: every result bit-exact (its
    decisions may differ from the threshold rule's, the values may not)."""
    b = big("rmat")
    from paper_1903_07754_amd import learned_gate as LG
    model = W.Model.load(LG.DEFAULT_MODEL)
    s = b.srcs[2]
    out, st, _ = W.bfs(b.g, s, gate="learned", model=model.handle)
    np.testing.assert_array_equal(W.u32(out), oracle.bfs(b.ro, b.col, s))
    out, st, _ = W.sssp(b.g, s, gate="learned", model=model.handle)
    np.testing.assert_array_equal(W.u32(out), oracle.sssp(b.ro, b.col, b.w, s))
    out, st, _ = W.cc(b.gs, gate="learned", model=model.handle)
    np.testing.assert_array_equal(W.u32(out), oracle.cc(b.ro, b.col))
    say(f"rmat learned gate bfs/sssp/cc ok (margin {model.margin():.2f})")


@pytest.mark.timeout(1200)
def test_config2_er24_bfs_sssp():
    check_bfs_sssp("er")


@pytest.mark.timeout(900)
def test_config2_er24_cc():
    check_cc("er")
    _cache.clear()


@pytest.mark.timeout(1500)
def test_config3_pagerank_rmat26():
    t = time.time()
    ro, col = gen.rmat(26, 16, seed=1)
    say(f"rmat26 n={len(ro) - 1} m={len(col)} generated in {time.time() - t:.0f}s")
    t = time.time()
    g = W.Graph.from_csr(ro, col)
    say(f"rmat26 layout built and uploaded in {time.time() - t:.0f}s")
    r, st = W.pagerank(g, 20, 0.85, time_pull=True)
    got = r.cpu().numpy()
    pull_us = st["pull_ms"] / st["pull_launches"] * 1e3
    say(f"rmat26 pagerank on the GPU: {st['ms']:.1f} ms, pull {pull_us:.0f} us per launch "
        f"({20 * len(col) / st['ms'] / 1e6:.1f} GTEPS)")
    del g
    t = time.time()
    ref = oracle.pagerank(ro, col, 20, 0.85)
    say(f"rmat26 oracle in {time.time() - t:.0f}s")
    e = rel_l1(got, ref)
    say(f"pagerank s26 rel L1 {e:.3e}")
    assert e <= 1e-5
    assert abs(got.astype(np.float64).sum() - 1.0) < 1e-4


@pytest.mark.timeout(900)
def test_config5_multisource_rmat22_64_sources():
    """The bench's 64-source workload (R-MAT scale 22, seeds 5 and 6): every
    one of the 64 rows equals the oracle's BFS, host-driven and persistent."""
    ro, col = gen.rmat(22, 16, seed=5)
    srcs = gen.pick_sources(ro, 64, seed=6)
    g = W.Graph.from_csr(ro, col)
    n = len(ro) - 1
    want = np.stack([oracle.bfs(ro, col, int(s)) for s in srcs])
    say(f"rmat22 oracle for 64 sources done (n={n} m={len(col)})")
    for persistent in (False, True):
        lv, st, _ = W.bfs_multisource(g, srcs, persistent=persistent)
        np.testing.assert_array_equal(lv.cpu().numpy().view(np.uint32), want)
        say(f"rmat22 64-source persistent={persistent} ok ({st['iterations']} iters, {st['ms']:.2f} ms)")
    g.close()


@pytest.mark.timeout(900)
def test_config5_batch_of_256_graphs():
    """The bench's 256-graph batch (scales 10..16, seeds 7, 3000+i, 4000+i):
    every part equals the oracle's BFS of its own graph."""
    scales = gen.batch_scales(256, 10, 16, seed=7)
    parts = [gen.rmat(int(s), 16, seed=3000 + i) for i, s in enumerate(scales)]
    srcs = np.array([int(gen.pick_sources(r, 1, seed=4000 + i)[0]) for i, (r, _) in enumerate(parts)],
                    np.uint32)
    gb = W.Graph.from_batch_csr(parts)
    first = gb.parts()
    want = [oracle.bfs(r, c, int(srcs[i])) for i, (r, c) in enumerate(parts)]
    for persistent in (False, True):
        got = W.u32(W.bfs_batch(gb, srcs, persistent=persistent)[0])
        for i in range(len(parts)):
            np.testing.assert_array_equal(got[first[i]:first[i + 1]], want[i])
        say(f"256-graph batch persistent={persistent} ok (n={gb.n})")
    gb.close()

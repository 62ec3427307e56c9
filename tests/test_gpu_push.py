"""GPU parity of the push engine and the hybrid baseline (push below the
threshold, a pull over every in-edge above it), through the C ABI.

Every engine shares the iteration semantics of the pull (values committed at
the end of the previous iteration; a vertex joins the next frontier exactly
when its value drops), so results must equal the oracle bit for bit, and the
per-iteration frontier sizes and out-degree sums must equal the oracle's pull
engine and its textbook push engine in every iteration. The hybrid's mode in
iteration k must be push exactly when A_k < floor(theta * m).
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1903_07754_amd as W  # noqa: E402

MODE_FULL, MODE_WEDGE, MODE_PUSH = 0, 1, 2


def graph_and_ref(app, ro, col, w, src, keep_ids=False):
    if app == "cc":
        gro, gcol = oracle.symmetrize(ro, col)
        g = W.Graph.from_csr(ro, col, symmetrize=True, keep_ids=keep_ids)
        want = oracle.cc(ro, col)
        push = oracle.push_engine("cc", gro, gcol)
    else:
        gro, gcol = ro, col
        g = W.Graph.from_csr(ro, col, w, keep_ids=keep_ids)
        want = oracle.bfs(ro, col, src) if app == "bfs" else oracle.sssp(ro, col, w, src)
        push = oracle.push_engine(app, ro, col, w if app == "sssp" else None, src)
    ref = oracle.pull_engine(app, gro, gcol, w if app == "sssp" else None, src, theta_ppm=10_000,
                             chunk=0)
    np.testing.assert_array_equal(ref.values, want)
    np.testing.assert_array_equal(push[0], want)
    assert push[1] == ref.iters
    np.testing.assert_array_equal(push[2], ref.F)
    return g, ref, want, int(gcol.shape[0])


def run(app, g, src, **kw):
    print(f"  [{app} n={g.n} m={g.m} src={src} {kw}]", flush=True)
    fn = {"bfs": W.bfs, "sssp": W.sssp}.get(app)
    if fn is None:
        out, st, tr = W.cc(g, trace_cap=g.n + 2, **kw)
    else:
        out, st, tr = fn(g, src, trace_cap=g.n + 2, **kw)
    torch.cuda.synchronize()
    return W.u32(out), st, tr


def check(app, ro, col, w=None, src=0, keep_ids=False, theta=None):
    g, ref, want, m = graph_and_ref(app, ro, col, w, src, keep_ids)
    for gate in ("push", "hybrid"):
        kw = {"gate": gate}
        if theta is not None and gate == "hybrid":
            kw["theta_ppm"] = theta
        got, st, tr = run(app, g, src, **kw)
        np.testing.assert_array_equal(got, want)
        assert st["iterations"] == ref.iters
        thr = (int(theta if theta is not None else 50_000) * m) // 1_000_000
        for k, r in enumerate(tr):
            assert r["frontier"] == ref.F[k], (gate, k)
            assert r["active_edges"] == ref.A[k], (gate, k)
            if gate == "push":
                assert r["mode"] == MODE_PUSH, k
            else:
                assert r["mode"] == (MODE_PUSH if ref.A[k] < thr else MODE_FULL), (k, ref.A[k], thr)
        npush = sum(1 for r in tr if r["mode"] == MODE_PUSH)
        assert st["push_iters"] == npush
        assert st["full_iters"] + st["push_iters"] == st["iterations"]
    g.close()


@pytest.mark.parametrize("app", ["bfs", "sssp", "cc"])
@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_push_and_hybrid_match_oracle(app, kind):
    if kind == "rmat":
        ro, col = gen.rmat(13, 16, seed=31)
    else:
        ro, col = gen.erdos_renyi(5000, 40_000, seed=32)
    w = gen.edge_weights(ro, col, seed=4)
    src = int(gen.pick_sources(ro, 1, seed=33)[0])
    check(app, ro, col, w, src)


@pytest.mark.parametrize("app", ["bfs", "sssp", "cc"])
def test_push_keep_ids_grid_and_thresholds(app):
    # a high-diameter mesh in the caller's vertex order, ragged n
    ro, col = gen.grid2d(37, 53)
    w = gen.edge_weights(ro, col, seed=4)
    check(app, ro, col, w, src=0, keep_ids=True)
    ro, col = gen.rmat(11, 8, seed=35)
    w = gen.edge_weights(ro, col, seed=4)
    src = int(gen.pick_sources(ro, 1, seed=36)[0])
    for theta in (1, 200_000, 1_000_000):
        check(app, ro, col, w, src, theta=theta)


def test_push_degenerate_sources():
    # a source without out-edges: one iteration, nothing pushed
    ro = np.array([0, 0, 1, 2, 2], np.uint64)
    col = np.array([0, 1], np.uint32)
    g = W.Graph.from_csr(ro, col, keep_ids=True)
    for gate in ("push", "hybrid"):
        lv, st, tr = W.bfs(g, 0, gate=gate, trace_cap=8)
        assert list(W.u32(lv)) == [0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]
        assert st["iterations"] == 1 and tr[0]["active_edges"] == 0
    g.close()


def test_push_batch_bfs():
    parts = [gen.rmat(s, 8, seed=500 + s) for s in (8, 10, 9)]
    srcs = np.array([int(gen.pick_sources(r, 1, seed=600 + i)[0]) for i, (r, _) in enumerate(parts)],
                    np.uint32)
    gb = W.Graph.from_batch_csr(parts)
    first = gb.parts()
    for gate in ("push", "hybrid"):
        out, st, _ = W.bfs_batch(gb, srcs, gate=gate)
        torch.cuda.synchronize()
        got = W.u32(out)
        for i, (r, c) in enumerate(parts):
            np.testing.assert_array_equal(got[int(first[i]):int(first[i + 1])], oracle.bfs(r, c, int(srcs[i])))
    gb.close()


def test_push_refusals():
    ro, col = gen.rmat(10, 8, seed=2)
    g = W.Graph.from_csr(ro, col)
    srcs = gen.pick_sources(ro, 4, seed=3)
    for gate in ("push", "hybrid"):
        with pytest.raises(W.WedgeError) as e:
            W.bfs_multisource(g, srcs, gate=gate)
        assert e.value.name == "WEDGE_ERR_UNSUPPORTED"
        with pytest.raises(W.WedgeError) as e:
            W.bfs(g, int(srcs[0]), gate=gate, persistent=True)
        assert e.value.name == "WEDGE_ERR_UNSUPPORTED"
        with pytest.raises(W.WedgeError) as e:
            W.bfs_noalloc(g, int(srcs[0]), gate=gate)
        assert e.value.name == "WEDGE_ERR_UNSUPPORTED"
    g.close()


def test_push_builds_out_edges_once():
    ro, col = gen.rmat(12, 16, seed=40)
    w = gen.edge_weights(ro, col, seed=4)
    g = W.Graph.from_csr(ro, col, w)
    src = int(gen.pick_sources(ro, 1, seed=41)[0])
    W.sssp(g, src)
    b0 = g.info["device_bytes"]
    W.sssp(g, src, gate="push")
    b1 = g.info["device_bytes"]
    assert b1 == b0 + 8 * g.m  # destinations and weights, 4 bytes each per edge
    d, _, _ = W.sssp(g, src, gate="push")
    torch.cuda.synchronize()
    assert g.info["device_bytes"] == b1
    np.testing.assert_array_equal(W.u32(d), oracle.sssp(ro, col, w, src))
    g.close()

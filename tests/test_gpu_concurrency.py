"""Concurrent use of the library from several host threads.

Each thread owns one graph and one stream and runs BFS, SSSP, PageRank and a
persistent (graph-captured) BFS on it while the other threads do the same;
every result must equal the oracle. A second test runs many threads on one
shared graph: every call must either return a correct result or refuse with
WEDGE_ERR_BUSY (the graph's workspace is not shared between runs).
"""
import threading

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1903_07754_amd as W  # noqa: E402


def rel_l1(got, ref):
    return float(np.abs(got.astype(np.float64) - ref).sum() / np.abs(ref).sum())


def run_threads(targets, timeout=90.0):
    errors = []

    def wrap(fn):
        def body():
            try:
                fn()
            except BaseException as e:  # reported to the main thread
                errors.append(e)
        return body

    threads = [threading.Thread(target=wrap(t), daemon=True) for t in targets]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout)
        assert not t.is_alive(), "a worker thread did not finish"
    if errors:
        raise errors[0]


def test_threads_on_separate_graphs():
    cases = [gen.rmat(12, 16, seed=71), gen.random_graph(3000, 40000, 72), gen.rmat(13, 8, seed=73)]
    want = []
    for ro, col in cases:
        w = gen.edge_weights(ro, col, seed=5)
        srcs = [int(s) for s in gen.pick_sources(ro, 2, seed=6)]
        want.append((ro, col, w, srcs, [oracle.bfs(ro, col, s) for s in srcs],
                     [oracle.sssp(ro, col, w, s) for s in srcs], oracle.pagerank(ro, col, 20, 0.85)))
    graphs = [W.Graph.from_csr(ro, col, w) for ro, col, w, *_ in want]

    def worker(i):
        ro, col, w, srcs, bfs_ref, sssp_ref, pr_ref = want[i]
        g = graphs[i]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            for rep in range(3):
                for s, lb, ds in zip(srcs, bfs_ref, sssp_ref):
                    np.testing.assert_array_equal(W.u32(W.bfs(g, s, stream=stream)[0]), lb)
                    np.testing.assert_array_equal(W.u32(W.sssp(g, s, stream=stream)[0]), ds)
                    np.testing.assert_array_equal(W.u32(W.bfs(g, s, stream=stream, persistent=True)[0]), lb)
                r, _ = W.pagerank(g, stream=stream)
                stream.synchronize()
                assert rel_l1(r.cpu().numpy(), pr_ref) <= 1e-5

    print(f"  [threads: {len(graphs)} graphs]", flush=True)
    run_threads([lambda i=i: worker(i) for i in range(len(graphs))])
    for g in graphs:
        g.close()


def test_threads_on_one_graph_are_correct_or_busy():
    ro, col = gen.rmat(12, 16, seed=74)
    g = W.Graph.from_csr(ro, col)
    srcs = [int(s) for s in gen.pick_sources(ro, 4, seed=7)]
    ref = {s: oracle.bfs(ro, col, s) for s in srcs}
    outcome = {"ok": 0, "busy": 0}
    lock = threading.Lock()

    def worker(s):
        stream = torch.cuda.Stream()
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for _ in range(20):
            try:
                lv = W.u32(W.bfs(g, s, out=out, stream=stream)[0])
            except W.WedgeError as e:
                assert e.name == "WEDGE_ERR_BUSY", e
                with lock:
                    outcome["busy"] += 1
                continue
            np.testing.assert_array_equal(lv, ref[s])
            with lock:
                outcome["ok"] += 1

    print(f"  [threads: one graph, {len(srcs)} threads]", flush=True)
    run_threads([lambda s=s: worker(s) for s in srcs])
    assert outcome["ok"] > 0 and outcome["ok"] + outcome["busy"] == 20 * len(srcs)
    # after the contention the graph is free and correct
    np.testing.assert_array_equal(W.u32(W.bfs(g, srcs[0])[0]), ref[srcs[0]])
    g.close()

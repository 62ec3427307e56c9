"""GPU parity of the batched BFS kinds against the CPU oracle.

Multi-source BFS (64-bit masks) must equal one oracle BFS per source, and its
per-iteration union frontier must equal {v : some source reaches v at level
k}. The many-graph batch must equal one oracle BFS per part. The persistent
launch (one kernel, grid barriers, captured in a hipGraph and replayed) must
give exactly the host-driven results and records.
"""
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1903_07754_amd as W  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

INF = oracle.INF


def union_trace(levels, outdeg):
    """|F_k| and A_k of the union frontier implied by per-source levels."""
    lv = np.asarray(levels)
    F, A = [], []
    k = 0
    while True:
        fr = (lv == k).any(axis=0)
        if not fr.any():
            break
        F.append(int(fr.sum()))
        A.append(int(outdeg[fr].sum()))
        k += 1
    return F, A


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("k", [1, 7, 63, 64])
def test_multisource_equals_per_source_bfs(k, persistent):
    ro, col = gen.rmat(13, 16, seed=61)
    g = W.Graph.from_csr(ro, col)
    srcs = gen.pick_sources(ro, k, seed=k)
    print(f"  [multisource k={k} persistent={persistent}]", flush=True)
    lv, st, tr = W.bfs_multisource(g, srcs, trace_cap=256, persistent=persistent)
    got = lv.cpu().numpy().view(np.uint32)
    want = np.stack([oracle.bfs(ro, col, int(s)) for s in srcs])
    np.testing.assert_array_equal(got, want)
    F, A = union_trace(want, np.diff(ro.astype(np.int64)))
    assert [r["frontier"] for r in tr] == F
    assert [r["active_edges"] for r in tr] == A
    thr = (10_000 * len(col)) // 1_000_000
    assert [r["mode"] for r in tr] == [1 if a < thr else 0 for a in A]


@pytest.mark.parametrize("gate,chunk", [("wedge", 1), ("wedge", 64), ("full", 32), ("threshold", 16)])
def test_multisource_gate_and_chunk_invariance(gate, chunk):
    ro, col = gen.random_graph(5000, 40000, 62)
    g = W.Graph.from_csr(ro, col)
    srcs = gen.pick_sources(ro, 40, seed=5)
    want = np.stack([oracle.bfs(ro, col, int(s)) for s in srcs])
    for persistent in (False, True):
        lv, _, _ = W.bfs_multisource(g, srcs, gate=gate, chunk=chunk, persistent=persistent)
        np.testing.assert_array_equal(lv.cpu().numpy().view(np.uint32), want)


def make_parts(count, seed, lo=4, hi=11):
    rng = np.random.default_rng(seed)
    scales = rng.integers(lo, hi + 1, count)
    parts = [gen.rmat(int(s), 16, seed=3000 + i) for i, s in enumerate(scales)]
    srcs = np.array([int(gen.pick_sources(r, 1, seed=i)[0]) for i, (r, _) in enumerate(parts)],
                    np.uint32)
    return parts, srcs


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("keep_ids", [False, True])
def test_batch_equals_per_part_bfs(persistent, keep_ids):
    parts, srcs = make_parts(40, 7)
    g = W.Graph.from_batch_csr(parts, keep_ids=keep_ids)
    first = g.parts()
    lv, st, tr = W.bfs_batch(g, srcs, trace_cap=256, persistent=persistent)
    got = W.u32(lv)
    for i, (r, c) in enumerate(parts):
        np.testing.assert_array_equal(got[first[i]:first[i + 1]], oracle.bfs(r, c, int(srcs[i])))
    # union frontier of the batch = union over parts of their level-k sets
    F = []
    k = 0
    while (got == k).any():
        F.append(int((got == k).sum()))
        k += 1
    assert [r["frontier"] for r in tr] == F


@pytest.mark.parametrize("rows", [4, 16])
def test_pull_shapes_give_identical_results(rows):
    """Every pull shape (rows per wave step) gives the oracle's levels and the
    default shape's per-iteration records, for each BFS kind, over chunk sizes
    whose chunk-list reads take each of the three slot forms."""
    ro, col = gen.rmat(13, 16, seed=67)
    g = W.Graph.from_csr(ro, col)
    srcs = gen.pick_sources(ro, 9, seed=14)
    want = np.stack([oracle.bfs(ro, col, int(s)) for s in srcs])
    keys = ("frontier", "active_edges", "mode", "marked_chunks", "chunk_edges")
    print(f"  [pull shape rows={rows}]", flush=True)
    for chunk in (1, 16, 128):
        for gate in ("threshold", "wedge", "full"):
            a, _, ta = W.bfs(g, int(srcs[0]), trace_cap=64, gate=gate, chunk=chunk)
            b, _, tb = W.bfs(g, int(srcs[0]), trace_cap=64, gate=gate, chunk=chunk, rows_per_wave=rows)
            np.testing.assert_array_equal(W.u32(b), want[0])
            assert [[r[k] for k in keys] for r in ta] == [[r[k] for k in keys] for r in tb]
            lv, _, _ = W.bfs_multisource(g, srcs, gate=gate, chunk=chunk, rows_per_wave=rows)
            np.testing.assert_array_equal(lv.cpu().numpy().view(np.uint32), want)
    parts, bsrcs = make_parts(20, 9)
    gb = W.Graph.from_batch_csr(parts)
    first = gb.parts()
    got = W.u32(W.bfs_batch(gb, bsrcs, rows_per_wave=rows)[0])
    for i, (r, c) in enumerate(parts):
        np.testing.assert_array_equal(got[first[i]:first[i + 1]], oracle.bfs(r, c, int(bsrcs[i])))


def test_pull_shape_errors():
    ro, col = gen.rmat(10, 16, seed=68)
    w = gen.edge_weights(ro, col, seed=3)
    g = W.Graph.from_csr(ro, col, w)
    gs = W.Graph.from_csr(ro, col, symmetrize=True)
    cases = [(lambda: W.bfs(g, 0, rows_per_wave=5), "WEDGE_ERR_INVALID_ARG"),
             (lambda: W.bfs(g, 0, rows_per_wave=16, persistent=True), "WEDGE_ERR_UNSUPPORTED"),
             (lambda: W.sssp(g, 0, rows_per_wave=4), "WEDGE_ERR_UNSUPPORTED"),
             (lambda: W.cc(gs, rows_per_wave=16), "WEDGE_ERR_UNSUPPORTED"),
             (lambda: W.pagerank(g, iters=2, rows_per_wave=4), "WEDGE_ERR_UNSUPPORTED")]
    for run, name in cases:
        with pytest.raises(W.WedgeError) as e:
            run()
        assert e.value.name == name
    # the default shape, spelled out, is accepted everywhere
    np.testing.assert_array_equal(W.u32(W.sssp(g, 0, rows_per_wave=8)[0]), oracle.sssp(ro, col, w, 0))


def test_persistent_bfs_matches_host_driven_records():
    ro, col = gen.rmat(14, 16, seed=63)
    g = W.Graph.from_csr(ro, col)
    for s in gen.pick_sources(ro, 3, seed=9):
        s = int(s)
        a, sa, ta = W.bfs(g, s, trace_cap=128)
        b, sb, tb = W.bfs(g, s, trace_cap=128, persistent=True)
        np.testing.assert_array_equal(W.u32(a), oracle.bfs(ro, col, s))
        np.testing.assert_array_equal(W.u32(b), W.u32(a))
        assert sa["iterations"] == sb["iterations"]
        for ra, rb in zip(ta, tb):
            for key in ("frontier", "active_edges", "mode", "marked_chunks", "chunk_edges"):
                assert ra[key] == rb[key], (key, ra, rb)


def test_persistent_replay_after_workspace_grows():
    """A captured persistent traversal holds the workspace addresses it was
    recorded with. A run that needs a larger Wedge bitmap or chunk list (SSSP
    at 16 edges per bit, after a persistent BFS at 32) reallocates them; the
    next persistent BFS into the same output must be recorded again, not
    replayed against the freed buffers."""
    ro, col = gen.rmat(14, 16, seed=67)
    w = gen.edge_weights(ro, col, seed=4)
    g = W.Graph.from_csr(ro, col, w)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    srcs = [int(s) for s in gen.pick_sources(ro, 3, seed=13)]
    print(f"  [persistent replay after growth: n={g.n} m={g.m}]", flush=True)
    W.bfs(g, srcs[0], out=out, chunk=32, persistent=True)
    np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, srcs[0]))
    W.sssp(g, srcs[1], out=dist, chunk=16)
    np.testing.assert_array_equal(W.u32(dist), oracle.sssp(ro, col, w, srcs[1]))
    W.bfs(g, srcs[2], out=out, chunk=32, persistent=True)
    np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, srcs[2]))
    W.sssp(g, srcs[0], out=dist, chunk=1)
    np.testing.assert_array_equal(W.u32(dist), oracle.sssp(ro, col, w, srcs[0]))
    W.bfs(g, srcs[1], out=out, chunk=32, persistent=True)
    np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, srcs[1]))


def test_graph_replays_with_eager_work_between():
    """The captured traversal is replayed many times (new sources each time, same
    graph), with the program's own device work and synchronisations between
    replays; every replay must equal the oracle."""
    ro, col = gen.rmat(12, 16, seed=64)
    g = W.Graph.from_csr(ro, col)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    x = torch.randn(1 << 20, device="cuda")
    for rep, s in enumerate(gen.pick_sources(ro, 6, seed=10)):
        W.bfs(g, int(s), out=out, persistent=True)
        y = (x * rep).sum()          # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, int(s)))
        assert torch.isfinite(y)
    srcs = gen.pick_sources(ro, 64, seed=11)
    want = np.stack([oracle.bfs(ro, col, int(s)) for s in srcs])
    for rep in range(3):
        lv, _, _ = W.bfs_multisource(g, srcs, persistent=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(lv.cpu().numpy().view(np.uint32), want)


def test_barrier_deadline_is_reported_not_hung(monkeypatch):
    """With a zero barrier deadline forced from the host, the persistent kernel
    gives up at its first wait, every block exits, and the call reports an
    error; the next run (default deadline) is correct again."""
    ro, col = gen.rmat(11, 16, seed=65)
    g = W.Graph.from_csr(ro, col)
    s = int(gen.pick_sources(ro, 1, seed=12)[0])
    monkeypatch.setenv("WEDGE_BARRIER_TIMEOUT_MS", "0")
    with pytest.raises(W.WedgeError) as e:
        W.bfs(g, s, persistent=True)
    assert e.value.name == "WEDGE_ERR_HIP"
    monkeypatch.delenv("WEDGE_BARRIER_TIMEOUT_MS")
    out, _, _ = W.bfs(g, s, persistent=True)
    np.testing.assert_array_equal(W.u32(out), oracle.bfs(ro, col, s))


def test_autotuner_picks_a_candidate_and_results_hold():
    ro, col = gen.rmat(12, 16, seed=66)
    g = W.Graph.from_csr(ro, col)
    srcs = gen.pick_sources(ro, 64, seed=13)
    out = torch.empty(64 * g.n, dtype=torch.int32, device="cuda")
    best, ms = W.tune_bfs(g, "multisource", srcs, out)
    assert best["chunk"] in (16, 32, 64) and best["blocks_per_cu"] in (0, 1, 2, 4)
    assert best["rows_per_wave"] in ((0,) if best["persistent"] else (4, 8, 16))
    assert ms > 0
    keys = ("chunk", "persistent", "blocks_per_cu", "rows_per_wave")
    assert W.tune_lookup("multisource", 64, g.m) == {k: best[k] for k in keys}
    lv, _, _ = W.bfs_multisource(g, srcs, chunk=best["chunk"], persistent=best["persistent"],
                                 blocks_per_cu=best["blocks_per_cu"], rows_per_wave=best["rows_per_wave"])
    want = np.stack([oracle.bfs(ro, col, int(s)) for s in srcs])
    np.testing.assert_array_equal(lv.cpu().numpy().view(np.uint32), want)


def test_multisource_errors():
    ro, col = gen.random_graph(100, 400, 3)
    g = W.Graph.from_csr(ro, col)
    with pytest.raises(W.WedgeError):
        W.bfs_multisource(g, np.arange(65, dtype=np.uint32) % 100)
    with pytest.raises(W.WedgeError):
        W.bfs_multisource(g, np.array([100], np.uint32))
    with pytest.raises(W.WedgeError) as e:
        W.bfs_batch(g, np.array([0], np.uint32))
    assert e.value.name == "WEDGE_ERR_UNSUPPORTED"


def test_autotuner_cache_file_survives_the_process(tmp_path, monkeypatch):
    # with WEDGE_TUNE_CACHE set, a tuning run writes its table to the file and a
    # new process finds the winner there without tuning again
    import json
    import subprocess
    import sys
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("WEDGE_TUNE_CACHE", str(path))
    ro, col = gen.rmat(11, 8, seed=67)
    g = W.Graph.from_csr(ro, col)
    srcs = gen.pick_sources(ro, 1, seed=14)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    best, _ = W.tune_bfs(g, "single", srcs, out)
    lines = path.read_text().splitlines()
    assert lines[0] == "wedge-tune-v1" and len(lines) >= 2
    keys = ("chunk", "persistent", "blocks_per_cu", "rows_per_wave")
    code = ("import json, sys; sys.path.insert(0, %r); import paper_1903_07754_amd as W; "
            "print(json.dumps(W.tune_lookup('single', 1, %d)))" % (str(ROOT), g.m))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       env={**os.environ, "WEDGE_TUNE_CACHE": str(path)})
    assert r.returncode == 0, r.stderr
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert got == {k: best[k] for k in keys}
    g.close()

"""The allocation-free BFS entry point (wedge_bfs_noalloc) against wedge_bfs.

wedge_bfs_noalloc runs the same kernels with its workspace in the library's
fixed device scratch. Through the C ABI, on two calls in a row (the second on
a smaller graph, so the scratch holds the first call's larger contents), its
levels and per-iteration records must equal wedge_bfs's exactly, and the
levels must equal the CPU oracle's BFS. The call must leave the graph's
device footprint unchanged (no workspace allocated), and a graph whose
workspace exceeds the scratch is refused before any device work.
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


def _pair(g, src, out_a, out_b, **kw):
    a, sa, ta = W.bfs_noalloc(g, src, out=out_a, trace_cap=g.n + 2, **kw)
    b, sb, tb = W.bfs(g, src, out=out_b, trace_cap=g.n + 2, **kw)
    torch.cuda.synchronize()
    assert sa["iterations"] == sb["iterations"]
    for ra, rb in zip(ta, tb):
        for k in ("iter", "mode", "chunk_edges", "frontier", "active_edges", "marked_chunks"):
            assert ra[k] == rb[k], (k, ra, rb)
    return W.u32(a), W.u32(b)


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_noalloc_equals_bfs_two_calls_second_smaller(kind):
    sizes = [(14, 16), (11, 8)]  # second call on a smaller graph
    for scale, ef in sizes:
        if kind == "rmat":
            ro, col = gen.rmat(scale, ef, seed=21 + scale)
        else:
            ro, col = gen.erdos_renyi(1 << scale, (1 << scale) * ef, seed=21 + scale)
        n = len(ro) - 1
        src = int(gen.pick_sources(ro, 1, seed=5)[0])
        print(f"  [noalloc {kind} scale={scale} n={n} m={len(col)} src={src}]", flush=True)
        g = W.Graph.from_csr(ro, col)
        bytes0 = g.info["device_bytes"]
        out_a = torch.empty(n, dtype=torch.int32, device="cuda")
        out_b = torch.empty(n, dtype=torch.int32, device="cuda")
        ref = oracle.bfs(ro, col, src)
        for gate, chunk in (("threshold", 0), ("wedge", 32), ("full", 0), ("wedge", 1)):
            a, b = _pair(g, src, out_a, out_b, gate=gate, chunk=chunk)
            assert np.array_equal(a, b), (gate, chunk)
            assert np.array_equal(a, ref), (gate, chunk)
        # a noalloc call on a fresh graph allocates no workspace for it
        g2 = W.Graph.from_csr(ro, col)
        before = g2.info["device_bytes"]
        a2, _, _ = W.bfs_noalloc(g2, src, out=out_a)
        torch.cuda.synchronize()
        assert g2.info["device_bytes"] == before
        assert np.array_equal(W.u32(a2), ref)
        assert before == bytes0
        g.close()
        g2.close()


def test_noalloc_keep_ids_and_ragged():
    # original vertex order (no values buffer in the scratch); n not a multiple of 64
    ro, col = gen.erdos_renyi(3001, 3001 * 5, seed=77)
    src = int(gen.pick_sources(ro, 1, seed=3)[0])
    g = W.Graph.from_csr(ro, col, keep_ids=True)
    out_a = torch.empty(3001, dtype=torch.int32, device="cuda")
    out_b = torch.empty(3001, dtype=torch.int32, device="cuda")
    for chunk in (16, 64, 1024):
        a, b = _pair(g, src, out_a, out_b, gate="wedge", chunk=chunk)
        assert np.array_equal(a, b)
        assert np.array_equal(a, oracle.bfs(ro, col, src))
    g.close()


def test_noalloc_refuses_what_needs_memory():
    # a ring of 3M vertices needs 12 bytes per vertex and more: beyond the 32 MiB scratch
    n = 3_000_000
    ro = np.arange(n + 1, dtype=np.uint64)
    col = ((np.arange(n, dtype=np.uint64) + 1) % n).astype(np.uint32)
    g = W.Graph.from_csr(ro, col)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(W.WedgeError) as e:
        W.bfs_noalloc(g, 0, out=out)
    assert e.value.name == "WEDGE_ERR_INVALID_ARG"
    g.close()
    ro, col = gen.rmat(10, 8, seed=2)
    g = W.Graph.from_csr(ro, col)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for kw in ({"gate": "learned"}, {"time_pull": True}, {"persistent": True}):
        with pytest.raises(W.WedgeError) as e:
            W.bfs_noalloc(g, 1, out=out, **kw)
        assert e.value.name == "WEDGE_ERR_UNSUPPORTED", kw
    g.close()

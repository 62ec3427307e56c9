"""GPU parity of the in-place (asynchronous) pull for CC and SSSP.

With WEDGE_RUN_INPLACE the pull gathers sources' values as the iteration
lowers them, so a drop can travel several hops in one iteration (the paper's
multi-hop propagation with coarse groups, Evaluation, Frontier Precision).
The per-iteration frontiers then depend on the schedule, but the fixed point
does not: final labels and distances must equal the oracle's definitions bit
for bit, and the run may take at most as many iterations as the synchronous
pull (iteration k's values are never above the synchronous iteration k's).
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


def check(app, ro, col, w=None, src=0, keep_ids=False):
    if app == "cc":
        g = W.Graph.from_csr(ro, col, symmetrize=True, keep_ids=keep_ids)
        want = oracle.cc(ro, col)
        gro, gcol = oracle.symmetrize(ro, col)
        jac = oracle.pull_engine("cc", gro, gcol, chunk=0).iters
    else:
        g = W.Graph.from_csr(ro, col, w, keep_ids=keep_ids)
        want = oracle.sssp(ro, col, w, src)
        jac = oracle.pull_engine("sssp", ro, col, w, src, chunk=0).iters
    for gate in ("threshold", "full", "wedge"):
        for chunk in ((0, 1, 64) if gate == "wedge" else (0,)):
            print(f"  [{app} inplace n={g.n} m={g.m} gate={gate} chunk={chunk}]", flush=True)
            if app == "cc":
                out, st, tr = W.cc(g, gate=gate, chunk=chunk, inplace=True, trace_cap=g.n + 2)
                ref_out, ref_st, _ = W.cc(g, gate=gate, chunk=chunk)
            else:
                out, st, tr = W.sssp(g, src, gate=gate, chunk=chunk, inplace=True, trace_cap=g.n + 2)
                ref_out, ref_st, _ = W.sssp(g, src, gate=gate, chunk=chunk)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(W.u32(out), want)
            np.testing.assert_array_equal(W.u32(ref_out), want)
            assert ref_st["iterations"] == jac
            assert st["iterations"] <= jac, (st["iterations"], jac)
            assert len(tr) == st["iterations"]
            assert tr[-1]["frontier"] > 0  # the last iteration consumes a non-empty frontier
    g.close()
    return jac


@pytest.mark.parametrize("app", ["cc", "sssp"])
def test_inplace_grid_at_most_synchronous_iterations(app):
    # a high-diameter mesh in the caller's (row-major) order, large enough that
    # a pull over every in-edge runs its waves in several rounds: a drop made by
    # an early wave can travel on within the same iteration
    side = 2048
    ro, col = gen.grid2d(side, side)
    w = gen.edge_weights(ro, col, seed=4)
    if app == "cc":
        g = W.Graph.from_csr(ro, col, symmetrize=True, keep_ids=True)
        want = oracle.cc(ro, col)
    else:
        g = W.Graph.from_csr(ro, col, w, keep_ids=True)
        want = oracle.sssp(ro, col, w, 0)
    print(f"  [{app} grid {side}x{side} inplace vs synchronous]", flush=True)
    run = (lambda **kw: W.cc(g, **kw)) if app == "cc" else (lambda **kw: W.sssp(g, 0, **kw))
    # under the threshold gate most iterations pull a few marked chunks, all
    # of whose waves run at once; pulls over every in-edge run in many rounds
    # of waves, and those are where a drop travels on within the iteration
    t_out, _, _ = run(inplace=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(W.u32(t_out), want)
    a_out, a, _ = run(inplace=True, gate="full")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(W.u32(a_out), want)
    b_out, b, _ = run(gate="full")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(W.u32(b_out), want)
    if app == "cc":
        # synchronous label propagation moves label 0 one hop per iteration:
        # the farthest vertex is 2*(side-1) hops away, plus the final empty check
        assert b["iterations"] == 2 * (side - 1) + 1
    print(f"  iterations: in-place {a['iterations']}, synchronous {b['iterations']}", flush=True)
    # never more iterations than the synchronous pull (how many fewer depends on
    # which waves run before which: it is a property of the schedule)
    assert a["iterations"] <= b["iterations"], (a["iterations"], b["iterations"])
    g.close()


@pytest.mark.parametrize("app", ["cc", "sssp"])
@pytest.mark.parametrize("kind", ["rmat", "er", "grid_relabelled"])
def test_inplace_matches_oracle(app, kind):
    if kind == "rmat":
        ro, col = gen.rmat(13, 16, seed=51)
    elif kind == "er":
        ro, col = gen.erdos_renyi(6001, 30_000, seed=52)
    else:
        ro, col = gen.grid2d(45, 71)
    w = gen.edge_weights(ro, col, seed=4)
    src = int(gen.pick_sources(ro, 1, seed=53)[0])
    check(app, ro, col, w, src)


def test_inplace_refusals():
    ro, col = gen.rmat(10, 8, seed=2)
    w = gen.edge_weights(ro, col, seed=4)
    g = W.Graph.from_csr(ro, col, w)
    for fn in (lambda: W.bfs(g, 1, inplace=True),
               lambda: W.sssp(g, 1, inplace=True, gate="push"),
               lambda: W.sssp(g, 1, inplace=True, gate="hybrid"),
               lambda: W.bfs_multisource(g, [1, 2], inplace=True),
               lambda: W.pagerank(g, 2, 0.85, inplace=True)):
        with pytest.raises(W.WedgeError) as e:
            fn()
        assert e.value.name == "WEDGE_ERR_UNSUPPORTED"
    g.close()

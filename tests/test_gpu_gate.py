"""GPU checks of the learned gate.

The HIP forward pass and gradient of the gate MLP must match the FP64 oracle
(<= 1e-5 relative); training must lower the loss; counterfactual traces must
carry the oracle's per-iteration frontier sizes, A and threshold decisions; and
whatever the gate decides, results must stay bit-exact. Without a model, or
with every feature outside the envelope, the decisions are the threshold
rule's.
"""
import numpy as np
import pytest

import gen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

import paper_1903_07754_amd as W  # noqa: E402
from paper_1903_07754_amd import _binding as B  # noqa: E402


def test_forward_and_gradient_match_oracle():
    m = W.Model.create(seed=3)
    rng = np.random.default_rng(1)
    p = rng.normal(0, 0.3, 1476).astype(np.float32)
    m.params(p)
    x = rng.normal(0, 1, (1000, 8)).astype(np.float32)
    y = m.predict(x)
    ref = mlp.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.abs(y - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    t = rng.normal(0, 1, (1000, 4)).astype(np.float32)
    mask = (rng.random((1000, 4)) < 0.9).astype(np.float32)
    g, loss = m.grad(x, t, mask)
    gref = mlp.grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), mask.astype(np.float64))
    assert np.linalg.norm(g - gref) <= 1e-5 * np.linalg.norm(gref)
    lref = mlp.loss(p.astype(np.float64), x, t, mask)
    assert abs(loss - lref) <= 1e-5 * lref


def test_ensemble_prediction_is_the_member_mean():
    m = W.Model.create(seed=3, members=4)
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.3, 4 * 1476).astype(np.float32)
    m.params(p)
    x = rng.normal(0, 1, (500, 8)).astype(np.float32)
    y = m.predict(x)
    ref = np.mean([mlp.forward(p[e * 1476:(e + 1) * 1476].astype(np.float64), x.astype(np.float64))
                   for e in range(4)], axis=0)
    assert np.abs(y - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def synthetic_samples(n, seed):
    rng = np.random.default_rng(seed)
    S = (B.TraceSample * n)()
    for s in S:
        s.n, s.m = 1 << 20, 1 << 24
        s.app = int(rng.integers(1, 4))
        s.frontier = int(rng.integers(1, 1 << 20))
        s.active = int(rng.integers(1, 1 << 24))
        s.iter = int(rng.integers(0, 30))
        s.prev_us = float(rng.uniform(1, 1000))
        s.prev_mode = int(rng.integers(0, 4))
        a = s.active / s.m
        s.t_us[0] = 400.0
        for j in range(1, 4):
            s.t_us[j] = 20.0 + 4000.0 * a * (1 + 0.1 * j)
    return S


def test_training_lowers_the_loss_and_learns_the_crossover():
    S = synthetic_samples(3000, 2)
    m = W.Model.create(seed=4)
    x = W.features(S)
    t = np.log1p(np.array([list(s.t_us) for s in S], np.float64))
    t = (t - t[:, :1]).astype(np.float32)        # training targets: relative to the full pull
    _, l0 = m.grad(x, t, np.ones_like(t))
    l1 = m.train(S, epochs=1500, lr=3e-3)
    assert l1 < l0 / 20, (l0, l1)
    y = m.predict(x)
    choice = y.argmin(1)
    best = np.array([np.argmin(s.t_us) for s in S])
    assert (choice == best).mean() > 0.9
    assert np.abs(y[:, 0]).mean() < 0.05         # the full pull's own relative target is 0
    lo, hi = m.envelope()
    assert np.all(lo <= x.min(0)) and np.all(hi >= x.max(0))
    assert np.isinf(lo[[4, 6]]).all() and np.isinf(hi[[4, 6]]).all()
    assert np.isfinite(lo[[0, 1, 2, 3, 5, 7]]).all()


@pytest.mark.parametrize("app", ["bfs", "cc", "sssp"])
def test_counterfactual_trace_matches_oracle_iterations(app):
    ro, col = gen.rmat(13, 16, seed=71)
    w = gen.edge_weights(ro, col, seed=2) if app == "sssp" else None
    s = int(gen.pick_sources(ro, 1, seed=3)[0]) if app != "cc" else 0
    if app == "cc":
        g = W.Graph.from_csr(ro, col, symmetrize=True)
        sro, scol = oracle.symmetrize(ro, col)
        ref = oracle.pull_engine("cc", sro, scol, theta_ppm=200_000, chunk=0)
    else:
        g = W.Graph.from_csr(ro, col, w)
        theta = 10_000 if app == "bfs" else 50_000  # the library's SSSP default
        ref = oracle.pull_engine(app, ro, col, w, s, theta_ppm=theta, chunk=0)
    tr = W.trace_counterfactual(g, app, s)
    assert len(tr) == ref.iters
    default_mode = 2 if app == "bfs" else 1
    for k, r in enumerate(tr):
        assert r.iter == k
        assert r.frontier == ref.F[k] and r.active == ref.A[k]
        assert r.threshold_mode == (default_mode if ref.mode[k] else 0)
        assert all(t > 0 for t in r.t_us)
        if k:
            assert r.prev_mode == tr[k - 1].threshold_mode
            assert r.prev_us == pytest.approx(tr[k - 1].t_us[tr[k - 1].threshold_mode])
    # the traversal after tracing is intact: a normal run still matches the oracle
    if app == "bfs":
        np.testing.assert_array_equal(W.u32(W.bfs(g, s)[0]), oracle.bfs(ro, col, s))


@pytest.mark.parametrize("app", ["bfs", "cc", "sssp"])
def test_learned_gate_keeps_results_exact(app):
    ro, col = gen.rmat(13, 16, seed=72)
    w = gen.edge_weights(ro, col, seed=5) if app == "sssp" else None
    s = int(gen.pick_sources(ro, 1, seed=6)[0])
    m = W.Model.create(seed=9, members=2)
    rng = np.random.default_rng(3)
    m.params(rng.normal(0, 1.0, 2 * 1476))       # an arbitrary ensemble: any decision is allowed
    if app == "cc":
        g = W.Graph.from_csr(ro, col, symmetrize=True)
        out, st, tr = W.cc(g, gate="learned", model=m.handle, trace_cap=256)
        want = oracle.cc(ro, col)
    elif app == "bfs":
        g = W.Graph.from_csr(ro, col)
        out, st, tr = W.bfs(g, s, gate="learned", model=m.handle, trace_cap=256)
        want = oracle.bfs(ro, col, s)
    else:
        g = W.Graph.from_csr(ro, col, w)
        out, st, tr = W.sssp(g, s, gate="learned", model=m.handle, trace_cap=256)
        want = oracle.sssp(ro, col, w, s)
    np.testing.assert_array_equal(W.u32(out), want)
    for r in tr:
        assert r["mode"] in (0, 1)
        if r["mode"]:
            assert r["chunk_edges"] in (16, 32, 64)


def test_learned_gate_without_model_or_outside_envelope_is_the_threshold_rule():
    ro, col = gen.rmat(13, 16, seed=73)
    w = gen.edge_weights(ro, col, seed=7)
    s = int(gen.pick_sources(ro, 1, seed=8)[0])
    g = W.Graph.from_csr(ro, col, w)
    _, _, base = W.sssp(g, s, trace_cap=256)
    _, _, none = W.sssp(g, s, gate="learned", model=None, trace_cap=256)
    m = W.Model.create(seed=1)
    m.envelope(np.full(8, 5.0), np.full(8, 6.0))   # no feature ever lies in [5, 6]
    _, _, outside = W.sssp(g, s, gate="learned", model=m.handle, trace_cap=256)
    for other in (none, outside):
        assert [(r["mode"], r["chunk_edges"], r["marked_chunks"]) for r in other] == \
               [(r["mode"], r["chunk_edges"], r["marked_chunks"]) for r in base]


def test_learned_gate_margin_keeps_the_threshold_rule_unless_confident():
    """With a margin no prediction gap can exceed, the learned gate takes every
    threshold decision; with margin 0 the same model decides by its argmin."""
    ro, col = gen.rmat(13, 16, seed=74)
    w = gen.edge_weights(ro, col, seed=9)
    s = int(gen.pick_sources(ro, 1, seed=10)[0])
    g = W.Graph.from_csr(ro, col, w)
    _, _, base = W.sssp(g, s, trace_cap=256)
    m = W.Model.create(seed=4, members=2)
    rng = np.random.default_rng(5)
    m.params(rng.normal(0, 1.0, 2 * 1476))
    m.margin(1e30)
    out, _, held = W.sssp(g, s, gate="learned", model=m.handle, trace_cap=256)
    np.testing.assert_array_equal(W.u32(out), oracle.sssp(ro, col, w, s))
    assert [(r["mode"], r["chunk_edges"], r["marked_chunks"]) for r in held] == \
           [(r["mode"], r["chunk_edges"], r["marked_chunks"]) for r in base]
    m.margin(0.0)
    out, _, free = W.sssp(g, s, gate="learned", model=m.handle, trace_cap=256)
    np.testing.assert_array_equal(W.u32(out), oracle.sssp(ro, col, w, s))
    assert all(r["mode"] == 0 or r["chunk_edges"] in (16, 32, 64) for r in free)


def test_learned_gate_refuses_persistent_launch():
    ro, col = gen.random_graph(200, 1000, 1)
    g = W.Graph.from_csr(ro, col)
    m = W.Model.create(seed=1)
    with pytest.raises(W.WedgeError) as e:
        W.bfs(g, 0, gate="learned", model=m.handle, persistent=True)
    assert e.value.name == "WEDGE_ERR_UNSUPPORTED"

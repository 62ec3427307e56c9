"""Pins of the gate-MLP oracle and host-side checks of the model API (no GPU).

The oracle's gradient is pinned by central finite differences, its forward
pass by torch's CPU Linear/ReLU stack, its Adam step by torch.optim.Adam; the
library's host feature formula must equal the oracle's; model files must
round-trip and corrupt ones must be refused.
"""
import os

import numpy as np
import pytest
import torch

from oracle import mlp
import paper_1903_07754_amd as W
from paper_1903_07754_amd import _binding as B


def rand_params(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.3, mlp.NPARAMS)


def test_param_count():
    assert mlp.NPARAMS == 1476 == B.MLP_PARAMS


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(100 + seed)
    p = rand_params(seed)
    x = rng.normal(0, 1, (7, 8))
    t = rng.normal(0, 1, (7, 4))
    mask = (rng.random((7, 4)) < 0.8).astype(float)
    g = mlp.grad(p, x, t, mask)
    h = 1e-6
    idx = rng.choice(mlp.NPARAMS, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p); e[i] = h
        fd = (mlp.loss(p + e, x, t, mask) - mlp.loss(p - e, x, t, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def torch_net(p):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a) for a in mlp.unpack(p)]
    net = torch.nn.Sequential(torch.nn.Linear(8, 32), torch.nn.ReLU(), torch.nn.Linear(32, 32),
                              torch.nn.ReLU(), torch.nn.Linear(32, 4)).double()
    with torch.no_grad():
        for layer, (w, b) in zip([net[0], net[2], net[4]], [(W1, b1), (W2, b2), (W3, b3)]):
            layer.weight.copy_(w)
            layer.bias.copy_(b)
    return net


def test_forward_matches_torch():
    p = rand_params(5)
    x = np.random.default_rng(6).normal(0, 1, (33, 8))
    want = torch_net(p)(torch.tensor(x)).detach().numpy()
    np.testing.assert_allclose(mlp.forward(p, x), want, rtol=1e-12, atol=1e-12)


def test_adam_matches_torch():
    p = rand_params(7)
    g = np.random.default_rng(8).normal(0, 1, mlp.NPARAMS)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m1 = np.zeros_like(p); m2 = np.zeros_like(p)
    q = p.copy()
    for step in range(1, 4):
        tp.grad = torch.tensor(g * step)
        opt.step()
        q, m1, m2 = mlp.adam_step(q, g * step, m1, m2, step)
    np.testing.assert_allclose(q, tp.detach().numpy(), rtol=1e-10, atol=1e-12)


def test_oracle_features_against_hand_values():
    """The gate's features pinned to values worked out by hand from their
    definitions in the library header (|F|/n, A/m, 1 - exp(-A/ceil(m/16)),
    app/3, log2(m)/32, min(k, 255)/64, log(1 + us)/16, mode/3), on inputs
    chosen so that a plausible misreading changes a value: m = 1000 makes
    ceil(m/16) = 63 differ from m/16 = 62.5; k = 300 tests the clamp at 255;
    prev_us = e - 1 makes log(1 + us) exactly 1 (log(us) would give 0.5413);
    A = 0 and A = m are the ends of the active-edge range."""
    e = 2.718281828459045
    cases = [
        # (frontier, active, n, m, k, prev_us, prev_mode, app) -> expected 8 features
        ((8, 0, 64, 1024, 0, 0.0, 0, 1),
         [0.125, 0.0, 0.0, 1 / 3, 0.3125, 0.0, 0.0, 0.0]),
        # A = 63 = ceil(1000/16): 1 - e^-1
        ((100, 63, 400, 1000, 255, e - 1.0, 1, 2),
         [0.25, 0.063, 0.6321205588285577, 2 / 3, 0.31143075889569023, 3.984375, 0.0625,
          1 / 3]),
        # k beyond the clamp, A = m (A/ceil(m/16) = 1000/63 = 15.873...)
        ((400, 1000, 400, 1000, 300, 0.0, 3, 3),
         [1.0, 1.0, 0.9999998722276757, 1.0, 0.31143075889569023, 3.984375, 0.0, 1.0]),
        # m = 2^20 (log2 m / 32 = 0.625; A/ceil(m/16) = 2^-16, so 1 - exp(-x) =
        # x - x^2/2 + ... = 1.52587890625e-05 - 1.164e-10), prev_us = e^2 - 1 -> 2/16
        ((1, 1, 2, 1 << 20, 64, 6.38905609893065, 2, 1),
         [0.5, 9.5367431640625e-07, 1.5258672647733285e-05, 1 / 3, 0.625, 1.0, 0.125,
          2 / 3]),
    ]
    for args, want in cases:
        got = mlp.features(*args)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15, err_msg=str(args))


def test_library_features_equal_oracle():
    rows = [(1, 1, 2**10, 2**14, 0, 0.0, 0, 1), (500, 123456, 2**20, 2**24, 7, 350.5, 2, 2),
            (2**18, 2**22, 2**18, 2**22, 300, 1e5, 3, 3)]
    S = (B.TraceSample * len(rows))()
    for s, (f, a, n, m, k, pu, pm, app) in zip(S, rows):
        s.frontier, s.active, s.n, s.m, s.iter, s.prev_us, s.prev_mode, s.app = f, a, n, m, k, pu, pm, app
    got = W.features(S)
    want = np.stack([mlp.features(*r) for r in rows]).astype(np.float32)
    np.testing.assert_allclose(got, want, rtol=2e-7, atol=0)


def test_model_file_roundtrip_and_corruption(tmp_path):
    m = W.Model.create(seed=42)
    p = m.params()
    assert p.shape == (1476,) and np.isfinite(p).all() and np.any(p != 0)
    # weights in +-1/sqrt(fan_in), biases zero
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert np.abs(W1).max() <= 1 / np.sqrt(8) and np.abs(W2).max() <= 1 / np.sqrt(32)
    assert not b1.any() and not b2.any() and not b3.any()
    m.envelope(np.arange(8) - 10.0, np.arange(8) + 10.0)
    f = tmp_path / "gate.bin"
    m.save(str(f))
    m2 = W.Model.load(str(f))
    np.testing.assert_array_equal(m2.params(), p)
    np.testing.assert_array_equal(m2.envelope()[0], np.arange(8) - 10.0)
    raw = bytearray(f.read_bytes())
    for pos in (0, 20, 200, len(raw) - 3):
        bad = bytearray(raw); bad[pos] ^= 0x40
        g = tmp_path / f"bad{pos}.bin"
        g.write_bytes(bytes(bad))
        with pytest.raises(W.WedgeError) as e:
            W.Model.load(str(g))
        assert e.value.name == "WEDGE_ERR_MODEL"
    (tmp_path / "short.bin").write_bytes(bytes(raw[:100]))
    with pytest.raises(W.WedgeError) as e:
        W.Model.load(str(tmp_path / "short.bin"))
    assert e.value.name == "WEDGE_ERR_MODEL"
    with pytest.raises(W.WedgeError) as e:
        W.Model.load(str(tmp_path / "missing.bin"))
    assert e.value.name == "WEDGE_ERR_MODEL"
    q = np.linspace(-1, 1, 1476).astype(np.float32)
    np.testing.assert_array_equal(m.params(q), q)
    np.testing.assert_array_equal(m.params(), q)


def fnv1a(data):
    h = 1469598103934665603
    for b in data:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def test_ensemble_create_roundtrip_and_errors(tmp_path):
    single = W.Model.create(seed=5)
    ens = W.Model.create(seed=5, members=3)
    assert ens.members == 3 and single.members == 1
    p = ens.params()
    assert p.shape == (3 * 1476,)
    # member 0 is the single model of the same seed; the others differ
    np.testing.assert_array_equal(p[:1476], single.params())
    assert np.any(p[1476:2952] != p[:1476]) and np.any(p[2952:] != p[1476:2952])
    f = tmp_path / "ens.bin"
    ens.save(str(f))
    back = W.Model.load(str(f))
    assert back.members == 3
    np.testing.assert_array_equal(back.params(), p)
    # a version-2 file (five-word header, one MLP) still loads as one member
    q = np.linspace(-2, 2, 1476).astype(np.float32)
    lo, hi = np.full(8, -1.0, np.float32), np.full(8, 1.0, np.float32)
    body = (b"WEDGEMLP" + np.array([2, 1476, 8, 32, 4], np.uint32).tobytes() + lo.tobytes()
            + hi.tobytes() + q.tobytes())
    v2 = tmp_path / "v2.bin"
    v2.write_bytes(body + np.array([fnv1a(body)], np.uint64).tobytes())
    old = W.Model.load(str(v2))
    assert old.members == 1
    np.testing.assert_array_equal(old.params(), q)
    np.testing.assert_array_equal(old.envelope()[1], hi)
    # argument errors
    for bad in (0, 9):
        with pytest.raises(W.WedgeError) as e:
            W.Model.create(seed=1, members=bad)
        assert e.value.name == "WEDGE_ERR_INVALID_ARG"
    buf = np.zeros(1476, np.float32)
    assert B.lib().wedge_model_params(ens.handle, buf.ctypes.data, 1476, 0) != B.OK
    # gradients are refused for ensembles before any device work
    x = np.zeros((4, 8), np.float32)
    t = np.zeros((4, 4), np.float32)
    mk = np.ones((4, 4), np.float32)
    g = np.zeros(1476, np.float32)
    st = B.lib().wedge_model_grad(ens.handle, x.ctypes.data, t.ctypes.data, mk.ctypes.data, 4,
                                  g.ctypes.data, None, None)
    assert B.STATUS[st] == "WEDGE_ERR_UNSUPPORTED"


def test_model_margin_roundtrip_versions_and_errors(tmp_path):
    m = W.Model.create(seed=11, members=2)
    assert m.margin() == 0.0
    assert m.margin(0.375) == pytest.approx(0.375)
    f = tmp_path / "m.bin"
    m.save(str(f))
    back = W.Model.load(str(f))
    assert back.margin() == pytest.approx(0.375) and back.members == 2
    np.testing.assert_array_equal(back.params(), m.params())
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(W.WedgeError) as e:
            m.margin(bad)
        assert e.value.name == "WEDGE_ERR_INVALID_ARG"
    # a version-3 file (six-word header: no margin) loads with margin 0
    q = np.linspace(-1, 1, 2 * 1476).astype(np.float32)
    lo, hi = np.full(8, -2.0, np.float32), np.full(8, 2.0, np.float32)
    body = (b"WEDGEMLP" + np.array([3, 1476, 8, 32, 4, 2], np.uint32).tobytes() + lo.tobytes()
            + hi.tobytes() + q.tobytes())
    v3 = tmp_path / "v3.bin"
    v3.write_bytes(body + np.array([fnv1a(body)], np.uint64).tobytes())
    old = W.Model.load(str(v3))
    assert old.margin() == 0.0 and old.members == 2
    np.testing.assert_array_equal(old.params(), q)
    # a version-4 file whose margin is negative is refused
    neg = np.array([-1.0], np.float32).view(np.uint32)[0]
    body = (b"WEDGEMLP" + np.array([4, 1476, 8, 32, 4, 2, neg], np.uint32).tobytes() + lo.tobytes()
            + hi.tobytes() + q.tobytes())
    v4 = tmp_path / "neg.bin"
    v4.write_bytes(body + np.array([fnv1a(body)], np.uint64).tobytes())
    with pytest.raises(W.WedgeError) as e:
        W.Model.load(str(v4))
    assert e.value.name == "WEDGE_ERR_MODEL"


class _StubModel:
    """Fixed predictions, an envelope and a margin: the decision rule alone."""

    def __init__(self, y, margin, lo=None, hi=None):
        self.y, self.m = np.asarray(y, np.float32), margin
        self.lo = np.full(8, -np.inf, np.float32) if lo is None else lo
        self.hi = np.full(8, np.inf, np.float32) if hi is None else hi

    def predict(self, x):
        return self.y

    def envelope(self):
        return self.lo, self.hi

    def margin(self):
        return self.m


def test_host_decision_rule_matches_the_device_rule():
    """learned_gate.choices: the model's argmin replaces the threshold rule's
    mode only when its predicted log-time is lower by more than the margin
    (ties to the lower index), and outside the envelope the rule decides."""
    from paper_1903_07754_amd import learned_gate as LG
    rows = [  # (predictions for modes 0..3, threshold mode, expected pick at margin 0.4)
        ([0.0, -1.0, 0.5, 0.5], 0, 1),     # gain 1.0 > 0.4: departs
        ([0.0, -0.3, 0.5, 0.5], 0, 0),     # gain 0.3: keeps the rule
        ([0.0, -0.4, 0.5, 0.5], 0, 0),     # gain exactly the margin: keeps the rule
        ([0.2, -0.5, -0.5, 0.1], 0, 1),    # tie between 1 and 2: the lower index
        ([0.0, 0.1, -0.2, 0.3], 2, 2),     # the rule's mode is the argmin
        ([-0.6, 0.0, 0.1, 0.2], 1, 0),     # to the full pull
    ]
    S = (B.TraceSample * len(rows))()
    for s, (_, thr, _) in zip(S, rows):
        s.frontier, s.active, s.n, s.m, s.iter, s.app, s.threshold_mode = 10, 100, 1 << 12, 1 << 16, 1, 1, thr
    y = [r[0] for r in rows]
    pick, inside = LG.choices(_StubModel(y, 0.4), S)
    assert inside.all()
    assert list(pick) == [r[2] for r in rows]
    pick0, _ = LG.choices(_StubModel(y, 0.0), S)
    assert list(pick0) == [1, 1, 1, 1, 2, 0]
    # outside the envelope every decision is the rule's
    lo = np.full(8, 5.0, np.float32)
    pick_out, inside = LG.choices(_StubModel(y, 0.0, lo=lo, hi=lo + 1), S)
    assert not inside.any() and list(pick_out) == [r[1] for r in rows]

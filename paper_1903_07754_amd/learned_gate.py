"""Learned fullness gate: trace collection, training and evaluation.

The model is trained on per-iteration timing traces that the method itself
produces (the per-iteration profiling of the paper's Evaluation, Frontier
Fullness Threshold): for every iteration of BFS, CC and SSSP on a corpus of
seeded R-MAT and Erdos-Renyi graphs of scales 18-22, the library times the
iteration in all four modes (full pull; Wedge Frontier at 16, 32, 64 edges per
bit) from the same state. Training and inference run in the library's HIP
kernels; this module only drives them. The gate departs from the threshold
rule only where the model predicts a gain above a decision margin, chosen by
training on the corpus scales up to 20 and measuring regret at scale 22 (the
same two-scale gap as from the corpus to the evaluation graphs). Evaluation uses held-out scale-24
graphs: regret against the per-iteration best mode, and end-to-end GTEPS of
real runs under the learned gate and under the threshold rule.

    python -m paper_1903_07754_amd.learned_gate collect --out traces.npz
    python -m paper_1903_07754_amd.learned_gate train --traces traces.npz --out gate.bin
    python -m paper_1903_07754_amd.learned_gate evaluate --model gate.bin --out eval.json
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

import gen  # noqa: E402

from . import _binding as B  # noqa: E402

DEFAULT_MODEL = os.path.join(HERE, "models", "gate.bin")
DEFAULT_TRACES = os.path.join(HERE, "models", "gate_traces.npz")
APPS = ("bfs", "cc", "sssp")
FIELDS = ("app", "iter", "prev_mode", "threshold_mode", "n", "m", "frontier", "active", "prev_us")


def log(msg):
    print(f"[gate] {msg}", flush=True)


def corpus_graph(i, first_seed=1000):
    """Graph i of the training corpus: alternately R-MAT and ER, scale 18 + (i mod 5)."""
    seed = first_seed + i
    scale = 18 + (i % 5)
    ro, col = gen.rmat(scale, 16, seed=seed)
    kind = "rmat"
    if i % 2 == 1:
        ro, col = gen.erdos_renyi(1 << scale, len(col), seed=seed)
        kind = "er"
    return kind, scale, seed, ro, col


def trace_graph(ro, col, seed, apps=APPS):
    w = gen.edge_weights(ro, col, seed=4)
    src = int(gen.pick_sources(ro, 1, seed=seed)[0])
    out = []
    g = B.Graph.from_csr(ro, col, w)
    for app in apps:
        if app == "cc":
            continue
        out.append(B.trace_counterfactual(g, app, src))
    g.close()
    if "cc" in apps:
        gs = B.Graph.from_csr(ro, col, symmetrize=True)
        out.append(B.trace_counterfactual(gs, "cc", 0))
        gs.close()
    return out


def concat(chunks):
    total = sum(len(c) for c in chunks)
    arr = (B.TraceSample * total)()
    off = 0
    for c in chunks:
        C.memmove(C.byref(arr, off * C.sizeof(B.TraceSample)), c, C.sizeof(B.TraceSample) * len(c))
        off += len(c)
    return arr


def to_arrays(samples):
    d = {f: np.array([getattr(s, f) for s in samples]) for f in FIELDS}
    d["t_us"] = np.array([list(s.t_us) for s in samples], np.float32)
    return d


def from_arrays(d):
    n = len(d["t_us"])
    arr = (B.TraceSample * n)()
    for i, s in enumerate(arr):
        for f in FIELDS:
            setattr(s, f, d[f][i].item())
        for j in range(4):
            s.t_us[j] = float(d["t_us"][i][j])
    return arr


def collect(count=200, first_seed=1000, apps=APPS):
    chunks = []
    t0 = time.time()
    for i in range(count):
        kind, scale, seed, ro, col = corpus_graph(i, first_seed)
        got = trace_graph(ro, col, seed, apps)
        chunks.extend(got)
        log(f"graph {i + 1}/{count} {kind} s{scale}: {sum(len(c) for c in got)} iterations "
            f"({time.time() - t0:.0f}s)")
    return concat(chunks)


def choices(model, samples, margin=None):
    """Mode index the learned gate picks per sample, as the device does: the
    threshold rule's choice outside the envelope, and inside it unless the
    model's argmin is predicted faster than that choice by more than the
    margin (the model's own unless given)."""
    x = B.features(samples)
    y = model.predict(x)
    lo, hi = model.envelope()
    inside = np.all((x >= lo) & (x <= hi), axis=1)
    thr = np.array([s.threshold_mode for s in samples])
    margin = model.margin() if margin is None else margin
    jb = y.argmin(1)
    rows = np.arange(len(thr))
    deviate = inside & (jb != thr) & (y[rows, thr] - y[rows, jb] > margin)
    return np.where(deviate, jb, thr), inside


def fixed_modes(samples):
    """Mode indices of the two fixed policies: every iteration full (0), and
    every iteration Wedge at the application's default group size (32 edges
    for BFS = mode 2, 16 for CC and SSSP = mode 1)."""
    app = np.array([s.app for s in samples])
    return np.zeros(len(app), int), np.where(app == 1, 2, 1)


def regret(samples, pick):
    t = np.array([list(s.t_us) for s in samples], np.float64)
    best = t.min(1)
    chosen = t[np.arange(len(t)), pick]
    return {"total_us": float(chosen.sum()), "regret_us": float((chosen - best).sum()),
            "best_total_us": float(best.sum())}


def train(samples, epochs=3000, lr=3e-3, seed=7, members=6):
    """Train an ensemble of `members` MLPs (independent initialisations and
    training runs); the gate uses the mean of their predictions. Single
    models trained from different seeds disagree widely on graphs larger than
    the training scales; their mean is far more stable."""
    m = B.Model.create(seed=seed, members=members)
    loss = m.train(samples, epochs=epochs, lr=lr)
    return m, loss


MARGINS = (0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.8, 1.0)


def subset(samples, idx):
    return (B.TraceSample * len(idx))(*[samples[int(i)] for i in idx])


def select_margin(samples, epochs=3000, lr=3e-3, seed=7, members=6):
    """Decision margin for extrapolating two scales beyond the corpus: train on
    the corpus scales up to the largest minus two, and take the margin with the
    lowest regret on the largest scale (the gate then serves graphs two scales
    beyond its training scales, the gap from scale 22 to the scale-24 graphs)."""
    scale = np.round(np.log2([s.n for s in samples])).astype(int)
    top = int(scale.max())
    fit, val = np.where(scale <= top - 2)[0], np.where(scale == top)[0]
    if len(fit) == 0 or len(val) == 0:
        return 0.0, {}
    m, _ = train(subset(samples, fit), epochs, lr, seed, members)
    vs = subset(samples, val)
    thr = np.array([s.threshold_mode for s in vs])
    table = {"threshold": regret(vs, thr)["regret_us"]}
    for mg in MARGINS:
        table[mg] = regret(vs, choices(m, vs, mg)[0])["regret_us"]
    best = min(MARGINS, key=lambda mg: (table[mg], mg))
    log(f"margin selection (fit on scales <= {top - 2}, regret on scale {top}): "
        + ", ".join(f"{k}: {v / 1e3:.1f} ms" for k, v in table.items()) + f" -> {best}")
    m.close()
    return best, table


def eval_graphs(seeds=(2000, 2001, 2002, 2003), scale=24):
    for i, seed in enumerate(seeds):
        ro, col = gen.rmat(scale, 16, seed=seed)
        kind = "rmat"
        if i % 2 == 1:
            ro, col = gen.erdos_renyi(1 << scale, len(col), seed=seed)
            kind = "er"
        yield kind, seed, ro, col


GATES = ("threshold", "learned", "wedge", "full")


def end_to_end(model, ro, col, seed, reps=3):
    """Best-of-reps wall time (ms) per app under the threshold rule, the learned
    gate, and the two fixed policies (every iteration Wedge / every iteration
    full); the learned runs include their inference cost."""
    import torch
    w = gen.edge_weights(ro, col, seed=4)
    src = int(gen.pick_sources(ro, 1, seed=seed)[0])
    g = B.Graph.from_csr(ro, col, w)
    gs = B.Graph.from_csr(ro, col, symmetrize=True)
    n = len(ro) - 1
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    res = {}
    for app in APPS:
        times = {}
        for gate in GATES:
            kw = {"gate": gate, "model": model.handle if gate == "learned" else None}
            best = 1e30
            for _ in range(reps):
                if app == "bfs":
                    _, st, _ = B.bfs(g, src, out=out, **kw)
                elif app == "sssp":
                    _, st, _ = B.sssp(g, src, out=out, **kw)
                else:
                    _, st, _ = B.cc(gs, out=out, **kw)
                best = min(best, st["ms"])
            times[gate] = best
        res[app] = times
    g.close()
    gs.close()
    return res


def evaluate(model, seeds=(2000, 2001, 2002, 2003), scale=24, traces_out=None):
    report = {"margin": model.margin(), "graphs": []}
    all_samples = []
    for kind, seed, ro, col in eval_graphs(seeds, scale):
        log(f"evaluating on {kind} s{scale} seed {seed}")
        samples = concat(trace_graph(ro, col, seed))
        all_samples.append(samples)
        pick, inside = choices(model, samples)
        thr = np.array([s.threshold_mode for s in samples])
        e2e = end_to_end(model, ro, col, seed)
        m = len(col)
        report["graphs"].append({
            "kind": kind, "seed": seed, "m": m, "iterations": len(samples),
            "model_decided": float(inside.mean()),
            "threshold": regret(samples, thr), "learned": regret(samples, pick),
            "always_full": regret(samples, fixed_modes(samples)[0]),
            "always_wedge": regret(samples, fixed_modes(samples)[1]),
            "end_to_end_ms": e2e,
            "end_to_end_gteps": {app: {k: round(m / v / 1e6, 3) for k, v in t.items()}
                                 for app, t in e2e.items()}})
    samples = concat(all_samples)
    if traces_out:
        np.savez_compressed(traces_out, **to_arrays(samples))
    pick, inside = choices(model, samples)
    thr = np.array([s.threshold_mode for s in samples])
    report["all"] = {"iterations": len(samples), "model_decided": float(inside.mean()),
                     "threshold": regret(samples, thr), "learned": regret(samples, pick),
                     "always_full": regret(samples, fixed_modes(samples)[0]),
                     "always_wedge": regret(samples, fixed_modes(samples)[1])}
    tot = {g: sum(t[g] for r in report["graphs"] for t in r["end_to_end_ms"].values()) for g in GATES}
    report["all"]["end_to_end_total_ms"] = {g: round(v, 3) for g, v in tot.items()}
    return report


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--count", type=int, default=200)
    c.add_argument("--first-seed", type=int, default=1000)
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--traces", default=DEFAULT_TRACES)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=3000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--seed", type=int, default=7)
    t.add_argument("--members", type=int, default=6)
    t.add_argument("--margin", type=float, default=None,
                   help="decision margin (default: selected by the extrapolation protocol)")
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--out", required=True)
    e.add_argument("--scale", type=int, default=24)
    e.add_argument("--traces-out", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        samples = collect(a.count, a.first_seed)
        np.savez_compressed(a.out, **to_arrays(samples))
        log(f"{len(samples)} samples -> {a.out}")
    elif a.cmd == "train":
        samples = from_arrays(dict(np.load(a.traces)))
        margin = a.margin
        if margin is None:
            margin, _ = select_margin(samples, a.epochs, a.lr, a.seed, a.members)
        m, loss = train(samples, a.epochs, a.lr, a.seed, a.members)
        m.margin(margin)
        m.save(a.out)
        pick, inside = choices(m, samples)
        thr = np.array([s.threshold_mode for s in samples])
        log(f"trained on {len(samples)} samples: final loss {loss:.4f}; training-set regret "
            f"threshold {regret(samples, thr)['regret_us']:.0f} us, "
            f"learned {regret(samples, pick)['regret_us']:.0f} us (margin {margin}) -> {a.out}")
    else:
        model = B.Model.load(a.model)
        rep = evaluate(model, scale=a.scale, traces_out=a.traces_out)
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
        log(json.dumps(rep["all"]))


if __name__ == "__main__":
    main()

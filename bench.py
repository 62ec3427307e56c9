#!/usr/bin/env python3
"""Benchmark of the Wedge-Frontier pull path on one MI355X.

One step = one pass of the whole path over the R-MAT scale-24 workload
(2^24 vertices, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), seeded vertex
relabelling, self-loops and duplicates removed; uint32 weights in [1, 255]):
  BFS from 4 seeded sources, SSSP from the same 4 sources (threshold gate,
  theta BFS 1%, SSSP 5%, CC 20%; 32 / 16 / 16 edges per Wedge bit), CC on the undirected view,
  and PageRank (20 iterations, d = 0.85, full pull).
Inputs are resident in HBM before the timed region. The value is whole-step
GTEPS: (4M + 4M + M + 20M) / step time, M = stored directed edges.

The JSON line also carries the roofline of the dominant kernel (the PageRank
pull, timed with HIP events on the launch stream over the timed steps) and the
CPU oracle timed on a bounded sample of the same workload on this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS per app (BFS/CC/SSSP/PR) R-MAT s24; learned gate vs threshold rule"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha():
    """Hash of the device sources the pull kernels are built from."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_common.h", "wedge_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1903_07754_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current device sources (else None)."""
    safe = kernel.replace("<", "_").replace(">", "")
    p = os.path.join(ROOT, "profiles", f"{safe}_{workload}_counters.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernels_hip_sha") != kernel_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pr_pull_bytes(info):
    """Algorithmic bytes of one PageRank pull launch: the in-edge sources (4/edge),
    the row layout (8 B mask + 4 B segment index per 64 positions, 4 B per
    destination segment), one compulsory 4 B read of contrib per vertex with
    out-edges, one 4 B write of S per destination with in-edges."""
    return (4 * info["m"] + 12 * info["rows"] + 4 * info["nonempty"]
            + 4 * (info["n"] - info["dangling"]) + 4 * info["nonempty"])


def slice_launches(g):
    """Kernel launches per full pull: one per non-empty source slice when the
    graph has the source-sliced in-edge copy, else one."""
    import numpy as np
    if not g.info["xs_rows"]:
        return 1
    b = g.layout("xs_bounds")[:g.info["xs_slices"] + 1].astype(np.int64)
    return int(np.count_nonzero(np.diff(b)))


def pr_kernel_name(g):
    """The PageRank pull the library launches for this graph: one launch per
    source slice over the sliced copy when the graph has one; else the LDS
    variant once every resident wave (2 blocks of 12 waves per compute unit)
    has at least four 8-row tiles, and at least 4096 vertices."""
    import torch
    info = g.info
    if info["xs_rows"]:
        return "k_pr_pull_slice"
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tiles = (info["rows"] + 7) // 8
    hot = info["n"] >= 4096 and tiles >= 4 * cus * 2 * 12
    return "k_pr_pull_hot" if hot else "k_pr_pull"


def full_pull_kernel_name(g, app):
    return f"k_pull_slice<{app}>" if g.info["xs_rows"] else f"k_pull_full<{app}>"


def roofline(name, ms, pulls, alg, workload, per_pull=1, extra=None):
    """HBM roofline entry of one kernel: `pulls` full pulls took `ms` in all
    (HIP events around each pull, on the library's stream); a pull is
    `per_pull` launches of the kernel (the source slices), so one launch
    moves alg / per_pull algorithmic bytes in ms / (pulls * per_pull)."""
    launches = pulls * per_pull
    alg_l = alg / per_pull
    avg = ms / 1e3 / launches
    achieved = alg_l / avg / 1e9
    traffic = measured_traffic(name, workload)
    r = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
         "avg_launch_us": round(avg * 1e6, 2), "launches": launches, "total_ms": round(ms, 3),
         "algorithmic_bytes_per_launch": int(alg_l)}
    if per_pull > 1:
        r["launches_per_pull"] = per_pull
    r.update(extra or {})
    if traffic:
        # the bytes the memory system actually moved (whole lines for 4-byte gathers)
        r["traffic_gbs"] = round(traffic / avg / 1e9, 1)
        r["traffic_frac"] = round(traffic / avg / 1e9 / HBM_PEAK_GBS, 4)
    return r


def minpull_bytes(info, weighted):
    """Algorithmic bytes of one full CC/SSSP pull launch (a lower bound): the
    in-edge sources (4/edge) and weights (4/edge, SSSP), the row layout, one
    4 B read of the current value per destination with in-edges, one
    compulsory 4 B read of the committed value per vertex with out-edges. The
    value and frontier-bit writes depend on the iteration and are not
    counted."""
    return ((8 if weighted else 4) * info["m"] + 12 * info["rows"] + 8 * info["nonempty"]
            + 4 * (info["n"] - info["dangling"]))


def cpu_baseline(ro, col, w, srcs, m):
    """The CPU oracle on a bounded sample of the bench workload, on this host.

    value: the oracle's synchronous full-scan pull engine (the method's own
    iteration semantics, OpenMP over destinations on every host thread; its
    CSC build and per-iteration frontier scan are serial) for BFS from the
    first bench source, plus 2 of the 20 PageRank iterations (FP64, OpenMP),
    on the same R-MAT s24 graph; units M + 2M over the summed time.
    engines: per the measurement plan, the textbook push engine on 1 core
    (BFS at s24) and the pull engine on 1 core and on every thread at s22
    (BFS), each with the threads it used."""
    import gen
    import oracle
    log("timing the CPU oracle on a sample of the workload")
    nthr = oracle.threads()
    t = {}
    t0 = time.perf_counter()
    oracle.pull_engine("bfs", ro, col, None, int(srcs[0]), chunk=0)
    t["bfs_pull_engine"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.pagerank(ro, col, 2, 0.85)
    t["pagerank_2_iters"] = time.perf_counter() - t0
    total = sum(t.values())
    log("oracle seconds: " + ", ".join(f"{k}={v:.2f}" for k, v in t.items()))
    engines = {}
    t0 = time.perf_counter()
    oracle.push_engine("bfs", ro, col, None, int(srcs[0]))
    dt = time.perf_counter() - t0
    engines["push_engine_bfs_rmat24_1core"] = {"s": round(dt, 3), "gteps": round(m / dt / 1e9, 4),
                                               "threads": 1}
    r22, c22 = gen.rmat(22, 16, seed=1)
    s22 = int(gen.pick_sources(r22, 1, seed=3)[0])
    m22 = len(c22)
    for thr in (1, nthr):
        t0 = time.perf_counter()
        oracle.pull_engine("bfs", r22, c22, None, s22, chunk=0, threads=thr)
        dt = time.perf_counter() - t0
        engines[f"pull_engine_bfs_rmat22_{thr}threads"] = {"s": round(dt, 3),
                                                          "gteps": round(m22 / dt / 1e9, 4),
                                                          "threads": thr}
    log("oracle engines: " + ", ".join(f"{k}={v['s']}s" for k, v in engines.items()))
    return {"value": round(3 * m / total / 1e9, 4), "unit": "GTEPS", "cores": nthr,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": ("same R-MAT s24 graph: BFS from 1 source by the oracle's synchronous "
                       "full-scan pull engine and 2 of the 20 PageRank iterations (FP64), both "
                       f"OpenMP on {nthr} threads; units M + 2M over the summed time"),
            "seconds": {k: round(v, 3) for k, v in t.items()}, "engines": engines}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pagerank_only(args):
    """PageRank alone (20 iterations, d = 0.85) on R-MAT at --scale: the
    full-pull roofline at sizes whose other applications would not be worth
    the time (the 67M-vertex, 1.06B-edge scale-26 graph)."""
    import torch

    import gen
    import paper_1903_07754_amd as W

    log(f"generating R-MAT scale {args.scale}")
    ro, col = gen.rmat(args.scale, 16, seed=1)
    n, m = len(ro) - 1, len(col)
    log(f"n={n} m={m}; building the layout")
    g = W.Graph.from_csr(ro, col)
    del ro, col
    rank = torch.empty(n, dtype=torch.float32, device="cuda")
    for i in range(args.warmup):
        W.pagerank(g, 20, 0.85, out=rank)
    torch.cuda.synchronize()
    ms, pull_ms, launches = 0.0, 0.0, 0
    for i in range(args.steps):
        _, st = W.pagerank(g, 20, 0.85, out=rank, time_pull=True)
        ms += st["ms"]
        pull_ms += st["pull_ms"]
        launches += st["pull_launches"]
        log(f"step {i + 1}/{args.steps} done")
    K = args.steps
    roof = roofline(pr_kernel_name(g), pull_ms, launches, pr_pull_bytes(g.info),
                    f"rmat{args.scale}", slice_launches(g))
    out = {"metric": "PageRank GTEPS (20 iterations, full pull) R-MAT s%d" % args.scale,
           "value": round(20 * m * K / (ms / 1e3) / 1e9, 3), "unit": "GTEPS", "n_gpus": 1,
           "steps": K, "warmup": args.warmup, "ms_per_step": round(ms / K, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"R-MAT s{args.scale} ef16 PageRank x20", "n": n, "m": m},
           "roofline": roof}
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {nbytes} bytes")


def timed(fn, reps):
    """Best wall time of `reps` synchronous calls (seconds)."""
    import torch
    best = 1e30
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def learned_section(W, g, gs, srcs, m, outs, reps=2):
    """BFS, SSSP (the bench's sources) and CC on the bench graph under the
    threshold rule and under the learned gate (the committed model, trained on
    scales 18-22 only): best-of-reps wall time per application."""
    import torch
    path = os.path.join(ROOT, "paper_1903_07754_amd", "models", "gate.bin")
    if not os.path.exists(path):
        return None
    model = W.Model.load(path)
    lev, dist, lab = outs
    res = {"model": "paper_1903_07754_amd/models/gate.bin", "unit": "GTEPS (runs*M/t)"}
    for app in ("bfs", "sssp", "cc"):
        row = {}
        for gate in ("threshold", "learned"):
            kw = {"gate": gate, "model": model.handle if gate == "learned" else None}
            if app == "bfs":
                fn = lambda: [W.bfs(g, s, out=lev, **kw) for s in srcs]
            elif app == "sssp":
                fn = lambda: [W.sssp(g, s, out=dist, **kw) for s in srcs]
            else:
                fn = lambda: W.cc(gs, out=lab, **kw)
            runs = 1 if app == "cc" else len(srcs)
            row[gate] = round(runs * m / timed(fn, reps) / 1e9, 3)
        row["learned_over_threshold"] = round(row["learned"] / row["threshold"], 3)
        res[app] = row
    torch.cuda.synchronize()
    model.close()
    return res


def engines_section(W, g, gs, src, m, outs, reps=2):
    """The paper's comparison on this GPU (Fig. 8 and Fig. 9 analogues): BFS and
    SSSP from the first bench source and CC, end to end under the Wedge
    threshold gate, the hybrid baseline (push below 5% of the edges, a pull over
    every in-edge above), the push engine alone and the pull over every in-edge
    alone (best of `reps` runs each); and per-iteration device times of the
    push engine, the full pull and the Wedge pull (translation included) from
    the same frontiers."""
    lev, dist, lab = outs
    res = {"unit": "ms per run (GTEPS = M/t)", "source": int(src)}
    for app in ("bfs", "sssp", "cc"):
        row = {}
        for gate in ("threshold", "hybrid", "push", "full"):
            if app == "bfs":
                fn = lambda: W.bfs(g, src, out=lev, gate=gate)
            elif app == "sssp":
                fn = lambda: W.sssp(g, src, out=dist, gate=gate)
            else:
                fn = lambda: W.cc(gs, out=lab, gate=gate)
            t = timed(fn, reps)
            row[gate] = {"ms": round(t * 1e3, 3), "gteps": round(m / t / 1e9, 3)}
        per_iter = {}
        for gate in ("push", "full", "wedge"):
            if app == "bfs":
                _, st, tr = W.bfs(g, src, out=lev, gate=gate, time_iters=True, trace_cap=4096)
            elif app == "sssp":
                _, st, tr = W.sssp(g, src, out=dist, gate=gate, time_iters=True, trace_cap=4096)
            else:
                _, st, tr = W.cc(gs, out=lab, gate=gate, time_iters=True, trace_cap=4096)
            per_iter[gate] = [round(r["ms"], 4) for r in tr]
            if gate == "push":
                per_iter["active_edges_pct"] = [round(100.0 * r["active_edges"] / (gs.m if app == "cc" else m), 4)
                                                for r in tr]
        wins = sum(1 for a, b in zip(per_iter["wedge"], per_iter["push"]) if a < b)
        row["per_iteration_ms"] = per_iter
        row["iterations_wedge_beats_push"] = f"{wins}/{len(per_iter['push'])}"
        row["threshold_over_hybrid"] = round(row["hybrid"]["ms"] / row["threshold"]["ms"], 3)
        res[app] = row
    return res


def inplace_section(W, g, gs, src, outs, reps=2, grid_side=4096):
    """Synchronous (Jacobi) against in-place (asynchronous) pulls for SSSP and CC
    (threshold gate; and the in-place pull over every in-edge in every
    iteration): on the bench graph, and on a grid_side^2 2-D mesh
    in row-major vertex order (a high-diameter stand-in for a road network,
    the graph class on which the paper saw drops travel several hops per
    iteration). Iterations and best-of-`reps` wall time per run."""
    import torch

    import gen
    lev, dist, lab = outs
    res = {"unit": "ms per run; iterations"}

    def both(name, sssp_g, cc_g, s, dout, lout):
        row = {}
        for app in ("sssp", "cc"):
            r = {}
            for mode, kw in (("jacobi", {}), ("inplace", {"inplace": True}),
                             ("inplace_full_pull", {"inplace": True, "gate": "full"})):
                if app == "sssp":
                    fn = lambda: W.sssp(sssp_g, s, out=dout, **kw)
                else:
                    fn = lambda: W.cc(cc_g, out=lout, **kw)
                _, st, _ = fn()
                r[mode] = {"iterations": st["iterations"], "ms": round(timed(fn, reps) * 1e3, 3)}
            r["speedup"] = round(r["jacobi"]["ms"] / min(r["inplace"]["ms"], r["inplace_full_pull"]["ms"]), 3)
            row[app] = r
        res[name] = row

    both("rmat24", g, gs, src, dist, lab)
    log(f"in-place: {grid_side}x{grid_side} grid")
    ro, col = gen.grid2d(grid_side, grid_side)
    w = gen.edge_weights(ro, col, seed=4)
    n = len(ro) - 1
    gg = W.Graph.from_csr(ro, col, w, keep_ids=True)
    ggs = W.Graph.from_csr(ro, col, symmetrize=True, keep_ids=True)
    d2 = torch.empty(n, dtype=torch.int32, device="cuda")
    l2 = torch.empty(n, dtype=torch.int32, device="cuda")
    both(f"grid{grid_side}x{grid_side}", gg, ggs, 0, d2, l2)
    res[f"grid{grid_side}x{grid_side}"]["n"] = n
    res[f"grid{grid_side}x{grid_side}"]["m"] = int(len(col))
    gg.close()
    ggs.close()
    return res


def configs_section(m_rmat24, steps=10):
    """The other configurations of the measurement plan, outside the headline:
    config 1 (R-MAT s16, BFS from 8 sources: median of `steps` runs after 2
    warm-ups per source), config 2's Erdos-Renyi graph (G(2^24, M of the R-MAT
    s24 graph), BFS and SSSP from 4 sources, CC; best of 2), and config 3
    (PageRank, 20 iterations, on R-MAT s26, with the pull's roofline)."""
    import numpy as np
    import torch

    import gen
    import paper_1903_07754_amd as W
    res = {}
    log("configs: R-MAT s16 BFS from 8 sources")
    ro, col = gen.rmat(16, 16, seed=1)
    srcs = [int(x) for x in gen.pick_sources(ro, 8, seed=2)]
    g = W.Graph.from_csr(ro, col)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    meds = []
    for sv in srcs:
        for _ in range(2):
            W.bfs(g, sv, out=out)
        ts = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            W.bfs(g, sv, out=out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        meds.append(float(np.median(ts)))
    res["config1_rmat16_bfs"] = {
        "n": g.n, "m": g.m, "sources": srcs, "median_ms_per_source": [round(x * 1e3, 4) for x in meds],
        "gteps": round(g.m * len(meds) / sum(meds) / 1e9, 3)}
    g.close()
    del ro, col

    log("configs: Erdos-Renyi G(2^24, m) BFS/SSSP x4, CC")
    ro, col = gen.erdos_renyi(1 << 24, m_rmat24, seed=2)
    w = gen.edge_weights(ro, col, seed=4)
    srcs = [int(x) for x in gen.pick_sources(ro, 4, seed=3)]
    n, m = len(ro) - 1, len(col)
    g = W.Graph.from_csr(ro, col, w)
    gs = W.Graph.from_csr(ro, col, symmetrize=True)
    del ro, col, w
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    row = {"n": n, "m": m, "m_undirected": gs.m, "unit": "ms per run; GTEPS = M/t"}
    for app in ("bfs", "sssp", "cc"):
        if app == "bfs":
            fn = lambda: [W.bfs(g, sv, out=out) for sv in srcs]
        elif app == "sssp":
            fn = lambda: [W.sssp(g, sv, out=out) for sv in srcs]
        else:
            fn = lambda: W.cc(gs, out=out)
        fn()
        runs = 1 if app == "cc" else len(srcs)
        t = timed(fn, 2) / runs
        row[app] = {"ms": round(t * 1e3, 3), "gteps": round(m / t / 1e9, 3)}
    res["config2_er24"] = row
    g.close()
    gs.close()

    log("configs: PageRank on R-MAT s26")
    ro, col = gen.rmat(26, 16, seed=1)
    n, m = len(ro) - 1, len(col)
    g = W.Graph.from_csr(ro, col)
    del ro, col
    rank = torch.empty(n, dtype=torch.float32, device="cuda")
    W.pagerank(g, 20, 0.85, out=rank)
    ms, pull_ms, launches = 0.0, 0.0, 0
    for _ in range(2):
        _, st = W.pagerank(g, 20, 0.85, out=rank, time_pull=True)
        ms += st["ms"]
        pull_ms += st["pull_ms"]
        launches += st["pull_launches"]
    roof = roofline(pr_kernel_name(g), pull_ms, launches, pr_pull_bytes(g.info), "rmat26",
                    slice_launches(g))
    res["config3_pagerank_rmat26"] = {"n": n, "m": m, "ms_per_run": round(ms / 2, 3),
                                      "gteps": round(20 * m * 2 / (ms / 1e3) / 1e9, 3),
                                      "roofline": roof}
    g.close()
    return res


def batched_section(reps=3):
    """Batched BFS against the plain threshold-gated single-query path on the
    same GPU: 64 sources on R-MAT scale 22 as 64-bit masks in one traversal,
    and 256 R-MAT graphs of scales drawn from 10..16 as one disjoint union.
    Both batched forms are timed host-driven, as one persistent launch
    replayed from a captured hipGraph, and in the autotuned configuration
    (chunk size, host-driven or persistent launch, blocks per CU, rows per wave)."""
    import numpy as np
    import torch

    import gen
    import paper_1903_07754_amd as W

    res = {}
    ro, col = gen.rmat(22, 16, seed=5)
    srcs = gen.pick_sources(ro, 64, seed=6)
    n, m = len(ro) - 1, len(col)
    g = W.Graph.from_csr(ro, col)
    out1 = torch.empty(n, dtype=torch.int32, device="cuda")
    outk = torch.empty(64 * n, dtype=torch.int32, device="cuda")
    log("batched: 64 sources on R-MAT s22")
    t_seq = timed(lambda: [W.bfs(g, int(s), out=out1) for s in srcs], reps)
    t_ms = timed(lambda: W.bfs_multisource(g, srcs, out=outk), reps)
    best, _ = W.tune_bfs(g, "multisource", srcs, outk)
    t_tuned = timed(lambda: W.bfs_multisource(g, srcs, out=outk, chunk=best["chunk"],
                                              persistent=best["persistent"],
                                              blocks_per_cu=best["blocks_per_cu"],
                                              rows_per_wave=best["rows_per_wave"]), reps)
    t_pers = timed(lambda: W.bfs_multisource(g, srcs, out=outk, persistent=True), reps)
    lv = outk.view(64, n)
    for i in (0, 31, 63):
        W.bfs(g, int(srcs[i]), out=out1)
        assert torch.equal(lv[i], out1), "multi-source row differs from the single-source run"
    res["multisource_s22"] = {
        "n": n, "m": m, "sources": 64, "unit": "GTEPS (64*M/t)",
        "single_query_threshold_ms": round(t_seq * 1e3, 3),
        "single_query_threshold_gteps": round(64 * m / t_seq / 1e9, 2),
        "batched_host_loop_ms": round(t_ms * 1e3, 3),
        "batched_persistent_graph_ms": round(t_pers * 1e3, 3),
        "batched_tuned_ms": round(t_tuned * 1e3, 3),
        "batched_tuned_gteps": round(64 * m / t_tuned / 1e9, 2),
        "tuned": best, "speedup_vs_single_query": round(t_seq / t_tuned, 2)}
    del g, lv, outk
    log("batched: 256 R-MAT graphs of scales 10..16")
    scales = gen.batch_scales(256, 10, 16, seed=7)
    parts = [gen.rmat(s, 16, seed=3000 + i) for i, s in enumerate(scales)]
    bsrcs = np.array([int(gen.pick_sources(r, 1, seed=4000 + i)[0]) for i, (r, _) in enumerate(parts)],
                     np.uint32)
    mtot = sum(len(c) for _, c in parts)
    gb = W.Graph.from_batch_csr(parts)
    singles = [W.Graph.from_csr(r, c) for r, c in parts]
    outs = [torch.empty(len(r) - 1, dtype=torch.int32, device="cuda") for r, _ in parts]
    outb = torch.empty(gb.n, dtype=torch.int32, device="cuda")
    t_seq = timed(lambda: [W.bfs(sg, int(s), out=o) for sg, s, o in zip(singles, bsrcs, outs)], reps)
    t_b = timed(lambda: W.bfs_batch(gb, bsrcs, out=outb), reps)
    t_bp = timed(lambda: W.bfs_batch(gb, bsrcs, out=outb, persistent=True), reps)
    best, _ = W.tune_bfs(gb, "batch", bsrcs, outb)
    t_tuned = timed(lambda: W.bfs_batch(gb, bsrcs, out=outb, chunk=best["chunk"],
                                        persistent=best["persistent"],
                                        blocks_per_cu=best["blocks_per_cu"],
                                        rows_per_wave=best["rows_per_wave"]), reps)
    first = gb.parts()
    for i in (0, 100, 255):
        assert torch.equal(outb[int(first[i]):int(first[i + 1])], outs[i]), "batch part differs"
    res["batch256_s10_16"] = {
        "graphs": 256, "n": gb.n, "m": mtot, "unit": "GTEPS (sum M_g / t)",
        "single_query_threshold_ms": round(t_seq * 1e3, 3),
        "single_query_threshold_gteps": round(mtot / t_seq / 1e9, 2),
        "batched_host_loop_ms": round(t_b * 1e3, 3),
        "batched_persistent_graph_ms": round(t_bp * 1e3, 3),
        "batched_tuned_ms": round(t_tuned * 1e3, 3),
        "batched_tuned_gteps": round(mtot / t_tuned / 1e9, 2),
        "tuned": best, "speedup_vs_single_query": round(t_seq / t_tuned, 2)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--sources", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-engines", action="store_true")
    ap.add_argument("--no-inplace", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip config 1 (s16), the ER s24 graph and PageRank on R-MAT s26")
    ap.add_argument("--pagerank-only", action="store_true",
                    help="time only the PageRank leg (used for the scale-26 roofline)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB 3 times (a known-size "
                         "kernel for calibrating HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.pagerank_only:
        pagerank_only(args)
        return

    import numpy as np
    import torch

    import gen
    import paper_1903_07754_amd as W

    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    log(f"device {dev_name}; generating R-MAT scale {args.scale}")
    t0 = time.perf_counter()
    ro, col = gen.rmat(args.scale, 16, seed=1)
    w = gen.edge_weights(ro, col, seed=4)
    srcs = [int(s) for s in gen.pick_sources(ro, args.sources, seed=3)]
    n, m = len(ro) - 1, len(col)
    log(f"n={n} m={m} generated in {time.perf_counter() - t0:.1f}s; building layouts")
    t0 = time.perf_counter()
    g = W.Graph.from_csr(ro, col, w)
    gs = W.Graph.from_csr(ro, col, symmetrize=True)
    log(f"layouts built and uploaded in {time.perf_counter() - t0:.1f}s "
        f"(directed {g.info['device_bytes'] / 2**30:.2f} GiB, undirected m={gs.m})")

    lev = torch.empty(n, dtype=torch.int32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    dist = torch.empty(n, dtype=torch.int32, device="cuda")
    rank = torch.empty(n, dtype=torch.float32, device="cuda")
    app_s = {"bfs": 0.0, "sssp": 0.0, "cc": 0.0, "pr": 0.0}
    pull = {"ms": 0.0, "launches": 0}
    fullpull = {"sssp": [0.0, 0], "cc": [0.0, 0]}

    def step(timed):
        for s in srcs:
            t = time.perf_counter(); W.bfs(g, s, out=lev); dt = time.perf_counter() - t
            if timed: app_s["bfs"] += dt
        for s in srcs:
            t = time.perf_counter(); _, st, _ = W.sssp(g, s, out=dist, time_pull=True)
            dt = time.perf_counter() - t
            if timed:
                app_s["sssp"] += dt
                fullpull["sssp"][0] += st["full_pull_ms"]
                fullpull["sssp"][1] += st["full_pull_launches"]
        t = time.perf_counter(); _, st, _ = W.cc(gs, out=lab, time_pull=True)
        dt = time.perf_counter() - t
        if timed:
            app_s["cc"] += dt
            fullpull["cc"][0] += st["full_pull_ms"]
            fullpull["cc"][1] += st["full_pull_launches"]
        t = time.perf_counter()
        _, st = W.pagerank(g, 20, 0.85, out=rank, time_pull=True)
        dt = time.perf_counter() - t
        if timed:
            app_s["pr"] += dt
            pull["ms"] += st["pull_ms"]
            pull["launches"] += st["pull_launches"]

    for i in range(args.warmup):
        step(False)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    K = args.steps
    units = (2 * len(srcs) + 1 + 20) * m
    value = units * K / elapsed / 1e9
    per_app = {
        "bfs": round(len(srcs) * m * K / app_s["bfs"] / 1e9, 3),
        "sssp": round(len(srcs) * m * K / app_s["sssp"] / 1e9, 3),
        "cc": round(m * K / app_s["cc"] / 1e9, 3),
        "pr": round(20 * m * K / app_s["pr"] / 1e9, 3),
    }
    per_app_ms = {k: round(v * 1e3 / K / (len(srcs) if k in ("bfs", "sssp") else 1), 3)
                  for k, v in app_s.items()}
    workload = f"rmat{args.scale}"
    cands = [
        (pr_kernel_name(g), pull["ms"], pull["launches"], pr_pull_bytes(g.info), slice_launches(g)),
        (full_pull_kernel_name(g, "SSSP"), fullpull["sssp"][0], fullpull["sssp"][1],
         minpull_bytes(g.info, True), slice_launches(g)),
        (full_pull_kernel_name(gs, "CC"), fullpull["cc"][0], fullpull["cc"][1],
         minpull_bytes(gs.info, False), slice_launches(gs)),
    ]
    roofs = []
    for name, ms, pulls, alg, per in cands:
        if not pulls:
            continue
        extra = None
        if name.startswith("k_pull_slice<SSSP") and g.info["xs_packed"]:
            # the packed copy reads one 4-byte word per in-edge where the
            # algorithmic figure counts a source and a weight (8 bytes)
            packed = alg - 4 * g.info["m"]
            extra = {"packed_edge_words": True,
                     "packed_bytes_per_launch": int(packed / per),
                     "packed_frac": round(packed / per / (ms / 1e3 / (pulls * per)) / 1e9 / HBM_PEAK_GBS, 4)}
        roofs.append(roofline(name, ms, pulls, alg, workload, per, extra))
    roofs.sort(key=lambda r: -r["total_ms"])  # the dominant kernel first
    roof = roofs[0]
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / K, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32/f32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT s{args.scale} ef16 (a,b,c,d)=(.57,.19,.19,.05): "
                               f"BFS x{len(srcs)} + SSSP x{len(srcs)} + CC + PageRank x20",
                   "n": n, "m": m, "m_undirected": gs.m, "gate": "threshold",
                   "theta_ppm": {"bfs": 10000, "cc": 200000, "sssp": 50000},
                   "chunk_edges": {"bfs": 32, "cc": 16, "sssp": 16}, "device": dev_name},
        "per_app_gteps": per_app, "per_app_ms": per_app_ms,
        "roofline": roof,
        "roofline_others": roofs[1:],
    }
    if not args.no_engines:
        log("engines: Wedge pull vs hybrid vs push vs full pull")
        out["engines"] = engines_section(W, g, gs, srcs[0], m, (lev, dist, lab))
    if not args.no_inplace:
        log("in-place vs synchronous pulls")
        out["inplace"] = inplace_section(W, g, gs, srcs[0], (lev, dist, lab))
    if not args.no_learned:
        log("learned gate vs threshold rule on the bench graph")
        out["learned_gate"] = learned_section(W, g, gs, srcs, m, (lev, dist, lab))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ro, col, w, srcs, m)
    if not args.no_batched or not args.no_configs:
        del g, gs, lev, lab, dist, rank
    if not args.no_batched:
        out["batched"] = batched_section()
    if not args.no_configs:
        out["configs"] = configs_section(m)
    print(json.dumps(out), flush=True)
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {nbytes} bytes")


if __name__ == "__main__":
    main()

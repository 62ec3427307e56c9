#!/usr/bin/env python3
"""Benchmark of the Wedge-Frontier pull path on one MI355X.

One step = one pass of the whole path over the R-MAT scale-24 workload
(2^24 vertices, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), seeded vertex
relabelling, self-loops and duplicates removed; uint32 weights in [1, 255]):
  BFS from 4 seeded sources, SSSP from the same 4 sources (threshold gate,
  theta 1% / 20%, 32 / 16 edges per Wedge bit), CC on the undirected view,
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


def pr_kernel_name(info):
    """The PageRank pull the library launches for this graph: the LDS variant
    once every resident wave (2 blocks of 12 waves per compute unit) has at
    least four 8-row tiles, and at least 4096 vertices."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tiles = (info["rows"] + 7) // 8
    hot = info["n"] >= 4096 and tiles >= 4 * cus * 2 * 12
    return "k_pr_pull_hot" if hot else "k_pr_pull"


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
    import oracle
    log("timing the CPU oracle on a sample of the workload")
    t = {}
    t0 = time.perf_counter(); oracle.bfs(ro, col, int(srcs[0])); t["bfs"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.cc(ro, col); t["cc"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.sssp(ro, col, w, int(srcs[0])); t["sssp"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.pagerank(ro, col, 2, 0.85); t["pr"] = time.perf_counter() - t0
    units = m + m + m + 2 * m
    total = sum(t.values())
    log("oracle seconds: " + ", ".join(f"{k}={v:.2f}" for k, v in t.items()))
    return {"value": round(units / total / 1e9, 4), "unit": "GTEPS", "cores": oracle.threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": ("same R-MAT s24 graph: BFS and SSSP from 1 source (sequential queue BFS, "
                       "Dial/Dijkstra), CC by union-find (sequential), PageRank 2 of 20 iterations "
                       "(FP64, OpenMP over destinations); units M+M+M+2M over the summed time"),
            "seconds": {k: round(v, 3) for k, v in t.items()}}


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
    avg_launch_s = pull_ms / 1e3 / launches
    alg = pr_pull_bytes(g.info)
    name = pr_kernel_name(g.info)
    workload = f"rmat{args.scale}"
    traffic = measured_traffic(name, workload)
    roof = {"kernel": name, "bound": "hbm", "achieved": round(alg / avg_launch_s / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(alg / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": traffic,
            "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": launches,
            "algorithmic_bytes_per_launch": int(alg)}
    if traffic:
        roof["traffic_gbs"] = round(traffic / avg_launch_s / 1e9, 1)
        roof["traffic_frac"] = round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
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
        (pr_kernel_name(g.info), pull["ms"], pull["launches"], pr_pull_bytes(g.info)),
        ("k_pull_full<SSSP>", fullpull["sssp"][0], fullpull["sssp"][1], minpull_bytes(g.info, True)),
        ("k_pull_full<CC>", fullpull["cc"][0], fullpull["cc"][1], minpull_bytes(gs.info, False)),
    ]
    roofs = []
    for name, ms, launches, alg in cands:
        if not launches:
            continue
        avg_launch_s = ms / 1e3 / launches
        achieved = alg / avg_launch_s / 1e9
        traffic = measured_traffic(name, workload)
        r = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1),
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
             "traffic": traffic, "avg_launch_us": round(avg_launch_s * 1e6, 2),
             "launches": launches, "total_ms": round(ms, 3),
             "algorithmic_bytes_per_launch": int(alg)}
        if traffic:
            # the bytes the memory system actually moved (whole lines for 4-byte gathers)
            r["traffic_gbs"] = round(traffic / avg_launch_s / 1e9, 1)
            r["traffic_frac"] = round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
        roofs.append(r)
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
                   "theta_ppm": {"bfs": 10000, "cc": 200000, "sssp": 200000},
                   "chunk_edges": {"bfs": 32, "cc": 16, "sssp": 16}, "device": dev_name},
        "per_app_gteps": per_app, "per_app_ms": per_app_ms,
        "roofline": roof,
        "roofline_others": roofs[1:],
    }
    if not args.no_learned:
        log("learned gate vs threshold rule on the bench graph")
        out["learned_gate"] = learned_section(W, g, gs, srcs, m, (lev, dist, lab))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ro, col, w, srcs, m)
    if not args.no_batched:
        del g, gs, lev, lab, dist, rank
        out["batched"] = batched_section()
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

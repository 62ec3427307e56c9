"""Pins of the CPU oracle against what the paper and mathematics fix.

Each check is independent of the oracle's own code path: exhaustive path
search, Floyd-Warshall, transitive closure, scipy's graph routines, numpy's
eigen-solver, hand-derived closed forms, exact rational arithmetic and the
worked example of the paper's Design Requirements section. Together they are
chosen so that a dropped term, a wrong sign or index, or a misaligned weight
array in the oracle fails at least one of them.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import gen
import oracle

INF = oracle.INF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers

def csr_from_pairs(n, pairs):
    src = np.array([p[0] for p in pairs], np.uint32)
    dst = np.array([p[1] for p in pairs], np.uint32)
    return gen.csr_from_edges(n, src, dst)


def edges_of(row_off, col):
    out = []
    for u in range(len(row_off) - 1):
        for j in range(int(row_off[u]), int(row_off[u + 1])):
            out.append((u, int(col[j]), j))
    return out


def brute_paths_levels(n, pairs, s):
    """Fewest edges on a simple directed path, by enumerating every simple path."""
    adj = {u: [v for (a, v) in pairs if a == u] for u in range(n)}
    best = [INF] * n
    best[s] = 0

    def dfs(u, depth, seen):
        for v in adj[u]:
            if v not in seen:
                if depth + 1 < best[v]:
                    best[v] = depth + 1
                dfs(v, depth + 1, seen | {v})

    dfs(s, 0, {s})
    return np.array(best, np.uint32)


def floyd_warshall(n, wedges):
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0)
    for u, v, w in wedges:
        d[u, v] = min(d[u, v], w)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


def to_u32(dist_row):
    return np.array([INF if np.isinf(x) else int(x) for x in dist_row], np.uint32)


def random_small(n, m, seed):
    return gen.random_graph(n, m, seed)


# ---------------------------------------------------------------------- BFS

def test_bfs_exhaustive_all_graphs_n4():
    """Every directed loop-free graph on 4 vertices, every source."""
    n = 4
    slots = [(u, v) for u in range(n) for v in range(n) if u != v]
    for mask in range(1 << len(slots)):
        pairs = [slots[i] for i in range(len(slots)) if mask >> i & 1]
        ro, col = csr_from_pairs(n, pairs) if pairs else (np.zeros(n + 1, np.uint64), np.zeros(0, np.uint32))
        for s in range(n):
            np.testing.assert_array_equal(oracle.bfs(ro, col, s), brute_paths_levels(n, pairs, s))


@pytest.mark.parametrize("seed", range(12))
def test_bfs_unit_floyd_warshall(seed):
    n = 6 + seed % 7
    ro, col = random_small(n, 2 * n, 100 + seed)
    d = floyd_warshall(n, [(u, v, 1) for u, v, _ in edges_of(ro, col)])
    for s in range(n):
        np.testing.assert_array_equal(oracle.bfs(ro, col, s), to_u32(d[s]))


def test_bfs_matches_scipy_medium():
    ro, col = gen.rmat(12, 8, seed=11)
    n = len(ro) - 1
    a = sp.csr_matrix((np.ones(len(col)), col.astype(np.int64), ro.astype(np.int64)), shape=(n, n))
    for s in gen.pick_sources(ro, 3, seed=5):
        ref = csg.shortest_path(a, unweighted=True, indices=int(s), directed=True)
        np.testing.assert_array_equal(oracle.bfs(ro, col, int(s)), to_u32(ref))


# ----------------------------------------------------------------------- CC

@pytest.mark.parametrize("seed", range(10))
def test_cc_transitive_closure(seed):
    n = 5 + seed
    ro, col = random_small(n, n, 200 + seed)
    reach = np.eye(n, dtype=bool)
    for u, v, _ in edges_of(ro, col):
        reach[u, v] = reach[v, u] = True
    for k in range(n):
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    want = np.array([np.flatnonzero(reach[v]).min() for v in range(n)], np.uint32)
    np.testing.assert_array_equal(oracle.cc(ro, col), want)


def test_cc_matches_scipy_medium():
    ro, col = gen.rmat(12, 2, seed=12)
    n = len(ro) - 1
    a = sp.csr_matrix((np.ones(len(col)), col.astype(np.int64), ro.astype(np.int64)), shape=(n, n))
    _, comp = csg.connected_components(a, directed=True, connection="weak")
    mins = np.full(comp.max() + 1, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    np.testing.assert_array_equal(oracle.cc(ro, col), mins[comp].astype(np.uint32))


def test_symmetrize_is_undirected_view():
    ro, col = random_small(30, 80, 7)
    sro, scol = oracle.symmetrize(ro, col)
    want = set()
    for u, v, _ in edges_of(ro, col):
        if u != v:
            want |= {(u, v), (v, u)}
    got = [(u, v) for u, v, _ in edges_of(sro, scol)]
    assert len(got) == len(set(got)) == len(want) and set(got) == want


# --------------------------------------------------------------------- SSSP

@pytest.mark.parametrize("seed,wmax", [(s, w) for s in range(8) for w in (1, 255, 10**6)])
def test_sssp_floyd_warshall(seed, wmax):
    """wmax <= 4096 runs the bucket queue, 10**6 the binary heap."""
    n = 6 + seed
    ro, col = random_small(n, 3 * n, 300 + seed)
    w = gen.edge_weights(ro, col, seed=seed, lo=1, hi=wmax)
    d = floyd_warshall(n, [(u, v, int(w[j])) for u, v, j in edges_of(ro, col)])
    for s in range(n):
        np.testing.assert_array_equal(oracle.sssp(ro, col, w, s), to_u32(d[s]))


@pytest.mark.parametrize("wmax", [255, 10**6])
def test_sssp_matches_scipy_dijkstra(wmax):
    ro, col = gen.rmat(12, 8, seed=13)
    n = len(ro) - 1
    w = gen.edge_weights(ro, col, seed=4, lo=1, hi=wmax)
    a = sp.csr_matrix((w.astype(np.float64), col.astype(np.int64), ro.astype(np.int64)), shape=(n, n))
    for s in gen.pick_sources(ro, 2, seed=6):
        ref = csg.dijkstra(a, directed=True, indices=int(s))
        np.testing.assert_array_equal(oracle.sssp(ro, col, w, int(s)), to_u32(ref))


# ----------------------------------------------------------------- PageRank

def pr_exact(n, pairs, iters, d):
    """The damped iteration in exact rationals (pins FP64 rounding only)."""
    out = [0] * n
    for u, _ in pairs:
        out[u] += 1
    r = [Fraction(1, n)] * n
    for _ in range(iters):
        dang = sum((r[u] for u in range(n) if out[u] == 0), Fraction(0))
        s = [Fraction(0)] * n
        for u, v in pairs:
            s[v] += r[u] / out[u]
        r = [(1 - d) / n + d * (s[v] + dang / n) for v in range(n)]
    return r


@pytest.mark.parametrize("seed", range(6))
def test_pagerank_exact_rationals(seed):
    n = 5 + seed
    ro, col = random_small(n, n + 2, 400 + seed)   # sparse: leaves dangling vertices
    pairs = [(u, v) for u, v, _ in edges_of(ro, col)]
    ex = pr_exact(n, pairs, 20, Fraction(17, 20))
    got = oracle.pagerank(ro, col, 20, 0.85)
    assert max(abs(float(e) - g) for e, g in zip(ex, got)) <= 1e-14


@pytest.mark.parametrize("n", [3, 7, 64])
def test_pagerank_cycle_and_complete(n):
    cyc = csr_from_pairs(n, [(i, (i + 1) % n) for i in range(n)])
    comp = csr_from_pairs(n, [(u, v) for u in range(n) for v in range(n) if u != v])
    for ro, col in (cyc, comp):
        r = oracle.pagerank(ro, col, 20, 0.85)
        np.testing.assert_allclose(r, 1.0 / n, rtol=0, atol=1e-15)


def test_pagerank_two_vertex_chain_fixed_point():
    """0 -> 1 with 1 dangling: stationary r(0) = 1/(2+d), r(1) = (1+d)/(2+d)."""
    d = 0.85
    ro, col = csr_from_pairs(2, [(0, 1)])
    r = oracle.pagerank(ro, col, 300, d)
    np.testing.assert_allclose(r, [1 / (2 + d), (1 + d) / (2 + d)], rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [2, 5, 40])
def test_pagerank_star_into_dangling_center(n):
    """Leaves 1..n-1 all point at 0, which has no out-edge. Solving the stationary
    equations by hand: r(0) = (1 + (n-1)d) / (n + (n-1)d), leaves share the rest."""
    d = 0.85
    ro, col = csr_from_pairs(n, [(i, 0) for i in range(1, n)])
    r = oracle.pagerank(ro, col, 400, d)
    x = (1 + (n - 1) * d) / (n + (n - 1) * d)
    np.testing.assert_allclose(r[0], x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r[1:], (1 - x) / (n - 1), rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", range(4))
def test_pagerank_is_google_matrix_eigenvector(seed):
    """After many iterations the rank vector is the Perron vector of the Google
    matrix d*(P + dangling/N) + (1-d)/N, taken from numpy's eigen-solver."""
    n, d = 12, 0.85
    ro, col = random_small(n, 20, 500 + seed)
    P = np.zeros((n, n))
    outdeg = np.diff(ro.astype(np.int64))
    for u, v, _ in edges_of(ro, col):
        P[v, u] += 1.0 / outdeg[u]
    P[:, outdeg == 0] = 1.0 / n
    G = d * P + (1 - d) / n
    vals, vecs = np.linalg.eig(G)
    pv = np.real(vecs[:, np.argmax(np.real(vals))])
    pv = pv / pv.sum()
    r = oracle.pagerank(ro, col, 400, d)
    np.testing.assert_allclose(r, pv, rtol=0, atol=1e-12)


def test_pagerank_mass_conserved_rmat():
    ro, col = gen.rmat(14, 16, seed=3)
    r = oracle.pagerank(ro, col, 20, 0.85)
    assert abs(r.sum() - 1.0) < 1e-12
    # thread count does not change the result
    np.testing.assert_array_equal(r, oracle.pagerank(ro, col, 20, 0.85, threads=1))


# ------------------------------------------- the method: frontier & engines

def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def test_design_requirements_worked_example():
    g = read_golden("fig4_example.txt")
    n = int(g["n"][0])
    pairs = [tuple(int(x) for x in e.split(":")) for e in g["edges"]]
    ro, col = csr_from_pairs(n, pairs)
    active = np.zeros(n, np.uint8)
    active[[int(x) for x in g["active"]]] = 1
    col_off, in_src, _ = oracle.csc(ro, col)
    # source orientation: the active subset is the out-edges of the active vertices
    act_edges = [(u, v) for u, v in pairs if active[u]]
    assert len(act_edges) == int(g["active_edges"][0])
    dests = sorted({v for _, v in act_edges})
    assert dests == [int(x) for x in g["dest_frontier"]]
    # destination orientation visits every in-edge of those destinations
    dest_edges = sum(int(col_off[v + 1] - col_off[v]) for v in dests)
    assert dest_edges == int(g["dest_frontier_edges"][0])
    # the Wedge Frontier at one edge per group names exactly the active edges
    bits1, k1 = oracle.wedge_frontier(in_src, active, 1)
    assert k1 == len(act_edges)
    assert list(np.flatnonzero(bits1)) == [int(x) for x in g["group1_marked"]]
    bits2, k2 = oracle.wedge_frontier(in_src, active, 2)
    assert list(np.flatnonzero(bits2)) == [int(x) for x in g["group2_marked"]]
    visited2 = sum(min((gi + 1) * 2, len(in_src)) - gi * 2 for gi in np.flatnonzero(bits2))
    assert visited2 == int(g["group2_visited"][0])
    # superfluous edges are bounded by the group size
    assert 0 <= visited2 - k1 <= (2 - 1) * k2


def test_csc_positions_and_weights_follow_edges():
    ro, col = random_small(50, 300, 9)
    w = gen.edge_weights(ro, col, seed=1)
    col_off, in_src, in_w = oracle.csc(ro, col, w)
    wmap = {(u, v): int(w[j]) for u, v, j in edges_of(ro, col)}
    seen = []
    for v in range(50):
        srcs = in_src[int(col_off[v]):int(col_off[v + 1])]
        assert np.all(np.diff(srcs.astype(np.int64)) > 0)  # sources ascend
        for p in range(int(col_off[v]), int(col_off[v + 1])):
            seen.append((int(in_src[p]), v))
            assert int(in_w[p]) == wmap[(int(in_src[p]), v)]
    assert sorted(seen) == sorted(wmap)


def hop_bounded_minplus(n, wedges, init, rounds):
    """d_{j+1}[v] = min(d_j[v], min_u d_j[u] + W[u, v]): synchronous rounds with no
    frontier at all (dense min-plus products)."""
    W = np.full((n, n), np.inf)
    for u, v, w in wedges:
        W[u, v] = min(W[u, v], w)
    d = [np.array(init, float)]
    for _ in range(rounds):
        cur = d[-1]
        d.append(np.minimum(cur, np.min(cur[:, None] + W, axis=0)))
    return d


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("app", ["bfs", "sssp"])
def test_pull_engine_iterations_equal_hop_bounded_rounds(app, seed):
    """With synchronous semantics, iteration k of the frontier-restricted pull
    leaves exactly the best value over paths of <= k+1 edges, and the next
    frontier is the set of vertices whose value dropped."""
    n = 8 + seed
    ro, col = random_small(n, 3 * n, 600 + seed)
    w = gen.edge_weights(ro, col, seed=seed, lo=1, hi=9) if app == "sssp" else None
    s = int(gen.pick_sources(ro, 1, seed=seed)[0])
    wed = [(u, v, int(w[j]) if w is not None else 1) for u, v, j in edges_of(ro, col)]
    init = [np.inf] * n
    init[s] = 0
    tr = oracle.pull_engine(app, ro, col, w, s, keep_frontiers=True)
    rounds = hop_bounded_minplus(n, wed, init, tr.iters + 1)
    for k in range(tr.iters):
        want_fr = (rounds[k] < rounds[k - 1]).astype(np.uint8) if k else (np.arange(n) == s).astype(np.uint8)
        np.testing.assert_array_equal(tr.frontiers[k], want_fr)
    np.testing.assert_array_equal(tr.values, to_u32(rounds[tr.iters]))
    assert np.array_equal(rounds[tr.iters], rounds[tr.iters - 1])   # converged


@pytest.mark.parametrize("seed", range(6))
def test_pull_engine_cc_iterations_are_hop_balls(seed):
    """After iteration k, a label is the minimum id within k+1 undirected hops."""
    n = 9 + seed
    ro, col = random_small(n, n + 3, 700 + seed)
    sro, scol = oracle.symmetrize(ro, col)
    hop = floyd_warshall(n, [(u, v, 1) for u, v, _ in edges_of(sro, scol)])
    tr = oracle.pull_engine("cc", sro, scol, keep_frontiers=True)
    ids = np.arange(n)
    for k in range(1, tr.iters):
        prev = np.array([ids[hop[:, v] <= k - 1].min() for v in range(n)])
        cur = np.array([ids[hop[:, v] <= k].min() for v in range(n)])
        np.testing.assert_array_equal(tr.frontiers[k], (cur < prev).astype(np.uint8))
    np.testing.assert_array_equal(tr.values, oracle.cc(ro, col))


@pytest.mark.parametrize("seed", range(5))
def test_engines_agree_with_definitions(seed):
    ro, col = gen.rmat(10 + seed % 3, 8, seed=800 + seed)
    w = gen.edge_weights(ro, col, seed=seed)
    sro, scol = oracle.symmetrize(ro, col)
    s = int(gen.pick_sources(ro, 1, seed=seed)[0])
    lv = oracle.bfs(ro, col, s)
    tb = oracle.pull_engine("bfs", ro, col, None, s)
    np.testing.assert_array_equal(tb.values, lv)
    # BFS frontier k is exactly the set of vertices at level k
    np.testing.assert_array_equal(tb.F, np.bincount(lv[lv != INF], minlength=tb.iters)[:tb.iters])
    pv, pit, pF = oracle.push_engine("bfs", ro, col, None, s)
    np.testing.assert_array_equal(pv, lv)
    assert pit == tb.iters and np.array_equal(pF, tb.F)
    for app, args, ref in (("sssp", (ro, col, w, s), oracle.sssp(ro, col, w, s)),
                           ("cc", (sro, scol, None, 0), oracle.cc(ro, col))):
        tr = oracle.pull_engine(app, *args)
        np.testing.assert_array_equal(tr.values, ref)
        pv, pit, pF = oracle.push_engine(app, *args)
        np.testing.assert_array_equal(pv, ref)
        assert pit == tr.iters and np.array_equal(pF, tr.F)


@pytest.mark.parametrize("chunk", [1, 2, 16, 32, 64, 128])
def test_gate_and_wedge_frontier_bounds(chunk):
    ro, col = gen.rmat(11, 16, seed=900 + chunk)
    n, m = len(ro) - 1, len(col)
    w = gen.edge_weights(ro, col, seed=2)
    s = int(gen.pick_sources(ro, 1, seed=chunk)[0])
    outdeg = np.diff(ro.astype(np.int64))
    base = None
    for theta in (0, 10_000, 200_000, 1_000_001):
        tr = oracle.pull_engine("sssp", ro, col, w, s, theta_ppm=theta, chunk=chunk,
                                keep_frontiers=True)
        # precision and threshold never change values or the frontier sequence
        if base is None:
            base = tr
        np.testing.assert_array_equal(tr.values, base.values)
        np.testing.assert_array_equal(tr.F, base.F)
        for k in range(tr.iters):
            A = int(outdeg[tr.frontiers[k].astype(bool)].sum())
            assert tr.A[k] == A
            assert tr.mode[k] == (1 if A < (theta * m) // 1_000_000 else 0)
            assert tr.K[k] <= A
            if tr.mode[k]:
                assert 0 <= int(tr.edges[k]) - A <= (chunk - 1) * int(tr.K[k])
                if chunk == 1:
                    assert tr.edges[k] == A
            else:
                assert tr.edges[k] == m
        if theta == 0:
            assert not tr.mode.any()
        if theta > 1_000_000:
            assert tr.mode.all()

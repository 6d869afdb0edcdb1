"""Pins that tie the oracle to the mathematics, not to itself.

Each check uses an independent route: exact rational arithmetic, dense-matrix
power iteration, Floyd-Warshall, union-find, numpy set operations, and closed
forms on graphs whose answer is known (cycles, paths, stars, complete graphs,
grids).  Exhaustive over every directed graph on <= 3 vertices (and a large
sample on 4), plus seeded random graphs up to 64 vertices.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle

ALPHA = 0.85


# ---------------------------------------------------------------- helpers --

def all_graphs(n):
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v]
    for mask in range(1 << len(pairs)):
        yield [pairs[i] for i in range(len(pairs)) if mask >> i & 1]


def dense_adj(g):
    A = np.zeros((g.n, g.n))
    for u in range(g.n):
        for e in range(g.out.off[u], g.out.off[u + 1]):
            A[u, g.out.idx[e]] = 1.0
    return A


def power_iteration(A, iters, alpha=ALPHA):
    """Textbook matvec: x_{k+1} = (1-a)/n + a M^T x_k, M = D^-1 A, zero rows
    for vertices without out-edges."""
    n = A.shape[0]
    deg = A.sum(1)
    M = np.divide(A, deg[:, None], out=np.zeros_like(A), where=deg[:, None] > 0)
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = (1 - alpha) / n + alpha * (M.T @ x)
    return x


def exact_pagerank(n, edges, iters, alpha=Fraction(17, 20)):
    deg = [0] * n
    for u, _ in edges:
        deg[u] += 1
    x = [Fraction(1, n)] * n
    for _ in range(iters):
        y = [(1 - alpha) / n] * n
        for u, v in edges:
            y[v] += alpha * x[u] / deg[u]
        x = y
    return x


def floyd_warshall(n, edges, w=None):
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0)
    for k, (u, v) in enumerate(edges):
        D[u, v] = min(D[u, v], 1.0 if w is None else float(w[k]))
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def union_find_labels(n, edges):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for u, v in edges:
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[max(ru, rv)] = min(ru, rv)
    return np.array([find(v) for v in range(n)], np.int32)  # root == min id


def graph_of(n, edges, w=None):
    return oracle.Graph(gg.from_pairs(n, edges if edges else np.zeros((0, 2)), w))


def random_small(seed, n=None):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 65)) if n is None else n
    k = int(rng.integers(0, 4 * n + 1))
    src = rng.integers(0, n, k)
    dst = rng.integers(0, n, k)
    w = rng.integers(1, 1001, k).astype(np.uint32)
    return n, list(zip(src.tolist(), dst.tolist())), w


def dedup(n, edges, w=None):
    """Reference edge set: self-loops dropped, repeated pairs merged (min w)."""
    best = {}
    for k, (u, v) in enumerate(edges):
        if u == v:
            continue
        wk = 0 if w is None else int(w[k])
        if (u, v) not in best or wk < best[(u, v)]:
            best[(u, v)] = wk
    keys = sorted(best)
    return keys, [best[k] for k in keys]


# --------------------------------------------------------- adjacency build --

@pytest.mark.parametrize("seed", range(20))
def test_build_adj_matches_set_semantics(seed):
    n, edges, w = random_small(seed)
    g = graph_of(n, edges, w)
    keys, ws = dedup(n, edges, w)
    got = [(u, int(g.out.idx[e])) for u in range(n) for e in range(g.out.off[u], g.out.off[u + 1])]
    assert got == keys
    assert g.out.w.tolist() == ws
    # CSC is the transpose with rows sorted by source
    tk = sorted((v, u) for u, v in keys)
    gotc = [(v, int(g.inc.idx[e])) for v in range(n) for e in range(g.inc.off[v], g.inc.off[v + 1])]
    assert gotc == tk


def test_build_adj_numpy_unique_rmat():
    el = gg.rmat(10)
    g = oracle.Graph(el)
    keep = el.src != el.dst
    key = np.unique(el.src[keep].astype(np.int64) * el.n + el.dst[keep])
    assert g.m == key.shape[0]
    rows = np.repeat(np.arange(el.n), np.diff(g.out.off))
    assert np.array_equal(rows.astype(np.int64) * el.n + g.out.idx, key)


def test_build_adj_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.build_adj(3, np.array([0, 5]), np.array([1, 1]))


# ---------------------------------------------------------------- PageRank --

@pytest.mark.parametrize("n", [1, 2, 3])
def test_pagerank_exhaustive_small_vs_power_iteration(n):
    for edges in all_graphs(n):
        g = graph_of(n, edges)
        for iters in (0, 1, 5, 20):
            x = oracle.pagerank(g, iters)
            ref = power_iteration(dense_adj(g), iters)
            np.testing.assert_allclose(x, ref, rtol=1e-13, atol=0)


def test_pagerank_n4_sample_vs_exact_rationals():
    rng = np.random.default_rng(7)
    graphs = list(all_graphs(4))
    for i in rng.choice(len(graphs), 300, replace=False):
        edges = graphs[i]
        g = graph_of(4, edges)
        x = oracle.pagerank(g, 6)
        ex = exact_pagerank(4, edges, 6)
        np.testing.assert_allclose(x, [float(f) for f in ex], rtol=1e-14, atol=0)


@pytest.mark.parametrize("seed", range(10))
def test_pagerank_random_vs_power_iteration(seed):
    n, edges, _ = random_small(seed)
    g = graph_of(n, edges)
    np.testing.assert_allclose(oracle.pagerank(g, 20), power_iteration(dense_adj(g), 20),
                               rtol=1e-12, atol=0)


def test_pagerank_cycle_uniform():
    g = oracle.Graph(gg.cycle(97))
    np.testing.assert_allclose(oracle.pagerank(g, 20), 1.0 / 97, rtol=1e-14)


def test_pagerank_edgeless():
    g = oracle.Graph(gg.empty(10))
    np.testing.assert_allclose(oracle.pagerank(g, 20), (1 - ALPHA) / 10, rtol=1e-15)
    np.testing.assert_allclose(oracle.pagerank(g, 0), 0.1, rtol=1e-15)


def test_pagerank_mass_conservation_without_dangling():
    g = oracle.Graph(gg.complete(9))
    for k in (1, 3, 20):
        assert abs(oracle.pagerank(g, k).sum() - 1.0) < 1e-13


def test_pagerank_mass_with_dangling():
    g = oracle.Graph(gg.rmat(9))
    deg = g.out.degrees()
    for k in range(1, 6):
        xk = oracle.pagerank(g, k - 1)
        xk1 = oracle.pagerank(g, k)
        expect = (1 - ALPHA) + ALPHA * xk[deg > 0].sum()
        assert abs(xk1.sum() - expect) < 1e-12


def test_pagerank_star_closed_form():
    # centre 0 -> leaves: leaves get (1-a)/n + a * x0/(n-1); x0 = (1-a)/n for k>=1
    n = 6
    g = oracle.Graph(gg.star(n))
    x = oracle.pagerank(g, 3)
    x0 = (1 - ALPHA) / n
    assert abs(x[0] - x0) < 1e-16
    np.testing.assert_allclose(x[1:], (1 - ALPHA) / n + ALPHA * x0 / (n - 1), rtol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_prdelta_eps0_equals_pagerank(seed):
    el = gg.rmat(8 + seed, seed=seed + 11)
    g = oracle.Graph(el)
    for iters in (1, 2, 10, 20):
        r, active = oracle.prdelta(g, iters, ALPHA, 0.0)
        x = oracle.pagerank(g, iters)
        np.testing.assert_allclose(r, x, rtol=1e-12, atol=0)


def test_prdelta_eps_shrinks_frontier():
    g = oracle.Graph(gg.rmat(10, seed=3))
    _, active = oracle.prdelta(g, 10, ALPHA, 0.1)
    assert active[0] <= g.n and active[-1] < active[0]


# --------------------------------------------------------------------- BFS --

@pytest.mark.parametrize("n", [1, 2, 3])
def test_bfs_exhaustive_vs_floyd_warshall(n):
    for edges in all_graphs(n):
        g = graph_of(n, edges)
        D = floyd_warshall(n, edges)
        for s in range(n):
            level, parent = oracle.bfs(g, s)
            ref = np.where(np.isinf(D[s]), -1, D[s]).astype(np.int32)
            assert np.array_equal(level, ref)
            assert oracle.check_bfs_parents(g, s, level, parent) == []


@pytest.mark.parametrize("seed", range(12))
def test_bfs_random_vs_floyd_warshall(seed):
    n, edges, _ = random_small(seed + 100)
    g = graph_of(n, edges)
    D = floyd_warshall(n, edges)
    for s in range(0, n, max(1, n // 4)):
        level, parent = oracle.bfs(g, s)
        ref = np.where(np.isinf(D[s]), -1, D[s]).astype(np.int32)
        assert np.array_equal(level, ref)
        assert oracle.check_bfs_parents(g, s, level, parent) == []


def test_bfs_closed_forms():
    n = 50
    lv, _ = oracle.bfs(oracle.Graph(gg.cycle(n)), 7)
    assert np.array_equal(lv, (np.arange(n) - 7) % n)
    lv, _ = oracle.bfs(oracle.Graph(gg.path(n)), 10)
    assert np.array_equal(lv, np.where(np.arange(n) >= 10, np.arange(n) - 10, -1))
    lv, _ = oracle.bfs(oracle.Graph(gg.star(n)), 0)
    assert lv[0] == 0 and np.all(lv[1:] == 1)
    lv, _ = oracle.bfs(oracle.Graph(gg.star(n, out=False)), 0)
    assert lv[0] == 0 and np.all(lv[1:] == -1)
    lv, _ = oracle.bfs(oracle.Graph(gg.complete(12)), 3)
    assert lv[3] == 0 and np.sum(lv == 1) == 11
    R, C = 30, 41
    lv, _ = oracle.bfs(oracle.Graph(gg.grid(R, C, 0.0, weighted=False)), 0)
    r, c = np.divmod(np.arange(R * C), C)
    assert np.array_equal(lv, r + c)


def test_bfs_parent_checker_catches_planted_errors():
    el = gg.rmat(10, seed=5)
    g = oracle.Graph(el)
    s = int(gg.pick_sources(el, 1, 3)[0])
    level, parent = oracle.bfs(g, s)
    assert oracle.check_bfs_parents(g, s, level, parent) == []
    bad = parent.copy()
    v = int(np.nonzero(level == 2)[0][0])
    bad[v] = int(np.nonzero(level == 2)[0][1])  # same level, not a valid parent
    assert oracle.check_bfs_parents(g, s, level, bad)
    bad = parent.copy()
    bad[v] = -1
    assert oracle.check_bfs_parents(g, s, level, bad)
    bad = parent.copy()
    u = int(np.nonzero(level == 1)[0][0])
    w = int(np.nonzero((level == 1) & ~np.isin(np.arange(g.n), g.out.idx[g.out.off[u]:g.out.off[u + 1]]))[0][0])
    cand = np.nonzero(level == 2)[0]
    # a level-1 vertex that has no edge to some level-2 vertex: plausible but wrong parent
    for t in cand:
        if t not in g.out.idx[g.out.off[u]:g.out.off[u + 1]]:
            bad[t] = u
            break
    assert oracle.check_bfs_parents(g, s, level, bad)


# ---------------------------------------------------------------------- CC --

@pytest.mark.parametrize("n", [1, 2, 3])
def test_cc_exhaustive_vs_union_find(n):
    for edges in all_graphs(n):
        lab, _ = oracle.cc(graph_of(n, edges))
        assert np.array_equal(lab, union_find_labels(n, edges))


def test_cc_n4_exhaustive_vs_union_find():
    for edges in all_graphs(4):
        lab, _ = oracle.cc(graph_of(4, edges))
        assert np.array_equal(lab, union_find_labels(4, edges))


@pytest.mark.parametrize("seed", range(12))
def test_cc_random_vs_union_find(seed):
    n, edges, _ = random_small(seed + 200)
    lab, _ = oracle.cc(graph_of(n, edges))
    assert np.array_equal(lab, union_find_labels(n, edges))


def test_cc_closed_forms():
    lab, rounds = oracle.cc(oracle.Graph(gg.path(40)))
    assert np.all(lab == 0) and rounds == 40   # min label moves one hop per round
    lab, _ = oracle.cc(oracle.Graph(gg.grid(20, 30, 0.0, weighted=False)))
    assert np.all(lab == 0)
    lab, rounds = oracle.cc(oracle.Graph(gg.empty(9)))
    assert np.array_equal(lab, np.arange(9)) and rounds == 1
    # k disjoint directed cycles of length 5 on a shuffled id space
    perm = gg.permutation(50, 3)
    src = np.concatenate([perm[5 * c + np.arange(5)] for c in range(10)])
    dst = np.concatenate([perm[5 * c + (np.arange(5) + 1) % 5] for c in range(10)])
    lab, _ = oracle.cc(oracle.Graph(gg.EdgeList(50, src, dst)))
    for c in range(10):
        members = perm[5 * c:5 * c + 5]
        assert np.all(lab[members] == members.min())


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_cc_union_find_oracle_exhaustive(n):
    """The oracle's union-find CC (raw records, no adjacency) gives the
    least-id labels and the component count of every graph on n <= 4."""
    for edges in all_graphs(n):
        src = np.array([u for u, _ in edges], np.int32)
        dst = np.array([v for _, v in edges], np.int32)
        lab, comps = oracle.cc_union_find(n, src, dst)
        ref = union_find_labels(n, edges)
        assert np.array_equal(lab, ref), edges
        assert comps == len(set(ref.tolist()))


@pytest.mark.parametrize("seed", range(8))
def test_cc_union_find_oracle_vs_label_propagation(seed):
    """Shuffled records (with repeats, self-loops and ids in any order) give
    the labels of the label-propagation oracle."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    m = int(rng.integers(0, 3 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    lab, comps = oracle.cc_union_find(n, src, dst)
    ref, _ = oracle.cc(oracle.Graph(gg.EdgeList(n, src, dst)))
    assert np.array_equal(lab, ref)
    assert comps == len(np.unique(ref))


def test_cc_union_find_oracle_closed_forms():
    # a path whose records run from the largest id down: every link goes
    # under a smaller root, the final pass resolves chains of any length
    n = 1000
    lab, comps = oracle.cc_union_find(n, np.arange(n - 1, 0, -1), np.arange(n - 2, -1, -1))
    assert np.all(lab == 0) and comps == 1
    lab, comps = oracle.cc_union_find(7, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert np.array_equal(lab, np.arange(7)) and comps == 7
    with pytest.raises(ValueError):
        oracle.cc_union_find(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))


def test_cc_rmat_vs_union_find():
    el = gg.rmat(12, seed=9)
    g = oracle.Graph(el)
    lab, _ = oracle.cc(g)
    edges = list(zip(el.src.tolist(), el.dst.tolist()))
    assert np.array_equal(lab, union_find_labels(el.n, edges))


# -------------------------------------------------------------------- SSSP --

@pytest.mark.parametrize("n", [2, 3])
def test_sssp_exhaustive_vs_floyd_warshall(n):
    rng = np.random.default_rng(n)
    for edges in all_graphs(n):
        w = rng.integers(1, 1001, len(edges)).astype(np.uint32)
        g = graph_of(n, edges, w)
        D = floyd_warshall(n, edges, w)
        for s in range(n):
            ref = np.where(np.isinf(D[s]), 0xFFFFFFFF, D[s]).astype(np.uint32)
            assert np.array_equal(oracle.dijkstra(g, s), ref)
            assert np.array_equal(oracle.bellman_ford(g, s)[0], ref)


@pytest.mark.parametrize("seed", range(12))
def test_sssp_random_vs_floyd_warshall(seed):
    n, edges, w = random_small(seed + 300)
    g = graph_of(n, edges, w)
    D = floyd_warshall(n, edges, w)
    for s in range(0, n, max(1, n // 3)):
        ref = np.where(np.isinf(D[s]), 0xFFFFFFFF, D[s]).astype(np.uint32)
        assert np.array_equal(oracle.dijkstra(g, s), ref)
        assert np.array_equal(oracle.bellman_ford(g, s)[0], ref)


def test_sssp_unit_weights_equal_bfs_levels():
    el = gg.rmat(11, seed=4)
    el.w = np.ones(el.m, np.uint32)
    g = oracle.Graph(el)
    lv, _ = oracle.bfs(g, 5)
    d = oracle.dijkstra(g, 5)
    assert np.array_equal(np.where(lv < 0, 0xFFFFFFFF, lv).astype(np.uint32), d)


def test_sssp_grid_manhattan():
    R, C = 25, 33
    el = gg.grid(R, C, 0.0, weighted=True, wlo=1, whi=1)
    d = oracle.dijkstra(oracle.Graph(el), 0)
    r, c = np.divmod(np.arange(R * C), C)
    assert np.array_equal(d, (r + c).astype(np.uint32))


def test_sssp_overflow_detected():
    el = gg.path(4)
    el.w = np.full(3, 0x7FFFFFFF, np.uint32)
    g = oracle.Graph(el)
    with pytest.raises(OverflowError):
        oracle.dijkstra(g, 0)
    with pytest.raises(OverflowError):
        oracle.bellman_ford(g, 0)


# ---------------------------------------------------------------- betweenness

def brute_bc(n, src, dst, s):
    """Dependencies by definition: all-pairs shortest-path lengths and counts
    (Floyd-Warshall over path counts), then
    delta_s(v) = sum over t != s, v of sigma_st(v) / sigma_st,
    sigma_st(v) = sigma_sv * sigma_vt when d(s,v) + d(v,t) = d(s,t)."""
    INF = float("inf")
    d = [[INF] * n for _ in range(n)]
    c = [[0] * n for _ in range(n)]
    for i in range(n):
        d[i][i] = 0
        c[i][i] = 1
    for a, b in set(zip(src, dst)):
        if a != b:
            d[a][b] = 1
            c[a][b] = 1
    # path counts by BFS layers from every vertex (unit weights)
    for i in range(n):
        dist = [INF] * n
        cnt = [0] * n
        dist[i], cnt[i] = 0, 1
        frontier = [i]
        adj = {}
        for a, b in set(zip(src, dst)):
            if a != b:
                adj.setdefault(a, []).append(b)
        while frontier:
            nxt = []
            for u in frontier:
                for w in adj.get(u, []):
                    if dist[w] == INF:
                        dist[w] = dist[u] + 1
                        nxt.append(w)
                    if dist[w] == dist[u] + 1:
                        cnt[w] += cnt[u]
            frontier = nxt
        d[i], c[i] = dist, cnt
    out = []
    for v in range(n):
        tot = Fraction(0)
        if v != s:
            for t in range(n):
                if t in (s, v) or d[s][t] == INF:
                    continue
                if d[s][v] + d[v][t] == d[s][t]:
                    tot += Fraction(c[s][v] * c[v][t], c[s][t])
        out.append(float(tot))
    return np.array(out)


@pytest.mark.parametrize("seed", range(5))
def test_bc_matches_definition(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 14))
    el = gg.uniform(n, int(rng.integers(n, 4 * n)), seed=300 + seed)
    g = oracle.Graph(el)
    for s in range(min(n, 4)):
        delta, sigma = oracle.bc(g, s)
        ref = brute_bc(n, list(el.src), list(el.dst), s)
        assert np.allclose(delta, ref, rtol=1e-12, atol=1e-12), (seed, s)


def test_bc_closed_forms():
    # path 0 -> 1 -> ... -> n-1 from 0: vertex v lies on the paths to the
    # n-1-v vertices after it
    n = 9
    g = oracle.Graph(gg.path(n))
    delta, sigma = oracle.bc(g, 0)
    assert list(delta) == [0.0] + [float(n - 1 - v) for v in range(1, n)]
    assert np.all(sigma == 1.0)
    # star out of the center: every leaf has dependency 0
    g = oracle.Graph(gg.star(7))
    delta, _ = oracle.bc(g, 0)
    assert np.all(delta == 0.0)
    # diamond 0->1, 0->2, 1->3, 2->3: two shortest paths to 3, each middle
    # vertex carries half of it
    el = gg.from_pairs(4, [(0, 1), (0, 2), (1, 3), (2, 3)])
    delta, sigma = oracle.bc(oracle.Graph(el), 0)
    assert list(sigma) == [1.0, 1.0, 1.0, 2.0]
    assert list(delta) == [0.0, 0.5, 0.5, 0.0]


# -------------------------------------------------------- eigenvector centrality

def dense_eigenvector(n, src, dst, iters):
    A = np.zeros((n, n))
    for a, b in set(zip(src, dst)):
        if a != b:
            A[a, b] = 1.0
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        y = A.T @ x
        nrm = np.linalg.norm(y)
        x = y / nrm if nrm > 0 else np.zeros(n)
    return x


@pytest.mark.parametrize("seed", range(4))
def test_eigenvector_matches_dense_power_iteration(seed):
    el = gg.uniform(40 + 7 * seed, 200, seed=400 + seed)
    x = oracle.eigenvector(oracle.Graph(el), 15)
    assert np.allclose(x, dense_eigenvector(el.n, list(el.src), list(el.dst), 15), rtol=1e-12,
                       atol=1e-15)


def test_eigenvector_closed_forms():
    n = 12
    x = oracle.eigenvector(oracle.Graph(gg.cycle(n)), 7)          # stays uniform
    assert np.allclose(x, 1.0 / np.sqrt(n), rtol=1e-14)
    x = oracle.eigenvector(oracle.Graph(gg.complete(9)), 3)
    assert np.allclose(x, 1.0 / 3.0, rtol=1e-14)
    star_in = gg.star(10, out=False)                                # leaves -> centre 0
    x1 = oracle.eigenvector(oracle.Graph(star_in), 1)
    assert x1[0] == 1.0 and np.all(x1[1:] == 0.0)
    x2 = oracle.eigenvector(oracle.Graph(star_in), 2)              # the centre points nowhere
    assert np.all(x2 == 0.0)
    assert np.all(oracle.eigenvector(oracle.Graph(gg.empty(5)), 4) == 0.0)

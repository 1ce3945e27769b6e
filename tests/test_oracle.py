"""Pins for the CPU oracle: checks against things other than the oracle itself.

Each test checks the oracle against brute force (Floyd-Warshall, dense
matrices), closed forms on small families, library routines (scipy.sparse
.csgraph), invariants of the fixed point, or the worked example of the
paper's Figure 2.  A plausible mistake in the oracle (a dropped term, a wrong
index, an off-by-one in a bin boundary or in the iteration count) fails at
least one of them.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle

INF = oracle.INF
HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------
# helpers written independently of the oracle
# ----------------------------------------------------------------------------

def floyd_warshall(g, unit=False):
    n = g.n
    D = np.full((n, n), np.inf)
    src = np.repeat(np.arange(n), g.degrees())
    w = np.ones(g.m) if (unit or g.w is None) else g.w.astype(np.float64)
    for u, v, c in zip(src, g.col, w):
        D[u, v] = min(D[u, v], c)
    np.fill_diagonal(D, 0.0)
    for k in range(n):
        D = np.minimum(D, D[:, k, None] + D[None, k, :])
    return D


def to_int_dist(row):
    out = np.where(np.isinf(row), INF, row)
    return out.astype(np.int64).astype(np.int32)


def scipy_matrix(g, weights=None):
    data = np.ones(g.m) if weights is None else weights.astype(np.float64)
    return sp.csr_matrix((data, g.col, g.off), shape=(g.n, g.n))


def edge_src(g):
    return np.repeat(np.arange(g.n), g.degrees())


def tiny_graphs(weighted):
    out = []
    for n, m, seed in [(1, 0, 1), (2, 1, 2), (5, 8, 3), (12, 30, 4), (20, 25, 5), (33, 120, 6), (48, 60, 7)]:
        out.append(gg.random_digraph(n, max(m, 1), seed, weighted=weighted) if n > 1 else gg.edgeless(1))
    return out


# ----------------------------------------------------------------------------
# BFS
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("gi", range(7))
def test_bfs_vs_floyd_warshall(gi):
    g = tiny_graphs(False)[gi]
    D = floyd_warshall(g, unit=True)
    for s in range(g.n):
        assert np.array_equal(oracle.bfs(g, s), to_int_dist(D[s]))


def test_bfs_closed_forms():
    n = 37
    assert np.array_equal(oracle.bfs(gg.path(n), 0), np.arange(n))
    lv = oracle.bfs(gg.path(n), 5)
    assert np.all(lv[:5] == INF) and np.array_equal(lv[5:], np.arange(n - 5))
    assert np.array_equal(oracle.bfs(gg.cycle(n), 0), np.arange(n))
    assert np.array_equal(oracle.bfs(gg.cycle(n), 3), (np.arange(n) - 3) % n)
    k = 50
    st = gg.star(k)
    assert np.array_equal(oracle.bfs(st, 0), np.r_[0, np.ones(k, dtype=np.int32)])
    lv = oracle.bfs(st, 7)
    expect = np.full(k + 1, 2)
    expect[0], expect[7] = 1, 0
    assert np.array_equal(lv, expect)
    r, c = 9, 13
    i, j = np.divmod(np.arange(r * c), c)
    assert np.array_equal(oracle.bfs(gg.grid(r, c), 0), i + j)
    assert np.array_equal(oracle.bfs(gg.edgeless(6), 2), np.where(np.arange(6) == 2, 0, INF))


def check_bfs_invariants(g, s, lv):
    src = edge_src(g)
    assert lv[s] == 0
    reached_u = lv[src] < INF
    # every edge out of a reached vertex: level[v] <= level[u] + 1
    assert np.all(lv[g.col[reached_u]] <= lv[src[reached_u]] + 1)
    # every reached v != s has an in-edge with equality
    tight = np.zeros(g.n, dtype=bool)
    eq = reached_u & (lv[g.col] == lv[src] + 1)
    tight[g.col[eq]] = True
    reached = lv < INF
    reached[s] = False
    assert np.all(tight[reached])


def test_bfs_scipy_and_invariants():
    g = gg.rmat(12, 16, seed=11)
    for s in [0, 1, 77, 4095]:
        lv = oracle.bfs(g, s)
        ref = csg.shortest_path(scipy_matrix(g), directed=True, unweighted=True, indices=s)
        assert np.array_equal(lv, to_int_dist(ref))
        check_bfs_invariants(g, s, lv)


def test_bfs_invariants_rmat14():
    g = gg.workload("rmat14")
    check_bfs_invariants(g, 0, oracle.bfs(g, 0))


# ----------------------------------------------------------------------------
# SSSP
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("gi", range(7))
def test_sssp_vs_floyd_warshall(gi):
    g = tiny_graphs(True)[gi]
    if g.w is None:
        g = gg.Graph(g.n, g.off, g.col, np.zeros(g.m, dtype=np.int32))
    D = floyd_warshall(g)
    for s in range(g.n):
        assert np.array_equal(oracle.sssp(g, s), to_int_dist(D[s]))


def test_sssp_unit_weights_equal_bfs():
    g = gg.rmat(11, 8, seed=5)
    g1 = gg.Graph(g.n, g.off, g.col, np.ones(g.m, dtype=np.int32))
    for s in [0, 3, 100]:
        assert np.array_equal(oracle.sssp(g1, s), oracle.bfs(g, s))


def test_sssp_closed_forms():
    n = 40
    w = gg.uniform_ints(n - 1, 100, seed=9) + 1
    g = gg.path(n, w)
    assert np.array_equal(oracle.sssp(g, 0), np.r_[0, np.cumsum(w)].astype(np.int32))
    k = 30
    ws = gg.uniform_ints(k, 50, seed=10) + 1
    st = gg.star(k, ws)
    assert np.array_equal(oracle.sssp(st, 0), np.r_[0, ws])
    r, c, cw = 7, 11, 13
    i, j = np.divmod(np.arange(r * c), c)
    assert np.array_equal(oracle.sssp(gg.grid(r, c, weight=cw), 0), cw * (i + j))
    # zero weights are allowed
    gz = gg.Graph(g.n, g.off, g.col, np.zeros(g.m, dtype=np.int32))
    assert np.array_equal(oracle.sssp(gz, 0), np.zeros(n, dtype=np.int32))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_sssp_zero_weights_vs_floyd_warshall(seed):
    """Weights uniform in [0, 2]: zero-weight edges and zero-weight cycles."""
    g = gg.random_digraph(30, 150, seed).with_weights(seed, 0, 2)
    assert (g.w == 0).sum() > 10
    D = floyd_warshall(g)
    for s in range(g.n):
        assert np.array_equal(oracle.sssp(g, s), to_int_dist(D[s]))
    gz = gg.cycle(17, w=np.zeros(17, np.int64))
    assert np.array_equal(oracle.sssp(gz, 5), np.zeros(17, np.int32))


def test_sssp_int32_boundary():
    """A path whose last vertex lies at INT32_MAX - 1 (62 edges of weight
    (2^31 - 2) / 62) with backward edges whose candidates exceed INT32_MAX:
    vertex i at i * W (closed form), and Floyd-Warshall agrees."""
    g = gg.boundary_path(63, 400, seed=4, hub_back=40)
    W = (2 ** 31 - 2) // 62
    assert W * 62 == 2 ** 31 - 2 and int(g.w.max()) == W
    d = oracle.sssp(g, 0)
    assert np.array_equal(d.astype(np.int64), np.arange(63, dtype=np.int64) * W)
    assert int(d[-1]) == 2 ** 31 - 2
    D = floyd_warshall(g)
    for s in (0, 1, 31, 62):
        assert np.array_equal(oracle.sssp(g, s), to_int_dist(D[s]))


def check_sssp_invariants(g, s, d):
    src = edge_src(g)
    d64 = d.astype(np.int64)
    w = g.w.astype(np.int64)
    assert d[s] == 0
    ru = d[src] < INF
    assert np.all(d64[g.col[ru]] <= d64[src[ru]] + w[ru])
    tight = np.zeros(g.n, dtype=bool)
    eq = ru & (d64[g.col] == d64[src] + w)
    tight[g.col[eq]] = True
    reached = d < INF
    reached[s] = False
    assert np.all(tight[reached])
    # a vertex is reachable exactly when BFS reaches it
    assert np.array_equal(d < INF, oracle.bfs(g, s) < INF)


def test_sssp_scipy_and_invariants():
    g = gg.rmat(12, 16, seed=12).with_weights(3)
    for s in [0, 5, 999]:
        d = oracle.sssp(g, s)
        ref = csg.dijkstra(scipy_matrix(g, g.w), directed=True, indices=s)
        assert np.array_equal(d, to_int_dist(ref))
        check_sssp_invariants(g, s, d)


def test_sssp_invariants_zipf():
    g = gg.zipf(1 << 15, 1.9, 1 << 13, seed=4).with_weights(5)
    s = g.max_degree_vertex()
    check_sssp_invariants(g, s, oracle.sssp(g, s))


# ----------------------------------------------------------------------------
# CC
# ----------------------------------------------------------------------------

def check_cc_invariants(g, lab):
    src = edge_src(g)
    v = np.arange(g.n)
    assert np.all(lab[src] == lab[g.col])
    assert np.all(lab <= v)
    assert np.all(lab[lab] == lab)
    # label[v] == v exactly for the minimum of each component
    mins = np.unique(lab)
    assert np.array_equal(np.flatnonzero(lab == v), mins)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cc_vs_scipy(seed):
    g = gg.random_digraph(3000, 2600, seed)
    lab = oracle.cc(g)
    ncomp, ref = csg.connected_components(scipy_matrix(g), directed=True, connection="weak")
    # same partition ...
    assert len(np.unique(lab)) == ncomp
    pairs = np.unique(np.stack([lab, ref]), axis=1)
    assert pairs.shape[1] == ncomp
    # ... labelled by its minimum id
    first = np.full(ncomp, g.n)
    np.minimum.at(first, ref, np.arange(g.n))
    assert np.array_equal(lab, first[ref])
    check_cc_invariants(g, lab)


def test_cc_closed_forms():
    assert np.array_equal(oracle.cc(gg.path(20)), np.zeros(20, dtype=np.int32))
    assert np.array_equal(oracle.cc(gg.star(15)), np.zeros(16, dtype=np.int32))
    assert np.array_equal(oracle.cc(gg.grid(5, 8)), np.zeros(40, dtype=np.int32))
    assert np.array_equal(oracle.cc(gg.edgeless(9)), np.arange(9))
    base = gg.cycle(11)
    k = 6
    lab = oracle.cc(gg.disjoint_copies(base, k))
    assert np.array_equal(lab, np.repeat(np.arange(k) * 11, 11))
    # direction is ignored: a reversed path is still one component
    g = gg.from_edges(10, np.arange(1, 10), np.arange(0, 9))
    assert np.array_equal(oracle.cc(g), np.zeros(10, dtype=np.int32))


def test_cc_invariants_rmat():
    g = gg.rmat(13, 4, seed=3)
    check_cc_invariants(g, oracle.cc(g))


# ----------------------------------------------------------------------------
# PageRank
# ----------------------------------------------------------------------------

def dense_pagerank(g, d, iters):
    n = g.n
    M = np.zeros((n, n))
    deg = g.degrees()
    for u, v in zip(edge_src(g), g.col):
        M[v, u] += 1.0 / deg[u]
    dangling = deg == 0
    x = np.full(n, 1.0 / n)
    for _ in range(iters):
        x = (1 - d) / n + d * (M @ x + x[dangling].sum() / n)
    return x


# ----------------------------------------------------------------------------
# k-core
# ----------------------------------------------------------------------------

def kcore_brute_force(g, k):
    """The k-core straight from its definition: the union of every vertex set
    in which each member has at least k neighbours inside the set."""
    n = g.n
    adj = np.zeros((n, n), dtype=bool)
    adj[edge_src(g), g.col] = True
    core = np.zeros(n, dtype=bool)
    for mask in range(1, 1 << n):
        inside = np.array([(mask >> v) & 1 for v in range(n)], dtype=bool)
        if (adj[inside][:, inside].sum(axis=1) >= k).all():
            core |= inside
    return core.astype(np.int32)


@pytest.mark.parametrize("n,m,seed", [(6, 9, 1), (8, 14, 2), (10, 22, 3), (10, 30, 4), (11, 12, 5)])
def test_kcore_vs_brute_force(n, m, seed):
    g = gg.symmetrised(gg.random_digraph(n, m, seed))
    for k in range(0, 7):
        assert np.array_equal(oracle.kcore(g, k), kcore_brute_force(g, k)), (n, m, seed, k)


def test_kcore_closed_forms():
    ones, zeros = (lambda n: np.ones(n, np.int32)), (lambda n: np.zeros(n, np.int32))
    K = gg.complete(7)  # every vertex has 6 neighbours
    assert np.array_equal(oracle.kcore(K, 6), ones(7)) and np.array_equal(oracle.kcore(K, 7), zeros(7))
    cyc = gg.symmetrised(gg.cycle(30))
    assert np.array_equal(oracle.kcore(cyc, 2), ones(30)) and np.array_equal(oracle.kcore(cyc, 3), zeros(30))
    p = gg.path(25, directed=False)  # the ends peel inwards
    assert np.array_equal(oracle.kcore(p, 1), ones(25)) and np.array_equal(oracle.kcore(p, 2), zeros(25))
    st = gg.star(40)
    assert np.array_equal(oracle.kcore(st, 1), ones(41)) and np.array_equal(oracle.kcore(st, 2), zeros(41))
    gr = gg.grid(9, 13)  # corners have 2 neighbours; at k = 3 the border peels and so does the rest
    assert np.array_equal(oracle.kcore(gr, 2), ones(117)) and np.array_equal(oracle.kcore(gr, 3), zeros(117))
    assert np.array_equal(oracle.kcore(gg.edgeless(5), 0), ones(5))
    assert np.array_equal(oracle.kcore(gg.edgeless(5), 1), zeros(5))
    # a 5-clique with a pendant path: only the clique is in the 4-core
    src = [i for i in range(5) for j in range(5) if i != j] + [4, 5, 6]
    dst = [j for i in range(5) for j in range(5) if i != j] + [5, 6, 7]
    g = gg.undirected(8, src, dst)
    assert np.array_equal(oracle.kcore(g, 4), np.array([1] * 5 + [0] * 3, np.int32))


def test_symmetrised_matches_edge_list_construction():
    """The oracle's C symmetrisation equals the undirected graph built from the
    edge list in Python (both directions, no self-loops or duplicates)."""
    for g in (gg.rmat(10, seed=3), gg.random_digraph(500, 3000, 2), gg.star(20), gg.edgeless(4),
              gg.from_edges(5, [0, 1, 1, 2, 3], [1, 0, 1, 4, 3], keep_self_loops=True)):
        a, b = oracle.symmetrised(g), gg.symmetrised(g)
        assert np.array_equal(a.off, b.off) and np.array_equal(a.col, b.col)


def test_kcore_invariants_rmat():
    g = gg.symmetrised(gg.rmat(12, 8, seed=5))
    prev = np.ones(g.n, np.int32)
    src = edge_src(g)
    for k in (1, 2, 4, 8, 16, 32):
        c = oracle.kcore(g, k)
        # inside the core every vertex keeps at least k core neighbours
        inside = np.zeros(g.n, np.int64)
        np.add.at(inside, src, c[g.col])
        assert (inside[c == 1] >= k).all()
        # cores are nested
        assert (c <= prev).all()
        prev = c


def test_pagerank_vs_dense():
    for g in [gg.random_digraph(30, 70, 4), gg.star(6), gg.path(9), gg.random_digraph(64, 300, 8),
              gg.rmat(7, 4, seed=2)]:
        for it in [0, 1, 2, 50]:
            x = oracle.pagerank(g, 0.85, it)
            assert np.allclose(x, dense_pagerank(g, 0.85, it), rtol=0, atol=1e-14)


def test_pagerank_converged_solve():
    g = gg.random_digraph(50, 200, 21)
    n, d = g.n, 0.85
    deg = g.degrees()
    G = np.zeros((n, n))
    for u, v in zip(edge_src(g), g.col):
        G[v, u] += 1.0 / deg[u]
    G[:, deg == 0] = 1.0 / n
    x_star = np.linalg.solve(np.eye(n) - d * G, np.full(n, (1 - d) / n))
    x = oracle.pagerank(g, d, 400)
    assert np.abs(x - x_star).max() < 1e-13


def test_pagerank_closed_forms():
    d = 0.85
    n = 17
    assert np.allclose(oracle.pagerank(gg.edgeless(n), d, 50), 1.0 / n, rtol=0, atol=0)
    for g in [gg.cycle(n), gg.complete(9)]:
        x = oracle.pagerank(g, d, 50)
        assert np.abs(x - 1.0 / g.n).max() < 1e-16
    # undirected star with k leaves: centre c_t = c* + (-d)^t (1/N - c*)
    k = 12
    N = k + 1
    cstar = ((1 - d) / N + d) / (1 + d)
    for t in [0, 1, 2, 49, 50, 51]:
        x = oracle.pagerank(gg.star(k), d, t)
        c = cstar + (-d) ** t * (1.0 / N - cstar)
        assert abs(x[0] - c) < 1e-15
        assert np.abs(x[1:] - (1 - c) / k).max() < 1e-15
    # 49, 50 and 51 iterations are distinguishable at the centre
    x49, x50, x51 = (oracle.pagerank(gg.star(k), d, t)[0] for t in (49, 50, 51))
    assert min(abs(x49 - x50), abs(x50 - x51)) > 1e-5


def test_pagerank_sums_to_one():
    for g in [gg.rmat(10, 8, seed=3), gg.random_digraph(100, 50, 1), gg.zipf(4096, 1.9, 1024, seed=1)]:
        for it in [1, 7, 50]:
            assert abs(oracle.pagerank(g, 0.85, it).sum() - 1.0) < 1e-12


def test_pagerank_threads_identical():
    g = gg.rmat(12, 8, seed=4)
    assert np.array_equal(oracle.pagerank(g, 0.85, 20, threads=1), oracle.pagerank(g, 0.85, 20, threads=4))


# ----------------------------------------------------------------------------
# Algorithm 1 / Section 4.1 mechanism
# ----------------------------------------------------------------------------

def test_figure2_worked_example():
    with open(os.path.join(HERE, "golden", "fig2_cyclic_example.json")) as f:
        fx = json.load(f)
    p = fx["p"]
    degs = fx["huge_degrees"]
    exp = fx["expect"]
    n = len(degs)
    g = gg.from_edges(max(degs) + n + 1, np.repeat(np.arange(n), degs),
                      np.concatenate([np.arange(n + 1, n + 1 + d) for d in degs]))
    work = np.arange(n, dtype=np.int32)
    prefix = oracle.prefix_work(work, g.off)
    assert list(prefix) == [0, 40, 47, 72]
    assert oracle.cyclic_thread(4, p) == exp["thread_of_edge_4"]
    assert oracle.owner(prefix, 4) == exp["owner_of_edge_4"]
    assert [oracle.cyclic_thread(k, p) for k in exp["first_sweep_edges"]] == exp["first_sweep_threads"]
    src, pos, thr = oracle.lb_edges(work, prefix, g.off, p)
    mine = np.flatnonzero(thr == 4)
    assert list(mine) == exp["edges_of_thread_4"]
    assert [oracle.owner(prefix, k) for k in mine] == exp["owners_of_edges_of_thread_4"]


def test_owner_vs_brute_force():
    rng = np.random.default_rng(5)
    for trial in range(60):
        nw = int(rng.integers(1, 40))
        degs = rng.integers(0 if trial % 3 == 0 else 1, 9, nw)
        if degs.sum() == 0:
            degs[-1] = 1
        prefix = np.r_[0, np.cumsum(degs)]
        for k in range(int(prefix[-1])):
            brute = [s for s in range(nw) if prefix[s] <= k < prefix[s + 1]]
            assert len(brute) == 1
            assert oracle.owner(prefix, k) == brute[0]


def test_inspect_bins_and_limits():
    g = gg.rmat(12, 16, seed=7)
    deg = g.degrees()
    fr = np.arange(g.n, dtype=np.int32)[::3]
    for t, cw, cg in [(0, 64, 256), (1, 64, 256), (64, 64, 256), (300, 64, 256), (int(deg.max()), 32, 128),
                      (int(deg.max()) + 1, 64, 256), (np.iinfo(np.int64).max, 64, 256)]:
        bins, work = oracle.inspect(fr, g.off, t, cw, cg)
        d = deg[fr]
        huge = (d >= t) & (d >= 1)
        assert np.array_equal(bins == 3, huge)
        assert np.array_equal(work, fr[huge])
        rest = ~huge
        assert np.array_equal(bins[rest] == 2, d[rest] >= cg)
        assert np.array_equal(bins[rest] == 1, (d[rest] >= cw) & (d[rest] < cg))
        assert np.array_equal(bins[rest] == 0, d[rest] < cw)
        if t == 0:  # threshold 0: every vertex that has an edge is huge (LB for all)
            assert np.array_equal(huge, d >= 1)
        if t > deg.max():  # threshold above the max degree: plain TWC
            assert work.size == 0


def test_prefix_and_lb_edges_cover_each_edge_once():
    g = gg.rmat(11, 16, seed=3)
    deg = g.degrees()
    fr = np.flatnonzero(deg > 0).astype(np.int32)[::2]
    bins, work = oracle.inspect(fr, g.off, 40, 64, 256)
    prefix = oracle.prefix_work(work, g.off)
    assert np.array_equal(prefix, np.r_[0, np.cumsum(deg[work])])
    for p in [1, 7, 64, 1000]:
        src, pos, thr = oracle.lb_edges(work, prefix, g.off, p)
        w = int(prefix[-1])
        # each huge edge exactly once, with the right source
        expect_pos = np.concatenate([np.arange(g.off[v], g.off[v + 1]) for v in work])
        assert np.array_equal(np.sort(pos), np.sort(expect_pos))
        assert np.all((pos >= g.off[src]) & (pos < g.off[src + 1]))
        # cyclic: thread i gets ceil((w - i) / p) edges, consecutive edges on consecutive threads
        cnt = np.bincount(thr, minlength=p)
        i = np.arange(p)
        assert np.array_equal(cnt, np.maximum(0, -(-(w - i) // p)))
        assert np.array_equal(thr, np.arange(w) % p)


def test_blocked_distribution_reading():
    for w, p in [(72, 20), (10, 3), (5, 8), (1000, 64)]:
        c = -(-w // p)
        thr = [oracle.blocked_thread(k, w, p) for k in range(w)]
        for i in range(p):
            mine = [k for k in range(w) if thr[k] == i]
            assert mine == list(range(i * c, min((i + 1) * c, w)))


def test_divergence_bound_two_sources_per_wave():
    """Section 4.1 threshold rule: when every huge vertex has at least W edges,
    W consecutive edges (one wave-wide slice of a cyclic sweep) belong to at
    most two sources."""
    rng = np.random.default_rng(2)
    W = 64
    for _ in range(20):
        degs = rng.integers(W, 5 * W, 30)
        prefix = np.r_[0, np.cumsum(degs)]
        owners = np.array([oracle.owner(prefix, k) for k in range(int(prefix[-1]))])
        for k0 in range(0, int(prefix[-1]) - W, 17):
            assert len(np.unique(owners[k0:k0 + W])) <= 2

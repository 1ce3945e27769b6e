"""GPU parity: the HIP path against the CPU oracle, element by element.

BFS, SSSP and CC labels are unique, so they must be bit-identical to the
oracle in every configuration of the balancer (threshold, workgroup size,
launch mode, grid size, dedup).  PageRank is fp32 on the device against the
fp64 oracle: L1 error <= 1e-5.  The graphs are small enough for the oracle to
run in milliseconds but span many workgroup chunks and ragged tails.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

PR_L1_TOL = 1e-5


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


def _graphs():
    rng_hubs = {0: 30000, 17: 4096, 99: 4095, 1234: 700, 5000: 64, 5001: 63, 5002: 65}
    return {
        "path300": lambda: gg.path(300, w=gg.uniform_ints(299, 100, 5) + 1),
        "cycle257": lambda: gg.cycle(257, w=np.full(257, 3)),
        "star3000": lambda: gg.star(3000, w=gg.uniform_ints(3000, 100, 6) + 1),
        "grid40x50": lambda: gg.grid(40, 50, weight=7),
        "complete70": lambda: gg.complete(70).with_weights(8),
        "edgeless10": lambda: gg.Graph(10, np.zeros(11, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32)),
        "rand5000": lambda: gg.random_digraph(5000, 40000, 3, weighted=True),
        "rmat14": lambda: gg.workload("rmat14").with_weights(2),
        "zipf16": lambda: gg.zipf(1 << 16, 1.9, 1 << 14, seed=3).with_weights(4),
        "hubs": lambda: gg.hub_graph(40000, rng_hubs, 3, seed=11).with_weights(9),
    }


GRAPHS = _graphs()
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


def device_graph(alb, name, symmetric=False):
    key = (name, symmetric)
    if key not in _cache:
        g = graph(name)
        if symmetric:
            _cache[key] = alb.Graph(g.off, g.col, None, build_symmetric=True)
        else:
            _cache[key] = alb.Graph(g.off, g.col, g.w)
    return _cache[key]


def configs(maxdeg):
    """The metamorphic matrix: every cell must give the oracle's answer."""
    out = []
    for thr in [None, "launched", "adaptive", 0, 1, 63, 64, 65, 256, maxdeg, maxdeg + 1, "twc", "lb_all"]:
        for wg in (64, 256, 1024):
            for launch in ("host", "persistent"):
                if thr == "twc":
                    c = dict(mode="twc")
                elif thr == "lb_all":
                    c = dict(mode="lb_all")
                else:
                    c = dict(mode="alb", threshold=thr)
                c.update(wg_size=wg, launch=launch)
                out.append(c)
    # few workgroups: many cyclic sweeps per thread, long grid-stride loops
    out.append(dict(mode="alb", threshold=64, wg_size=64, grid_wgs=3, launch="persistent"))
    out.append(dict(mode="lb_all", wg_size=64, grid_wgs=1, launch="host"))
    out.append(dict(mode="alb", threshold=100, wg_size=256, grid_wgs=7, launch="host"))
    # the blocked distribution (Section 4.1's alternative)
    for thr in (0, 64, 1024):
        for launch in ("host", "persistent"):
            out.append(dict(mode="alb", threshold=thr, distribution=1, launch=launch))
    out.append(dict(mode="lb_all", distribution=1, wg_size=64, grid_wgs=2, launch="persistent"))
    return out


def source_of(g):
    return g.max_degree_vertex() if g.m else 0


@pytest.mark.parametrize("name", list(GRAPHS))
def test_bfs_matrix(alb, name):
    g = graph(name)
    dg = device_graph(alb, name)
    s = source_of(g)
    ref = oracle.bfs(g, s)
    reached = ref < oracle.INF
    m_reached = int(g.degrees()[reached].sum())
    for c in configs(int(g.degrees().max()) if g.m else 0):
        lv, st = alb.bfs(dg, s, **c)
        assert np.array_equal(lv, ref), (name, c)
        # BFS frontiers are the level sets: every reached vertex is active once
        assert st["frontier_vertices"] == int(reached.sum()), (name, c, st)
        assert st["edges_examined"] == m_reached, (name, c, st)
        if c["launch"] == "persistent":
            # the reached-vertex filter (automatic only from 2^23 vertices) forced on
            lv, st = alb.bfs(dg, s, visited_filter=True, **c)
            assert np.array_equal(lv, ref), (name, c, "visited_filter")
            assert st["edges_examined"] == m_reached, (name, c, st)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_sssp_matrix(alb, name):
    g = graph(name)
    dg = device_graph(alb, name)
    s = source_of(g)
    ref = oracle.sssp(g, s)
    for c in configs(int(g.degrees().max()) if g.m else 0):
        d, st = alb.sssp(dg, s, **c)
        assert np.array_equal(d, ref), (name, c)
        if c.get("mode") == "twc":
            assert st["huge_vertices"] == 0
    d, _ = alb.sssp(dg, s, dedup=True, threshold=64)
    assert np.array_equal(d, ref), name
    check_no_dedup(alb, lambda **o: alb.sssp(dg, s, **o)[0], ref, g)


def check_no_dedup(alb, run, ref, g):
    """Without deduplication a vertex can be pushed once per improving edge,
    so a round's worklist is bounded only by the edges examined.  With a
    capacity well above what these graphs push, the run must finish (the
    huge-edge chunk index grows with the capacity) and equal the oracle."""
    got = run(dedup=False, threshold=64, worklist_capacity=64 * (g.n + g.m) + 64)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", list(GRAPHS))
def test_cc_matrix(alb, name):
    g = graph(name)
    dg = device_graph(alb, name, symmetric=True)
    ref = oracle.cc(g)
    for c in configs(dg.max_out_degree):
        lab, _ = alb.cc(dg, **c)
        assert np.array_equal(lab, ref), (name, c)
        if c["launch"] == "persistent":
            # the label-0 filter (on request only) forced on
            lab, _ = alb.cc(dg, visited_filter=True, **c)
            assert np.array_equal(lab, ref), (name, c, "visited_filter")
    check_no_dedup(alb, lambda **o: alb.cc(dg, **o)[0], ref, g)


def reversed_graph(g):
    src = np.repeat(np.arange(g.n), g.degrees())
    return gg.from_edges(g.n, g.col, src)


@pytest.mark.parametrize("name", list(GRAPHS) + ["inhubs"])
def test_pagerank_pull_matrix(alb, name):
    """Pull PageRank over the in-edges: within L1 1e-5 of the fp64 oracle and
    bit-identical to the push version (both sum in exact fixed point)."""
    if name == "inhubs":  # huge in-degrees: the hub graph with every edge reversed
        g = reversed_graph(graph("hubs"))
    else:
        g = graph(name)
    dg = alb.Graph(g.off, g.col, build_transpose=True)
    ref = oracle.pagerank(g, 0.85, 50)
    push, _ = alb.pagerank(dg, 0.85, 50)
    indeg = np.bincount(g.col, minlength=g.n) if g.m else np.zeros(g.n, np.int64)
    maxin = int(indeg.max()) if g.n else 0
    cfgs = [dict()]
    for thr in (0, 1, 64, 1024, maxin, maxin + 1):
        for wg in (64, 256, 1024):
            cfgs.append(dict(threshold=thr, wg_size=wg))
    cfgs += [dict(mode="twc"), dict(mode="lb_all"), dict(threshold=64, grid_wgs=3, wg_size=64),
             dict(wave_cutoff=8, wg_cutoff=100, threshold=5000)]
    for c in cfgs:
        x, st = alb.pagerank_pull(dg, 0.85, 50, **c)
        assert np.abs(x.astype(np.float64) - ref).sum() <= PR_L1_TOL, (name, c)
        assert np.array_equal(x, push), (name, c)
        assert st["rounds"] == 50
    x, _ = alb.pagerank_pull(dg, 0.85, 0)
    assert np.all(x == np.float32(1.0 / g.n))
    with pytest.raises(alb.AlbError):
        alb.pagerank_pull(device_graph(alb, "rmat14"), 0.85, 5)  # no transpose
    dg.close()


@pytest.mark.parametrize("name", list(GRAPHS))
def test_kcore_matrix(alb, name):
    g = gg.symmetrised(graph(name))
    dg = device_graph(alb, name, symmetric=True)
    maxdeg = dg.max_out_degree
    ks = sorted({0, 1, 2, 3, 5, 16, max(1, maxdeg // 2), maxdeg, maxdeg + 1})
    refs = {k: oracle.kcore(g, k) for k in ks}
    for i, c in enumerate(configs(maxdeg)):
        for k in (ks if i % 7 == 0 else ks[1:4]):
            got, st = alb.kcore(dg, k, **c)
            assert np.array_equal(got, refs[k]), (name, k, c)
            if c["launch"] == "persistent" and i % 7 == 0:
                # the left-the-core filter (on request only) forced on
                got, _ = alb.kcore(dg, k, visited_filter=True, **c)
                assert np.array_equal(got, refs[k]), (name, k, c, "visited_filter")


@pytest.mark.parametrize("name", list(GRAPHS))
def test_pagerank_matrix(alb, name):
    g = graph(name)
    dg = device_graph(alb, name)
    ref = oracle.pagerank(g, 0.85, 50)
    for c in configs(int(g.degrees().max()) if g.m else 0)[::3]:
        x, st = alb.pagerank(dg, 0.85, 50, **c)
        err = np.abs(x.astype(np.float64) - ref).sum()
        assert err <= PR_L1_TOL, (name, c, err)
        assert st["rounds"] == 50
    x, _ = alb.pagerank(dg, 0.85, 0)
    assert np.all(x == np.float32(1.0 / g.n))


@pytest.mark.parametrize("name", ["rmat14", "hubs", "star3000"])
def test_pagerank_bitwise_reproducible(alb, name):
    """Sums are exact fixed point, so every configuration gives the same bits."""
    g = graph(name)
    dg = device_graph(alb, name)
    first = None
    for c in configs(int(g.degrees().max())):
        x, _ = alb.pagerank(dg, 0.85, 50, **c)
        if first is None:
            first = x
        assert np.array_equal(x, first), (name, c)


def test_no_dedup_bounded_in_degree(alb):
    """In-degree at most one: pushes per round are bounded by n even without
    deduplication, so the default capacity always suffices."""
    for g in [graph("path300"), graph("cycle257")]:
        dg = alb.Graph(g.off, g.col, g.w)
        for launch in ("host", "persistent"):
            d, _ = alb.sssp(dg, 0, dedup=False, threshold=1, launch=launch)
            assert np.array_equal(d, oracle.sssp(g, 0))
        dg.close()


def test_cc_disjoint_components(alb):
    g = gg.disjoint_copies(gg.star(700), 9)
    dg = alb.Graph(g.off, g.col, None, symmetric=True)
    lab, _ = alb.cc(dg, threshold=64)
    assert np.array_equal(lab, np.repeat(np.arange(9) * 701, 701))
    dg.close()


def test_unreachable_and_single_vertex(alb):
    g = gg.from_edges(6, [0, 1, 3], [1, 2, 4])
    dg = alb.Graph(g.off, g.col, np.ones(g.m, np.int32))
    lv, _ = alb.bfs(dg, 0)
    inf = alb.INF
    assert list(lv) == [0, 1, 2, inf, inf, inf]
    d, _ = alb.sssp(dg, 3)
    assert list(d) == [inf, inf, inf, 0, 1, inf]
    one = alb.Graph(np.zeros(2, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert list(alb.bfs(one, 0)[0]) == [0]
    assert list(alb.sssp(one, 0)[0]) == [0]
    x, _ = alb.pagerank(one, 0.85, 50)
    assert abs(float(x[0]) - 1.0) < 1e-6


def test_device_outputs_on_torch_stream(alb):
    import torch

    g = graph("rmat14")
    dg = device_graph(alb, "rmat14")
    ref = oracle.sssp(g, 0)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        res, st = alb.sssp(dg, 0, out=out, threshold=256)
    s.synchronize()
    assert res is out
    assert np.array_equal(out.cpu().numpy(), ref)
    pr = torch.empty(g.n, dtype=torch.float32, device="cuda")
    alb.pagerank(dg, 0.85, 50, out=pr)
    torch.cuda.synchronize()
    assert np.abs(pr.cpu().numpy().astype(np.float64) - oracle.pagerank(g, 0.85, 50)).sum() <= PR_L1_TOL


def test_option_errors(alb):
    dg = device_graph(alb, "rmat14")
    lv = np.empty(dg.n, np.int32)
    with pytest.raises(alb.AlbError) as e:
        alb.bfs(dg, 0, wg_size=128)
    assert e.value.status == alb.ALB_E_UNSUPPORTED
    with pytest.raises(alb.AlbError) as e:
        alb.bfs(dg, 0, distribution=2)
    assert e.value.status == alb.ALB_E_UNSUPPORTED
    with pytest.raises(alb.AlbError) as e:
        alb.bfs(dg, dg.n)
    assert e.value.status == alb.ALB_E_INVAL
    with pytest.raises(alb.AlbError) as e:
        alb.cc(dg)  # not symmetric
    assert e.value.status == alb.ALB_E_INVAL
    with pytest.raises(alb.AlbError) as e:
        alb.kcore(dg, 2)  # not symmetric
    assert e.value.status == alb.ALB_E_INVAL
    with pytest.raises(alb.AlbError) as e:
        alb.kcore(device_graph(alb, "rmat14", symmetric=True), -1)
    assert e.value.status == alb.ALB_E_INVAL
    with pytest.raises(alb.AlbError) as e:
        alb.bfs(dg, 0, launch="persistent", grid_wgs=10**6)
    assert e.value.status == alb.ALB_E_INVAL
    unweighted = alb.Graph(dg_off(), dg_col())
    with pytest.raises(alb.AlbError) as e:
        alb.sssp(unweighted, 0)
    assert e.value.status == alb.ALB_E_INVAL
    unweighted.close()
    del lv


def dg_off():
    return graph("rmat14").off


def dg_col():
    return graph("rmat14").col


def test_worklist_overflow_reported(alb):
    """A capacity smaller than a round's pushes is reported, not silently truncated."""
    dg = device_graph(alb, "rmat14")
    for launch in ("host", "persistent"):
        with pytest.raises(alb.AlbError) as e:
            alb.bfs(dg, 0, worklist_capacity=8, launch=launch)
        assert e.value.status == alb.ALB_E_OVERFLOW
    # the same graph still works afterwards
    lv, _ = alb.bfs(dg, 0)
    assert np.array_equal(lv, oracle.bfs(graph("rmat14"), 0))


@pytest.mark.parametrize("name", ["rmat14", "zipf16", "hubs", "rand5000"])
def test_default_threshold_follows_the_graph(alb, name):
    """The default huge threshold is m / (20 x workgroups) within [64, 4096],
    and the results under it (with the small-round rule for BFS) are the
    oracle's."""
    g = graph(name)
    dg = device_graph(alb, name)
    d, st = alb.sssp(dg, 0)
    grid = st["launched_threads"] // 256
    assert st["huge_threshold"] == max(64, min(g.m // (20 * grid), 4096))
    assert np.array_equal(d, oracle.sssp(g, 0))
    lv, st = alb.bfs(dg, 0)
    assert st["huge_threshold"] == max(64, min(g.m // (20 * grid), 4096))
    assert np.array_equal(lv, oracle.bfs(g, 0))


@pytest.mark.parametrize("threshold", [None, 64, "twc"])
def test_contended_atomics_fan_in(alb, threshold):
    """Device-scope atomics under contention: 0 -> k middle vertices -> a few
    sinks, so that in one round every workgroup's lanes race on the same
    sink words (SSSP atomic minimum, BFS compare-and-swap, CC on the
    symmetrised graph); every result must equal the oracle's."""
    k, sinks = 200_000, 3
    n = 1 + k + sinks
    rng = np.random.default_rng(17)
    mid = np.arange(1, k + 1)
    src = np.concatenate([np.zeros(k, np.int64), np.repeat(mid, sinks)])
    dst = np.concatenate([mid, np.tile(np.arange(k + 1, n), k)])
    w = rng.integers(1, 10_000, size=src.size)  # max(w) * (n - 1) stays below 2^31
    g = gg.from_edges(n, src, dst, w)
    opts = {"mode": "twc"} if threshold == "twc" else {"threshold": threshold}
    dg = alb.Graph(g.off, g.col, g.w)
    d, _ = alb.sssp(dg, 0, **opts)
    assert np.array_equal(d, oracle.sssp(g, 0))
    lv, _ = alb.bfs(dg, 0, **opts)
    assert np.array_equal(lv, oracle.bfs(g, 0))
    dg.close()
    ds = alb.Graph(g.off, g.col, None, build_symmetric=True)
    lab, _ = alb.cc(ds, **opts)
    assert np.array_equal(lab, oracle.cc(g))
    ds.close()

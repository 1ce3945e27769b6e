"""One traced round on the GPU against the oracle's Algorithm 1 / Algorithm 2
rules: bins, the huge worklist and its prefix, the cyclic thread of every huge
edge, TWC locality, each frontier edge processed exactly once, and the
wave-aggregated pushes."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


@pytest.fixture(scope="module")
def hubgraph():
    hubs = {0: 30000, 17: 4096, 99: 4095, 1234: 700, 5000: 64, 5001: 63, 5002: 65, 7000: 255, 7001: 256, 7002: 257}
    return gg.hub_graph(40000, hubs, 3, seed=11)


def check_round(alb, g, dg, frontier, **opts):
    r = alb.trace_round(dg, frontier, off=g.off, **opts)
    st = r["stats"]
    T = st["launched_threads"]
    t = st["huge_threshold"]
    wg = opts.get("wg_size", 256)
    c_wave = opts.get("wave_cutoff", 64)
    c_wg = opts.get("wg_cutoff", wg)
    bins_ref, work_ref = oracle.inspect(frontier, g.off, t, c_wave, c_wg)
    # Algorithm 1: the same bin for every entry and the same huge set
    assert np.array_equal(r["bins"], bins_ref)
    work = r["work"]
    assert np.array_equal(np.sort(work), np.sort(work_ref))
    # prefixWork: exclusive scan of the huge degrees in the device's worklist order
    assert np.array_equal(r["prefix"], oracle.prefix_work(work, g.off))
    # every edge of the frontier processed exactly once, no other edge touched
    deg = g.degrees()
    expect_hits = np.zeros(g.m, np.int32)
    for v in frontier:
        expect_hits[g.off[v]:g.off[v + 1]] += 1
    assert np.array_equal(r["edge_hits"], expect_hits)
    # Algorithm 2: huge edge k on global thread k mod T (cyclic), or on thread
    # k / ceil(e / T) (blocked)
    src, pos, thr = oracle.lb_edges(work, r["prefix"], g.off, T)
    if opts.get("distribution", 0) == 1:
        e = int(r["prefix"][-1])
        thr = np.array([oracle.blocked_thread(k, e, T) for k in range(e)], np.int64)
    assert np.array_equal(r["edge_thread"][pos], thr.astype(np.int32))
    assert np.array_equal(src, np.repeat(work, deg[work]))
    # TWC: every other edge of a vertex stays inside one workgroup (runs of
    # worklist entries are claimed dynamically, so which workgroup is not
    # fixed); wavefront-bin vertices inside one wavefront
    wg_of = np.full(len(frontier), -1)
    for i, v in enumerate(frontier):
        b = r["bins"][i]
        if b == 3 or deg[v] == 0:
            continue
        th = r["edge_thread"][g.off[v]:g.off[v + 1]]
        wgs = np.unique(th // wg)
        assert len(wgs) == 1, (i, v, b)
        wg_of[i] = int(wgs[0])
        if b == 1:
            assert len(np.unique(th // 64)) == 1
    # claims are runs of at least one wavefront's worth of consecutive entries
    # (the last one may be short): the workgroup changes at most that often
    seq = wg_of[wg_of >= 0]
    assert int((seq[1:] != seq[:-1]).sum()) <= -(-len(frontier) // 64)
    # pushes: every processed edge pushed its destination once
    dsts = np.concatenate([g.col[g.off[v]:g.off[v + 1]] for v in frontier]) if len(frontier) else np.zeros(0)
    assert np.array_equal(np.sort(r["next"]), np.sort(dsts))
    assert st["edges_examined"] == int(deg[frontier].sum())
    assert st["huge_vertices"] == len(work_ref)
    assert st["huge_edges"] == int(deg[work_ref].sum())
    return r


@pytest.mark.parametrize("launch", ["host", "persistent"])
@pytest.mark.parametrize("wg", [64, 256, 1024])
def test_trace_matrix(alb, hubgraph, launch, wg):
    g = hubgraph
    dg = alb.Graph(g.off, g.col)
    rng = np.random.default_rng(wg)
    fronts = [
        np.array([0], np.int32),                                     # one huge vertex (the first-round case)
        np.arange(g.n, dtype=np.int32),                              # everything, many chunks
        rng.choice(g.n, 12345, replace=False).astype(np.int32),      # ragged tail
        np.array([5000, 5001, 5002, 7000, 7001, 7002, 17, 99], np.int32),
    ]
    for fr in fronts:
        for thr in [0, 1, 64, 65, 256, 4096, 30000, 30001, None]:
            check_round(alb, g, dg, fr, threshold=thr, wg_size=wg, launch=launch)
        check_round(alb, g, dg, fr, mode="twc", wg_size=wg, launch=launch)
        check_round(alb, g, dg, fr, mode="lb_all", wg_size=wg, launch=launch)
    dg.close()


def test_trace_small_grid_many_sweeps(alb, hubgraph):
    """T = 64 * 2 threads: each thread walks hundreds of cyclic sweeps."""
    g = hubgraph
    dg = alb.Graph(g.off, g.col)
    fr = np.array([0, 17, 99, 1234, 3], np.int32)
    for launch in ("host", "persistent"):
        r = check_round(alb, g, dg, fr, threshold=64, wg_size=64, grid_wgs=2, launch=launch)
        assert r["stats"]["launched_threads"] == 128
    dg.close()


def test_trace_cutoffs(alb, hubgraph):
    g = hubgraph
    dg = alb.Graph(g.off, g.col)
    fr = np.arange(0, g.n, 3, dtype=np.int32)
    check_round(alb, g, dg, fr, threshold=5000, wave_cutoff=8, wg_cutoff=100)
    check_round(alb, g, dg, fr, threshold=5000, wave_cutoff=1, wg_cutoff=2)
    check_round(alb, g, dg, fr, mode="twc", wave_cutoff=32, wg_cutoff=32)
    dg.close()


def test_two_sources_per_wave_at_default_threshold(alb):
    """With threshold >= 64 a wavefront's 64 consecutive huge edges belong to at
    most two sources (Section 4.1): checked on the traced thread assignment."""
    g = gg.hub_graph(20000, {i * 37: 64 + 13 * i for i in range(60)}, 1, seed=5)
    dg = alb.Graph(g.off, g.col)
    fr = np.array([i * 37 for i in range(60)], np.int32)
    r = check_round(alb, g, dg, fr, threshold=64)
    T = r["stats"]["launched_threads"]
    src, pos, thr = oracle.lb_edges(r["work"], r["prefix"], g.off, T)
    # one sweep of one wavefront: its 64 lanes in the same pass over the grid
    k = np.arange(len(src))
    sweep = (thr // 64) * (len(src) // T + 1) + k // T
    for w in np.unique(sweep):
        assert len(np.unique(src[sweep == w])) <= 2
    dg.close()


@pytest.mark.parametrize("launch", ["host", "persistent"])
def test_trace_blocked_distribution(alb, hubgraph, launch):
    """The blocked alternative of Section 4.1: thread i takes a contiguous run
    of ceil(e / T) huge edges."""
    g = hubgraph
    dg = alb.Graph(g.off, g.col)
    for fr in (np.array([0], np.int32), np.array([0, 17, 99, 1234, 3], np.int32),
               np.arange(g.n, dtype=np.int32)):
        for thr in (0, 64, 4096, None):
            check_round(alb, g, dg, fr, threshold=thr, distribution=1, launch=launch)
        check_round(alb, g, dg, fr, threshold=64, distribution=1, wg_size=64, grid_wgs=2, launch=launch)
    dg.close()

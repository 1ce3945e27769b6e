"""Parity at the benchmark sizes, in the launch configuration bench.py times.

  SSSP on RMAT scale 22 (4.19M vertices, ~65M edges, weights U[1,100]) from
  the highest-degree vertex: every distance equal to Dijkstra's.
  Zipf(1.9) out-degree graph, n = 2^24, degrees capped at 4,194,304 (~372M
  edges): BFS levels equal to the queue BFS, CC labels equal to union-find,
  PageRank (50 iterations, push and pull) within L1 1e-5 of the fp64 oracle.
  k-core membership on the Zipf graph with 2^20 vertices equal to peeling.
  BFS and SSSP on the 2048 x 2048 grid (thousands of rounds, two grid
  barriers each): equal to the oracle's.
"""
import os
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def log(msg):
    print("[%s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


@pytest.fixture(scope="module")
def rmat22w():
    t = time.time()
    g = gg.workload("rmat22w")
    log("rmat22w generated in %.1fs: m=%d" % (time.time() - t, g.m))
    return g


@pytest.fixture(scope="module")
def zipf24():
    t = time.time()
    g = gg.workload("zipf24")
    log("zipf24 generated in %.1fs: m=%d" % (time.time() - t, g.m))
    return g


def test_sssp_rmat22_full(alb, rmat22w):
    g = rmat22w
    s = g.max_degree_vertex()
    t = time.time()
    ref = oracle.sssp(g, s)
    log("oracle dijkstra %.1fs" % (time.time() - t))
    dg = alb.Graph(g.off, g.col, g.w)
    for c in [dict(), dict(threshold=4096), dict(threshold=256), dict(mode="twc"), dict(mode="lb_all"),
              dict(threshold=4096, launch="host"), dict(distribution=1), dict(threshold="adaptive"),
              dict(threshold="launched"), dict(wg_size=1024), dict(grid_wgs=alb.GRID_ALL), dict(dedup=False),
              dict(wave_cutoff=32, wg_cutoff=512)]:
        d, st = alb.sssp(dg, s, **c)
        assert np.array_equal(d, ref), c
        log("sssp %s ok: rounds %d, %.2f ms" % (c, st["rounds"], st["device_ms"]))
    dg.close()


def test_bfs_zipf24_full(alb, zipf24):
    g = zipf24
    s = g.max_degree_vertex()
    t = time.time()
    ref = oracle.bfs(g, s)
    log("oracle bfs %.1fs" % (time.time() - t))
    dg = alb.Graph(g.off, g.col)
    # the default turns the reached-vertex filter on at this size; also without it
    for c in [dict(), dict(threshold=4096), dict(mode="twc"), dict(threshold=4096, launch="host"),
              dict(distribution=1), dict(mode="lb_all"), dict(threshold="adaptive"), dict(wg_size=1024),
              dict(visited_filter=False), dict(mode="twc", visited_filter=False)]:
        lv, st = alb.bfs(dg, s, **c)
        assert np.array_equal(lv, ref), c
        log("bfs %s ok: rounds %d, huge %d, %.2f ms" % (c, st["rounds"], st["huge_vertices"], st["device_ms"]))
    dg.close()


def test_cc_zipf24_full(alb, zipf24):
    g = zipf24
    t = time.time()
    ref = oracle.cc(g)
    log("oracle cc %.1fs" % (time.time() - t))
    t = time.time()
    dg = alb.Graph(g.off, g.col, None, build_symmetric=True)
    log("symmetrised on the host in %.1fs: m=%d" % (time.time() - t, dg.m))
    # also with the label-0 filter (on request only)
    for c in [dict(), dict(threshold=4096), dict(mode="twc"), dict(distribution=1), dict(threshold=64),
              dict(visited_filter=True), dict(mode="twc", visited_filter=True)]:
        lab, st = alb.cc(dg, **c)
        assert np.array_equal(lab, ref), c
        log("cc %s ok: rounds %d, %.2f ms" % (c, st["rounds"], st["device_ms"]))
    dg.close()


def test_kcore_zipf20():
    """k-core on the symmetrised Zipf(1.9) graph with 2^20 vertices (capped at
    2^18; ~46M undirected edge entries): membership equal to the oracle's
    peeling for several k, under the default balancer and TWC only."""
    from paper_1911_09135_amd import alb

    g = gg.zipf(1 << 20, 1.9, 1 << 18, seed=230)
    t = time.time()
    gs = oracle.symmetrised(g)
    log("symmetrised for the oracle in %.1fs: m=%d" % (time.time() - t, gs.m))
    dg = alb.Graph(g.off, g.col, None, build_symmetric=True)
    assert dg.m == gs.m
    for k in (2, 12, 16, 18, 20, 24):  # the core shrinks from almost all vertices to none
        ref = oracle.kcore(gs, k)
        for c in (dict(), dict(mode="twc"), dict(visited_filter=True)):
            got, st = alb.kcore(dg, k, **c)
            assert np.array_equal(got, ref), (k, c)
        log("kcore k=%d ok: %d in core, rounds %d" % (k, int(ref.sum()), st["rounds"]))
    dg.close()


def test_pagerank_zipf24_full(alb, zipf24):
    g = zipf24
    t = time.time()
    ref = oracle.pagerank(g, 0.85, 50, threads=min(16, os.cpu_count() or 1))
    log("oracle pagerank %.1fs" % (time.time() - t))
    dg = alb.Graph(g.off, g.col)
    x0 = None
    for c in [dict(), dict(threshold=4096), dict(mode="twc")]:
        x, st = alb.pagerank(dg, 0.85, 50, **c)
        err = float(np.abs(x.astype(np.float64) - ref).sum())
        assert err <= 1e-5, (c, err)
        if x0 is None:
            x0 = x
        assert np.array_equal(x, x0)
        log("pagerank %s ok: L1 %.2e, %.2f ms" % (c, err, st["device_ms"]))
    dg.close()
    # the pull version over the transposed graph: the same ranks bit for bit
    dt = alb.Graph(g.off, g.col, build_transpose=True)
    for c in [dict(), dict(threshold=22)]:
        x, st = alb.pagerank_pull(dt, 0.85, 50, **c)
        assert np.array_equal(x, x0), c
        log("pagerank pull %s ok: huge %d, %.2f ms" % (c, st["huge_vertices"], st["device_ms"]))
    dt.close()


def test_sssp_batch_rmat_set_full(alb):
    """The batch workload: 256 SSSP queries over 64 weighted RMAT graphs of
    scales 12..20 in one launch (device outputs, as bench.py times it).  32
    queries, spread over every scale, against Dijkstra on their graph alone;
    every query against the single-query call."""
    import torch

    t = time.time()
    graphs = gg.rmat_set(64, 12, 20, seed=7)
    members, sources = gg.query_sources(graphs, 256, seed=8)
    log("64 graphs generated in %.1fs: m=%d" % (time.time() - t, sum(g.m for g in graphs)))
    gs = alb.GraphSet(graphs)
    outs = [torch.empty(graphs[int(m)].n, dtype=torch.int32, device="cuda") for m in members]
    _, st = alb.sssp_batch(gs, members, sources, outs=outs)
    torch.cuda.synchronize()
    log("batch: %d rounds, kernel %.2f ms" % (st["rounds"], st["kernel_ms"]))
    by_scale = {}
    for q, m in enumerate(members):
        by_scale.setdefault(graphs[int(m)].n, []).append(q)
    sample = sorted({qs[k] for qs in by_scale.values() for k in range(min(4, len(qs)))})
    for q in sample:
        g = graphs[int(members[q])]
        ref = oracle.sssp(g, int(sources[q]))
        assert np.array_equal(outs[q].cpu().numpy(), ref), ("query", q, g.n)
    log("%d sampled queries equal Dijkstra" % len(sample))
    for gi, g in enumerate(graphs):
        dg = alb.Graph(g.off, g.col, g.w)
        for q in np.nonzero(members == gi)[0]:
            d, _ = alb.sssp(dg, int(sources[q]))
            assert np.array_equal(d, outs[q].cpu().numpy()), ("query", int(q))
        dg.close()
    gs.close()


def test_grid2048_bfs_sssp_full(alb):
    """The low-skew, high-diameter workload of bench.py --workload zipf24:
    BFS takes 4,095 rounds and SSSP ~4,300, so every barrier's visibility
    guarantee is exercised thousands of times in one launch."""
    g = gg.grid(2048, 2048).with_weights(5)
    dg = alb.Graph(g.off, g.col, g.w)
    for kind, fn, ref in (("bfs", alb.bfs, oracle.bfs), ("sssp", alb.sssp, oracle.sssp)):
        want = ref(g, 0)
        for c in [dict(), dict(mode="twc")]:
            log("grid2048 %s %s" % (kind, c))
            got, st = fn(dg, 0, **c)
            assert st["rounds"] > 4000
            assert np.array_equal(got, want), (kind, c)
    dg.close()

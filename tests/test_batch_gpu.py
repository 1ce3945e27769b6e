"""Query batches on a graph set: every query's labels equal the oracle's on
its member graph alone (bit-exact), whatever the balancer configuration, the
mix of member sizes and the other queries in the launch."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


def _members():
    hubs = {0: 9000, 17: 2048, 99: 1023, 500: 64, 501: 63}
    edgeless = gg.Graph(7, np.zeros(8, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    return [
        gg.rmat(12, seed=101).with_weights(21),
        gg.path(300, w=gg.uniform_ints(299, 100, 5) + 1),
        gg.star(3000, w=gg.uniform_ints(3000, 100, 6) + 1),
        edgeless,
        gg.rmat(10, seed=102).with_weights(22),
        gg.grid(30, 40, weight=7),
        gg.hub_graph(12000, hubs, 3, seed=11).with_weights(9),
        gg.random_digraph(2000, 16000, 3, weighted=True),
        gg.zipf(1 << 14, 1.9, 1 << 12, seed=5).with_weights(4),
    ]


@pytest.fixture(scope="module")
def members():
    return _members()


@pytest.fixture(scope="module")
def gset(alb, members):
    gs = alb.GraphSet(members)
    yield gs
    gs.close()


@pytest.fixture(scope="module")
def queries(members):
    """(member, source) pairs: every member, several sources, repeats, the
    hubs and isolated vertices."""
    qs = []
    for i, g in enumerate(members):
        srcs = [0, g.n - 1, g.max_degree_vertex()]
        srcs += [int(x) for x in gg.uniform_ints(3, g.n, seed=40 + i)]
        qs += [(i, s) for s in srcs]
    qs += [(0, 0), (0, 0), (6, 17)]  # the same query twice in one batch
    mb = np.array([q[0] for q in qs], np.int32)
    src = np.array([q[1] for q in qs], np.int32)
    return mb, src


_ref = {}


def reference(members, kind, mb, s):
    key = (kind, mb, s)
    if key not in _ref:
        g = members[mb]
        _ref[key] = oracle.bfs(g, s) if kind == "bfs" else oracle.sssp(g, s)
    return _ref[key]


def check(members, kind, mb, src, outs):
    assert len(outs) == len(mb)
    for q, (m, s) in enumerate(zip(mb, src)):
        got = outs[q] if isinstance(outs[q], np.ndarray) else outs[q].cpu().numpy()
        assert np.array_equal(got, reference(members, kind, int(m), int(s))), (kind, q, int(m), int(s))


def test_member_table(alb, gset, members):
    base = 0
    assert len(gset.members) == len(members)
    for (n, m, vb), g in zip(gset.members, members):
        assert (n, m, vb) == (g.n, g.m, base)
        base += g.n
    assert gset.n == base and gset.m == sum(g.m for g in members)


CONFIGS = [
    dict(),
    dict(threshold="adaptive"),
    dict(threshold="launched"),
    dict(threshold=0),
    dict(threshold=1),
    dict(threshold=64),
    dict(threshold=1 << 30),
    dict(mode="twc"),
    dict(mode="lb_all"),
    dict(wg_size=64),
    dict(wg_size=1024),
    dict(wg_size=64, grid_wgs=2, threshold=64),
    dict(wg_size=256, grid_wgs=3),
    dict(wave_cutoff=8, wg_cutoff=100, threshold=5000),
    dict(threshold=64, distribution=1),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=[str(c) for c in CONFIGS])
@pytest.mark.parametrize("kind", ["bfs", "sssp"])
def test_batch_matches_oracle(alb, gset, members, queries, kind, cfg):
    mb, src = queries
    fn = alb.bfs_batch if kind == "bfs" else alb.sssp_batch
    outs, st = fn(gset, mb, src, **cfg)
    check(members, kind, mb, src, outs)
    assert st["kernel_launches"] == 1
    assert st["frontier_vertices"] >= len(mb)  # every query's source is active in round 0


@pytest.mark.parametrize("kind", ["bfs", "sssp"])
def test_per_query_thresholds(alb, gset, members, queries, kind):
    mb, src = queries
    fn = alb.bfs_batch if kind == "bfs" else alb.sssp_batch
    rng = np.random.default_rng(3)
    for thr in (np.zeros(len(mb), np.int64),
                rng.choice([0, 1, 64, 65, 1024, 1 << 30], len(mb)).astype(np.int64),
                np.array([gset.members[int(m)][0] for m in mb], np.int64)):
        outs, st = fn(gset, mb, src, thresholds=thr)
        check(members, kind, mb, src, outs)
        assert st["huge_threshold"] == -1


def test_sssp_dedup_off(alb, gset, members, queries):
    mb, src = queries
    outs, _ = alb.sssp_batch(gset, mb, src, dedup=False)
    check(members, "sssp", mb, src, outs)


def test_single_query_batches(alb, gset, members):
    for i, g in enumerate(members):
        s = g.max_degree_vertex()
        for kind, fn in (("bfs", alb.bfs_batch), ("sssp", alb.sssp_batch)):
            outs, st = fn(gset, [i], [s])
            check(members, kind, [i], [s], outs)


def test_batch_equals_single_calls(alb, members, queries):
    """The same queries one at a time through alb_bfs / alb_sssp on each member
    alone give the batch's labels."""
    mb, src = queries
    gs = alb.GraphSet(members)
    outs_b, _ = alb.sssp_batch(gs, mb, src)
    outs_bfs, _ = alb.bfs_batch(gs, mb, src)
    for i, g in enumerate(members):
        dg = alb.Graph(g.off, g.col, g.w)
        for q in np.nonzero(mb == i)[0]:
            d, _ = alb.sssp(dg, int(src[q]))
            l, _ = alb.bfs(dg, int(src[q]))
            assert np.array_equal(d, outs_b[q]) and np.array_equal(l, outs_bfs[q])
        dg.close()
    gs.close()


def test_device_outputs(alb, gset, members, queries):
    import torch

    mb, src = queries
    outs = [torch.full((gset.members[int(m)][0],), -7, dtype=torch.int32, device="cuda") for m in mb]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        alb.sssp_batch(gset, mb, src, outs=outs)
    s.synchronize()
    check(members, "sssp", mb, src, outs)


def test_repeated_calls_reuse_workspace(alb, gset, members, queries):
    mb, src = queries
    alb.bfs_batch(gset, mb, src)
    b0 = gset.device_bytes()
    for k in (len(mb), 5, len(mb)):
        outs, _ = alb.bfs_batch(gset, mb[:k], src[:k])
        check(members, "bfs", mb[:k], src[:k], outs)
    assert gset.device_bytes() == b0


def test_batch_errors(alb, gset, members, queries):
    mb, src = queries
    with pytest.raises(alb.AlbError, match="out of range"):
        alb.bfs_batch(gset, [0], [members[0].n])
    with pytest.raises(alb.AlbError, match="out of range"):
        alb.bfs_batch(gset, [len(members)], [0])
    with pytest.raises(alb.AlbError, match="persistent"):
        alb.bfs_batch(gset, mb, src, launch="host")
    with pytest.raises(alb.AlbError, match="mode ALB"):
        alb.bfs_batch(gset, mb, src, thresholds=np.zeros(len(mb), np.int64), mode="twc")
    with pytest.raises(alb.AlbError, match=">= 0"):
        alb.bfs_batch(gset, mb, src, thresholds=np.full(len(mb), -1, np.int64))
    with pytest.raises(alb.AlbError, match="capacity"):
        alb.sssp_batch(gset, mb, src, worklist_capacity=len(mb))
    # the handle still works after each refusal
    outs, _ = alb.sssp_batch(gset, mb, src)
    check(members, "sssp", mb, src, outs)


def test_unweighted_set_refuses_sssp(alb):
    gs = alb.GraphSet([gg.rmat(8, seed=3), gg.path(10)], weighted=False)
    with pytest.raises(alb.AlbError, match="weights"):
        alb.sssp_batch(gs, [0], [0])
    outs, _ = alb.bfs_batch(gs, [0, 1], [0, 0])
    assert np.array_equal(outs[1], np.arange(10, dtype=np.int32))
    gs.close()


def test_single_calls_on_a_set_work_on_the_union(alb, members):
    gs = alb.GraphSet(members[:3])
    lv, _ = alb.bfs(gs, 0)
    n0 = members[0].n
    assert np.array_equal(lv[:n0], oracle.bfs(members[0], 0))
    assert (lv[n0:] == alb.INF).all()
    gs.close()


def test_maximum_batch_count(alb):
    """65,535 queries (the most one launch takes) on a small graph, every
    result checked; one more query is refused."""
    p = gg.path(10)
    gs = alb.GraphSet([p, gg.star(5)], weighted=False)
    count = 65535
    mb = (np.arange(count) % 3 == 2).astype(np.int32)
    src = (np.arange(count) % 5).astype(np.int32)
    outs, st = alb.bfs_batch(gs, mb, src)
    refs = {(m, s): oracle.bfs(p if m == 0 else gg.star(5), s) for m in (0, 1) for s in range(5)}
    for q in range(count):
        assert np.array_equal(outs[q], refs[(int(mb[q]), int(src[q]))]), q
    with pytest.raises(alb.AlbError, match="count"):
        alb.bfs_batch(gs, np.zeros(count + 1, np.int32), np.zeros(count + 1, np.int32))
    gs.close()

"""Batch plans (a batch captured into a HIP graph and replayed) and the
autotuner: every replay and every tuned setting gives the oracle's labels."""
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
def members():
    return [
        gg.rmat(12, seed=101).with_weights(21),
        gg.star(3000, w=gg.uniform_ints(3000, 100, 6) + 1),
        gg.rmat(10, seed=102).with_weights(22),
        gg.hub_graph(12000, {0: 9000, 17: 2048, 99: 1023}, 3, seed=11).with_weights(9),
        gg.zipf(1 << 14, 1.9, 1 << 12, seed=5).with_weights(4),
    ]


@pytest.fixture(scope="module")
def gset(alb, members):
    gs = alb.GraphSet(members)
    yield gs


@pytest.fixture(scope="module")
def queries(members):
    mb, src = gg.query_sources(members, 23, seed=8)
    return mb, src


def expected(members, kind, mb, src):
    f = oracle.bfs if kind == "bfs" else oracle.sssp
    return [f(members[int(m)], int(s)) for m, s in zip(mb, src)]


def same(outs, ref):
    for o, r in zip(outs, ref):
        got = o if isinstance(o, np.ndarray) else o.cpu().numpy()
        if not np.array_equal(got, r):
            return False
    return True


@pytest.mark.parametrize("kind", ["bfs", "sssp"])
def test_plan_replays_match_oracle(alb, gset, members, queries, kind):
    """Each replay is checked; eager batches on the same graph run between
    replays and must not disturb them."""
    import torch

    mb, src = queries
    ref = expected(members, kind, mb, src)
    outs = [torch.full((gset.members[int(m)][0],), -5, dtype=torch.int32, device="cuda") for m in mb]
    plan = alb.BatchPlan(gset, kind, mb, src, outs=outs)
    eager = alb.bfs_batch if kind == "sssp" else alb.sssp_batch  # the other algorithm
    for rep in range(4):
        for o in outs:
            o.fill_(-5)
        res, st = plan.run()
        assert same(res, ref), rep
        assert st["kernel_launches"] == 1 and st["rounds"] > 0
        eager(gset, mb[::-1], src[::-1])  # other work on the same graph in between
        torch.cuda.synchronize()
    plan.close()


def test_plan_host_outputs_and_thresholds(alb, gset, members, queries):
    mb, src = queries
    ref = expected(members, "sssp", mb, src)
    thr = np.array([0, 1, 64, 4096, 1 << 30] * 5, np.int64)[: len(mb)]
    plan = alb.BatchPlan(gset, "sssp", mb, src, thresholds=thr)
    for _ in range(3):
        res, st = plan.run()
        assert same(res, ref)
        assert st["huge_threshold"] == -1
    plan.close()


def test_graph_destroy_refused_while_plan_lives(alb, members):
    gs = alb.GraphSet(members[:2])
    plan = alb.BatchPlan(gs, "bfs", [0, 1], [0, 0])
    assert alb._lib.alb_graph_destroy(gs.handle) == alb.ALB_E_INVAL
    plan.close()
    gs.close()


def test_autotune_single_graph(alb, members):
    g = members[0]
    dg = alb.Graph(g.off, g.col, g.w)
    alb.autotune_reset()
    srcs = gg.query_sources([g], 4, seed=3)[1]
    opts, ms = alb.autotune(dg, "sssp", srcs)
    assert opts["wg_size"] in (256, 1024) and opts["threshold"] in (64, 256, 1024, 4096, 16384)
    assert opts["wave_cutoff"] >= 1 and opts["wg_cutoff"] >= 1 and ms > 0
    for s in srcs:
        d, _ = alb.sssp(dg, int(s), **opts)
        assert np.array_equal(d, oracle.sssp(g, int(s)))
    # a graph with the same degree signature reuses the cached result
    opts2, ms2 = alb.autotune(dg, "sssp", srcs[:1])
    assert opts2 == opts and ms2 == ms
    dg.close()


@pytest.mark.parametrize("kind", ["bfs", "sssp"])
def test_autotune_batch(alb, gset, members, queries, kind):
    mb, src = queries
    opts, thr = alb.autotune_batch(gset, kind, mb, src)
    assert thr.shape == (len(mb),) and (thr >= 0).all()
    fn = alb.bfs_batch if kind == "bfs" else alb.sssp_batch
    outs, _ = fn(gset, mb, src, thresholds=thr, **opts)
    assert same(outs, expected(members, kind, mb, src))


@pytest.mark.parametrize("kind", ["bfs", "sssp"])
def test_per_query_cutoffs(alb, gset, members, queries, kind):
    """Per-query thresholds and TWC cutoffs, eager and as a plan: extreme
    cutoffs (everything in one bin) and mixed ones, all equal to the oracle;
    invalid cutoffs are refused."""
    mb, src = queries
    ref = expected(members, kind, mb, src)
    cand = [(64, 64, 256), (1 << 30, 1, 1), (1 << 30, 1 << 30, 1 << 30), (0, 64, 256), (256, 32, 512),
            (4096, 128, 1024), (1, 1 << 30, 2)]
    tuning = [cand[i % len(cand)] for i in range(len(mb))]
    fn = alb.bfs_batch_tuned if kind == "bfs" else alb.sssp_batch_tuned
    outs, st = fn(gset, mb, src, tuning)
    assert same(outs, ref)
    assert st["huge_threshold"] == -1
    for extreme in [(64, 1, 1), (64, 1 << 30, 1 << 30)]:
        outs, _ = fn(gset, mb, src, [extreme] * len(mb))
        assert same(outs, ref), extreme
    plan = alb.BatchPlan(gset, kind, mb, src, tuning=tuning)
    for _ in range(2):
        res, _ = plan.run()
        assert same(res, ref)
    plan.close()
    with pytest.raises(alb.AlbError) as ei:
        fn(gset, mb, src, [(64, 0, 256)] * len(mb))
    assert ei.value.status == alb.ALB_E_INVAL


def test_autotune_batch_with_cutoffs(alb, gset, members, queries):
    mb, src = queries
    opts, tuning, uniform_ms, tuned_ms = alb.autotune_batch_tuned(gset, "sssp", mb, src)
    assert len(tuning) == len(mb)
    assert all(t >= 0 and cw >= 1 and cg >= 1 for t, cw, cg in tuning)
    assert 0 < tuned_ms <= uniform_ms  # kept settings only ever gain
    outs, _ = alb.sssp_batch_tuned(gset, mb, src, tuning, **opts)
    assert same(outs, expected(members, "sssp", mb, src))

"""The serving loop on the GPU: a mix of BFS and SSSP requests on a graph set,
submitted faster than they complete, so that they batch and the lanes'
batches overlap on the device; every result equals the oracle's, and the
same request alone gives the same result as in the mix."""
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
        gg.rmat(13, seed=201).with_weights(31),
        gg.rmat(11, seed=202).with_weights(32),
        gg.zipf(1 << 14, 1.9, 1 << 12, seed=5).with_weights(4),
        gg.star(3000, w=gg.uniform_ints(3000, 100, 6) + 1),
        gg.path(500, w=gg.uniform_ints(499, 100, 7) + 1),
    ]


@pytest.fixture(scope="module")
def gset(alb, members):
    return alb.GraphSet(members)


def requests(members, count, seed):
    mb, src = gg.query_sources(members, count, seed=seed)
    rng = np.random.default_rng(seed)
    algo = np.where(rng.random(count) < 0.5, "bfs", "sssp")
    return list(zip(algo, mb.tolist(), src.tolist()))


def reference(members, algo, m, s, cache={}):
    key = (algo, m, s)
    if key not in cache:
        cache[key] = (oracle.bfs if algo == "bfs" else oracle.sssp)(members[m], s)
    return cache[key]


@pytest.mark.parametrize("lanes,max_batch", [(1, 256), (2, 256), (3, 7)])
def test_mix_matches_oracle(alb, gset, members, lanes, max_batch):
    reqs = requests(members, 120, seed=lanes)
    with alb.Server(gset, lanes=lanes, max_batch=max_batch) as srv:
        tickets = [srv.submit(a, m, s) for a, m, s in reqs]
        sizes = []
        for t, (a, m, s) in zip(tickets, reqs):
            out, info = srv.wait(t)
            assert np.array_equal(out, reference(members, a, m, s)), (a, m, s)
            sizes.append(info["batch_size"])
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert max(sizes) > 1  # requests queued behind a running batch were batched
    assert max(sizes) <= max_batch


def test_same_alone_and_in_the_mix(alb, gset, members):
    reqs = requests(members, 40, seed=11)
    with alb.Server(gset, lanes=2) as srv:
        alone = []
        for a, m, s in reqs:
            out, info = srv.wait(srv.submit(a, m, s))
            assert info["batch_size"] == 1
            alone.append(out)
        tickets = [srv.submit(a, m, s) for a, m, s in reqs]
        for t, ref in zip(tickets, alone):
            out, _ = srv.wait(t)
            assert np.array_equal(out, ref)


def test_small_budget_splits_batches(alb, gset, members):
    n0 = members[0].n
    budget = 2 * 2 * (44 * n0 + 64)  # two lanes, two requests of member 0 per batch
    with alb.Server(gset, lanes=2, hbm_budget=budget) as srv:
        reqs = [("sssp", 0, int(s)) for s in gg.query_sources([members[0]], 9, seed=2)[1]]
        tickets = [srv.submit(*r) for r in reqs]
        for t, (a, m, s) in zip(tickets, reqs):
            out, info = srv.wait(t)
            assert info["batch_size"] <= 2
            assert np.array_equal(out, reference(members, a, m, s))


def test_lanes_overlap_on_the_device(alb, gset, members):
    """Batches of two lanes run on the device at the same time: their
    persistent launches' device windows (first workgroup joined to last
    round left, on the device's wall clock) intersect; every result is still
    the oracle's."""
    reqs = [("sssp", 0, int(s)) for s in gg.query_sources([members[0]], 64, seed=21)[1]]
    with alb.Server(gset, lanes=2, max_batch=4, whole_device_when_alone=False) as srv:
        tickets = [srv.submit(*r) for r in reqs]
        for t, (a, m, s) in zip(tickets, reqs):
            out, _ = srv.wait(t)
            assert np.array_equal(out, reference(members, a, m, s))
        log = srv.batch_log()
    assert len(log) >= 2 and {r["lane"] for r in log} == {0, 1}
    assert all(0 < r["device_begin_ms"] <= r["device_end_ms"] for r in log)
    pairs = [(a, b) for a in log for b in log if a["lane"] == 0 and b["lane"] == 1 and
             a["device_begin_ms"] < b["device_end_ms"] and b["device_begin_ms"] < a["device_end_ms"]]
    print("batches %d, overlapping lane pairs %d" % (len(log), len(pairs)))
    assert pairs, log


@pytest.mark.parametrize("lanes,max_batch", [(1, 64), (2, 256)])
def test_join_running_matches_oracle(alb, gset, members, lanes, max_batch):
    """Continuous batching inside a launch: every result equals the oracle's."""
    reqs = requests(members, 150, seed=30 + lanes)
    with alb.Server(gset, lanes=lanes, max_batch=max_batch, join_running=True) as srv:
        tickets = [srv.submit(a, m, s) for a, m, s in reqs]
        for t, (a, m, s) in zip(tickets, reqs):
            out, info = srv.wait(t)
            assert np.array_equal(out, reference(members, a, m, s)), (a, m, s)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0


def test_requests_join_a_running_launch(alb, gset, members):
    """Requests submitted while a launch is on the device join it between
    rounds: two waves of SSSP requests, the second submitted after the first
    has completed but while the launch is still running (a long idle window),
    are served by ONE launch that admitted all of them; results equal the
    oracle's, also for a slot reused by the second wave."""
    import time

    srcs = gg.query_sources([members[0]], 24, seed=41)[1]
    wave1 = [("sssp", 0, int(s)) for s in srcs[:12]]
    wave2 = [("sssp", 0, int(s)) for s in srcs[12:]] + [("sssp", 2, 5), ("sssp", 4, 0)]
    with alb.Server(gset, lanes=1, max_batch=16, join_running=True, join_idle_us=2_000_000) as srv:
        t1 = [srv.submit(*r) for r in wave1]
        for t, r in zip(t1, wave1):
            out, _ = srv.wait(t)
            assert np.array_equal(out, reference(members, *r))
        time.sleep(0.05)
        assert srv.batch_log() == []  # the launch is still running (its record is written when it ends)
        t2 = [srv.submit(*r) for r in wave2]
        for t, r in zip(t2, wave2):
            out, info = srv.wait(t)
            assert np.array_equal(out, reference(members, *r))
        deadline = time.time() + 10
        while not srv.batch_log() and time.time() < deadline:
            time.sleep(0.05)
        log = srv.batch_log()
    assert len(log) == 1, log
    assert log[0]["batch_size"] == len(wave1) + len(wave2) and log[0]["status"] == 0
    assert 0 < log[0]["device_begin_ms"] < log[0]["device_end_ms"]


@pytest.mark.parametrize("lanes", [1, 2])
def test_join_running_writes_pinned_outputs(alb, gset, members, lanes):
    """Continuous batching with outputs in pinned host memory: the launch
    converts a finished query's labels straight into the request's array
    (no host copy); pinned and pageable outputs mixed in one launch, every
    array pre-filled with a value no result holds, all equal the oracle."""
    import torch

    reqs = requests(members, 120, seed=50 + lanes)
    outs = []
    for i, (a, m, s) in enumerate(reqs):
        n = members[m].n
        if i % 3 == 2:
            o = np.full(n, -7, np.int32)  # pageable: the staged copy
        else:
            o = torch.full((n,), -7, dtype=torch.int32, pin_memory=True).numpy()
        outs.append(o)
    with alb.Server(gset, lanes=lanes, max_batch=64, join_running=True) as srv:
        tickets = [srv.submit(a, m, s, out=o) for (a, m, s), o in zip(reqs, outs)]
        for t, (a, m, s), o in zip(tickets, reqs, outs):
            got, _ = srv.wait(t)
            assert got is o
            assert np.array_equal(o, reference(members, a, m, s)), (a, m, s)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["direct_outputs"] == sum(1 for i in range(len(reqs)) if i % 3 != 2)


def test_join_running_edge_sources_and_deadlines(alb, gset, members):
    """Join mode on sources that end at once or run long: the directed path's
    last vertex (no out-edges) and first vertex (499 rounds), the star's
    centre and a leaf, an RMAT vertex without out-edges; then four 499-round
    path queries hold every slot and a request queued behind them with a 1 ms
    deadline completes as timed out, while the four still equal the oracle."""
    deg0 = np.nonzero(members[0].degrees() == 0)[0]
    iso = int(deg0[0]) if deg0.size else 0
    reqs = [("bfs", 4, 499), ("sssp", 4, 499), ("bfs", 4, 0), ("sssp", 4, 0), ("sssp", 3, 0), ("bfs", 3, 7),
            ("sssp", 0, iso), ("bfs", 0, iso)]
    with alb.Server(gset, lanes=1, max_batch=4, join_running=True) as srv:
        tickets = [srv.submit(*r) for r in reqs]
        for t, r in zip(tickets, reqs):
            out, _ = srv.wait(t)
            assert np.array_equal(out, reference(members, *r)), r
        long = [srv.submit("sssp", 4, 0) for _ in range(4)]
        late = srv.submit("bfs", 1, 0, timeout_ms=1)
        with pytest.raises(alb.AlbError) as e:
            srv.wait(late)
        assert e.value.status == alb.ALB_E_TIMEOUT
        for t in long:
            out, _ = srv.wait(t)
            assert np.array_equal(out, reference(members, "sssp", 4, 0))
        st = srv.stats()
    assert st["timed_out"] == 1 and st["failed"] == 0 and st["completed"] == len(reqs) + 4


@pytest.mark.parametrize("opts", [dict(threshold=64, wave_cutoff=32, wg_cutoff=512),
                                  dict(threshold=64, distribution=1), dict(mode="twc")])
def test_join_running_with_traversal_options(alb, gset, members, opts):
    """The serving launch takes the server's traversal options: a low huge
    threshold with other TWC cutoffs, the blocked distribution of huge
    edges, TWC only; every result equals the oracle's."""
    reqs = requests(members, 60, seed=70)
    with alb.Server(gset, lanes=1, max_batch=32, join_running=True, **opts) as srv:
        tickets = [srv.submit(a, m, s) for a, m, s in reqs]
        for t, (a, m, s) in zip(tickets, reqs):
            out, _ = srv.wait(t)
            assert np.array_equal(out, reference(members, a, m, s)), (a, m, s, opts)


def test_join_running_long_and_short_lanes(alb, gset, members):
    """join_long_edges: requests on the member with the most edges run on
    lane 0, all others on lane 1, each lane keeping its own running launch;
    every result equals the oracle's."""
    big = int(np.argmax([g.m for g in members]))
    reqs = requests(members, 120, seed=90)
    with alb.Server(gset, lanes=2, max_batch=64, join_running=True, join_long_edges=members[big].m) as srv:
        tickets = [srv.submit(a, m, s) for a, m, s in reqs]
        for t, (a, m, s) in zip(tickets, reqs):
            out, info = srv.wait(t)
            assert np.array_equal(out, reference(members, a, m, s)), (a, m, s)
            assert info["lane"] == (0 if m == big else 1), (m, info)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0

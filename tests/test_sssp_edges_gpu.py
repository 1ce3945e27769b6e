"""SSSP at the edges of what the library accepts: zero weights (zero-weight
cycles included) and the largest distances graph creation admits, where
max(w) * (n - 1) = INT32_MAX - 1 and relaxations out of the farthest vertex
offer candidates beyond INT32_MAX.  Every result must equal the oracle's
(int64 Dijkstra), bit for bit, single queries and batches alike."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


def configs():
    out = []
    for thr in (None, 0, 1, 64, "twc"):
        for launch in ("host", "persistent"):
            c = dict(mode="twc") if thr == "twc" else dict(threshold=thr)
            c["launch"] = launch
            out.append(c)
    out.append(dict(threshold=64, wg_size=1024))
    out.append(dict(threshold=1, distribution=1))
    out.append(dict(threshold=64, dedup=False, worklist_capacity=1 << 22))
    return out


def zero_weight_graphs():
    return {
        "rmat14_w0-3": gg.workload("rmat14").with_weights(31, 0, 3),
        "zipf15_w0-1": gg.zipf(1 << 15, 1.9, 1 << 13, seed=8).with_weights(32, 0, 1),
        "rand3000_w0": gg.random_digraph(3000, 30000, 5).with_weights(33, 0, 0),
        "cycle300_w0": gg.cycle(300, w=np.zeros(300, np.int64)),
        "grid30x30_w0-2": gg.grid(30, 30, weight=1).with_weights(34, 0, 2),
    }


def boundary_graphs():
    # 2^31 - 2 = 2 * 3^2 * 7 * 11 * 31 * 151 * 331: n - 1 = 62 and 21,483 divide it
    return {
        "path63": gg.boundary_path(63, 500, seed=4, hub_back=62),
        "path21484": gg.boundary_path(21484, 200_000, seed=5, hub_back=6000),
    }


@pytest.mark.parametrize("kind", ["zero", "boundary"])
def test_sssp_single(alb, kind):
    graphs = zero_weight_graphs() if kind == "zero" else boundary_graphs()
    for name, g in graphs.items():
        if kind == "boundary":
            assert int(g.w.max()) * (g.n - 1) == 2 ** 31 - 2, name
        dg = alb.Graph(g.off, g.col, g.w)
        for s in sorted({0, g.max_degree_vertex(), g.n - 1}):
            ref = oracle.sssp(g, s)
            for c in configs():
                if g.n > 10_000 and c.get("launch") == "host":
                    continue  # ~21K rounds: one launch per phase per round is slow, not different
                d, _ = alb.sssp(dg, s, **c)
                assert np.array_equal(d, ref), (name, s, c)
        dg.close()


def test_boundary_distances_reach_int32_max_minus_one(alb):
    g = boundary_graphs()["path21484"]
    dg = alb.Graph(g.off, g.col, g.w)
    d, _ = alb.sssp(dg, 0)
    W = (2 ** 31 - 2) // (g.n - 1)
    assert np.array_equal(d.astype(np.int64), np.arange(g.n, dtype=np.int64) * W)
    assert int(d[-1]) == 2 ** 31 - 2
    dg.close()
    # one more unit of weight on a path edge is refused at creation
    w = g.w.copy()
    w[0] = W + 1
    with pytest.raises(alb.AlbError) as e:
        alb.Graph(g.off, g.col, w)
    assert e.value.status == alb.ALB_E_RANGE


def test_sssp_batch_edges(alb):
    """Zero-weight and boundary members in one batch, next to ordinary ones."""
    members = list(zero_weight_graphs().values()) + list(boundary_graphs().values())
    members.append(gg.rmat(12, seed=101).with_weights(21))
    gs = alb.GraphSet(members)
    mem, src = [], []
    for i, g in enumerate(members):
        for s in sorted({0, g.max_degree_vertex(), g.n - 1}):
            mem.append(i)
            src.append(s)
    refs = [oracle.sssp(members[m], s) for m, s in zip(mem, src)]
    for opts in (dict(), dict(threshold=1), dict(mode="twc"), dict(threshold=64, wg_size=1024)):
        outs, _ = alb.sssp_batch(gs, mem, src, **opts)
        for q, (o, r) in enumerate(zip(outs, refs)):
            assert np.array_equal(o, r), (q, mem[q], src[q], opts)
    gs.close()

"""Input generators: determinism, CSR well-formedness and the sampled laws."""
import numpy as np
import pytest

import graphgen as gg


def check_csr(g):
    assert g.off.dtype == np.int32 and g.col.dtype == np.int32
    assert g.off[0] == 0 and g.off[-1] == g.m
    assert np.all(np.diff(g.off) >= 0)
    if g.m:
        assert g.col.min() >= 0 and g.col.max() < g.n
    src = np.repeat(np.arange(g.n), g.degrees())
    assert not np.any(src == g.col), "self-loop"
    key = src.astype(np.int64) * g.n + g.col
    assert np.all(np.diff(key) > 0), "rows not sorted or duplicate edge"


def test_rmat_deterministic_and_wellformed():
    a = gg.rmat(10, 16, seed=1)
    b = gg.rmat(10, 16, seed=1)
    c = gg.rmat(10, 16, seed=2)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.col, b.col)
    assert not (np.array_equal(a.off, c.off) and np.array_equal(a.col, c.col))
    check_csr(a)
    assert a.n == 1024 and 0 < a.m <= 16 * 1024
    # no noise, no permutation: vertex 0 is the hub
    assert a.max_degree_vertex() == 0


def test_rmat14_sizes():
    g = gg.workload("rmat14")
    check_csr(g)
    assert g.n == 16384
    assert 200_000 < g.m < 262_144
    assert g.max_degree_vertex() == 0


def test_zipf_degree_law():
    s, cap, n = 1.9, 1000, 400_000
    d = gg.zipf_degrees(n, s, cap, seed=3)
    assert d.min() == 1 and d.max() == cap
    k = np.arange(1, 200_000, dtype=np.float64)
    zeta = (k ** -s).sum() + 200_000 ** (1 - s) / (s - 1)
    p1 = 1.0 / zeta
    assert abs((d == 1).mean() - p1) < 4 * np.sqrt(p1 * (1 - p1) / n)
    p2 = 2 ** -s / zeta
    assert abs((d == 2).mean() - p2) < 4 * np.sqrt(p2 * (1 - p2) / n)
    tail = 1.0 - (np.arange(1, cap, dtype=np.float64) ** -s).sum() / zeta
    assert abs((d == cap).mean() - tail) < 4 * np.sqrt(tail / n) + 1e-6


def test_zipf_graph_wellformed():
    g = gg.zipf(1 << 14, 1.9, 1 << 12, seed=3)
    check_csr(g)
    g2 = gg.zipf(1 << 14, 1.9, 1 << 12, seed=3)
    assert np.array_equal(g.col, g2.col)


def test_weights_range_and_determinism():
    w = gg.uniform_weights(100_000, seed=2, lo=1, hi=100)
    assert w.min() == 1 and w.max() == 100
    assert np.array_equal(w, gg.uniform_weights(100_000, seed=2, lo=1, hi=100))
    counts = np.bincount(w, minlength=101)[1:]
    assert counts.min() > 800


@pytest.mark.parametrize("builder", [lambda: gg.path(9), lambda: gg.cycle(9), lambda: gg.star(9),
                                     lambda: gg.grid(4, 5), lambda: gg.complete(6),
                                     lambda: gg.random_digraph(50, 200, 3),
                                     lambda: gg.disjoint_copies(gg.cycle(5), 3)])
def test_families_wellformed(builder):
    check_csr(builder())


def test_from_edges_dedup_keeps_first_weight():
    g = gg.from_edges(3, [0, 0, 1, 0], [1, 1, 2, 2], w=[5, 7, 3, 1])
    assert list(g.off) == [0, 2, 3, 3]
    assert list(g.col) == [1, 2, 2]
    assert list(g.w) == [5, 1, 3]

"""Seeded synthetic graph inputs.

This module only builds inputs (CSR arrays, weights, source choices).  It holds
none of the traversal or load-balancing arithmetic; the GPU library and the
CPU oracle both consume what it produces, and neither is imported here.

Generated graphs follow one recipe everywhere: CSR with int32 offsets and
int32 columns, rows sorted by destination, self-loops and duplicate edges
removed.  Randomness is counter-based (SplitMix64 finaliser over
(seed, stream, index)), so results do not depend on thread counts.

The workloads mirror the paper's inputs (Table 2 power-law graphs, Section 5):
  * RMAT with Graph500 parameters (a, b, c) = (0.57, 0.19, 0.19), no noise and
    no vertex permutation, so vertex 0 is the hub;
  * a capped-Zipf out-degree graph with uniform random targets, the stand-in
    for the paper's extreme out-degree skew (rmat25's 125.7M max out-degree);
  * small families with closed-form answers (path, cycle, star, grid, ...).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, u64]
        lib.gg_zipf.restype = vp
        lib.gg_zipf.argtypes = [i32, dbl, i64, u64]
        lib.gg_zipf_degrees.restype = ctypes.c_int
        lib.gg_zipf_degrees.argtypes = [i32, dbl, i64, u64, vp]
        lib.gg_n.restype = i32
        lib.gg_n.argtypes = [vp]
        lib.gg_m.restype = i64
        lib.gg_m.argtypes = [vp]
        lib.gg_fetch.restype = None
        lib.gg_fetch.argtypes = [vp, vp, vp]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        lib.gg_uniform_weights.restype = None
        lib.gg_uniform_weights.argtypes = [i64, i32, i32, u64, vp]
        lib.gg_uniform_ints.restype = None
        lib.gg_uniform_ints.argtypes = [i64, ctypes.c_uint32, u64, u64, vp]
        lib.gg_uniform_doubles.restype = None
        lib.gg_uniform_doubles.argtypes = [i64, u64, u64, vp]
        lib.gg_draw.restype = u64
        lib.gg_draw.argtypes = [u64, u64, u64]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Graph:
    """A directed graph in CSR form (int32 offsets n+1, int32 columns m)."""

    n: int
    off: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray] = None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.off.astype(np.int64))

    def with_weights(self, seed: int, lo: int = 1, hi: int = 100) -> "Graph":
        return Graph(self.n, self.off, self.col, uniform_weights(self.m, seed, lo, hi), self.name)

    def max_degree_vertex(self) -> int:
        """Highest out-degree vertex, lowest id on ties."""
        d = self.degrees()
        return int(np.argmax(d)) if self.n else 0


def _from_handle(h, name: str) -> Graph:
    lib = _load()
    if not h:
        raise MemoryError("graph generation failed (allocation or int32 overflow)")
    try:
        n = lib.gg_n(h)
        m = lib.gg_m(h)
        off = np.empty(n + 1, dtype=np.int32)
        col = np.empty(max(m, 0), dtype=np.int32)
        lib.gg_fetch(h, _ptr(off), _ptr(col))
    finally:
        lib.gg_free(h)
    return Graph(n, off, col, None, name)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1) -> Graph:
    lib = _load()
    h = lib.gg_rmat(scale, edge_factor, a, b, c, seed)
    return _from_handle(h, "rmat%d_ef%d_s%d" % (scale, edge_factor, seed))


def zipf(n: int, s: float = 1.9, cap: int = 4194304, seed: int = 3) -> Graph:
    lib = _load()
    h = lib.gg_zipf(n, s, cap, seed)
    return _from_handle(h, "zipf%.2f_n%d_cap%d_s%d" % (s, n, cap, seed))


def zipf_degrees(n: int, s: float, cap: int, seed: int) -> np.ndarray:
    lib = _load()
    deg = np.empty(n, dtype=np.int64)
    if lib.gg_zipf_degrees(n, s, cap, seed, _ptr(deg)) != 0:
        raise ValueError("bad Zipf parameters")
    return deg


def uniform_weights(m: int, seed: int, lo: int = 1, hi: int = 100) -> np.ndarray:
    lib = _load()
    w = np.empty(m, dtype=np.int32)
    if m:
        lib.gg_uniform_weights(m, lo, hi, seed, _ptr(w))
    return w


def uniform_ints(count: int, n: int, seed: int, stream: int = 0) -> np.ndarray:
    lib = _load()
    out = np.empty(count, dtype=np.int32)
    if count:
        lib.gg_uniform_ints(count, n, seed, stream, _ptr(out))
    return out


def uniform_doubles(count: int, seed: int, stream: int = 0) -> np.ndarray:
    lib = _load()
    out = np.empty(count, dtype=np.float64)
    if count:
        lib.gg_uniform_doubles(count, seed, stream, _ptr(out))
    return out


# --------------------------------------------------------------------------
# Edge-list helpers and small families with closed-form answers.
# --------------------------------------------------------------------------

def from_edges(n: int, src, dst, w=None, name: str = "", keep_self_loops: bool = False) -> Graph:
    """CSR from an edge list: rows sorted by destination, duplicates removed
    (the first weight of a duplicated (src, dst) pair in input order is kept)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("edge endpoint out of range")
    keep = np.ones(src.shape, dtype=bool) if keep_self_loops else (src != dst)
    src, dst = src[keep], dst[keep]
    if w is not None:
        w = np.asarray(w, dtype=np.int64)[keep]
    key = src * n + dst
    order = np.lexsort((np.arange(key.size), key))
    key = key[order]
    first = np.ones(key.size, dtype=bool)
    first[1:] = key[1:] != key[:-1]
    order = order[first]
    s, d = src[order], dst[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, s + 1, 1)
    off = np.cumsum(off).astype(np.int32)
    ww = None if w is None else w[order].astype(np.int32)
    return Graph(n, off, d.astype(np.int32), ww, name)


def undirected(n: int, src, dst, w=None, name: str = "") -> Graph:
    """Both directions of every listed edge (same weight each way)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    ww = None if w is None else np.concatenate([np.asarray(w), np.asarray(w)])
    return from_edges(n, np.concatenate([src, dst]), np.concatenate([dst, src]), ww, name)


def symmetrised(g: Graph) -> Graph:
    """Both directions of every edge of g, self-loops and duplicates removed
    (unweighted): the undirected graph that k-core and CC work on."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    return undirected(g.n, src, g.col.astype(np.int64), name=g.name + "_sym")


def path(n: int, w=None, directed: bool = True) -> Graph:
    s = np.arange(n - 1)
    f = from_edges if directed else undirected
    return f(n, s, s + 1, w, name="path%d" % n)


def cycle(n: int, w=None) -> Graph:
    s = np.arange(n)
    return from_edges(n, s, (s + 1) % n, w, name="cycle%d" % n)


def star(k: int, w=None) -> Graph:
    """Undirected star: centre 0 and leaves 1..k."""
    leaves = np.arange(1, k + 1)
    return undirected(k + 1, np.zeros(k, dtype=np.int64), leaves, w, name="star%d" % k)


def grid(r: int, c: int, weight: Optional[int] = None) -> Graph:
    """Undirected r x c grid, vertex (i, j) = i * c + j."""
    ids = np.arange(r * c).reshape(r, c)
    s = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    d = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    w = None if weight is None else np.full(s.size, weight, dtype=np.int64)
    return undirected(r * c, s, d, w, name="grid%dx%d" % (r, c))


def complete(n: int) -> Graph:
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return from_edges(n, s.ravel(), d.ravel(), name="complete%d" % n)


def edgeless(n: int) -> Graph:
    return Graph(n, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), None, "edgeless%d" % n)


def random_digraph(n: int, m: int, seed: int, weighted: bool = False, wmax: int = 100) -> Graph:
    """m directed edges with uniform endpoints (self-loops and duplicates removed)."""
    s = uniform_ints(m, n, seed, 0)
    d = uniform_ints(m, n, seed, 1)
    g = from_edges(n, s, d, name="rand%d_%d_s%d" % (n, m, seed))
    if weighted:
        g = g.with_weights(seed + 1000, 1, wmax)
    return g


def disjoint_copies(g: Graph, k: int) -> Graph:
    """k disjoint copies of g; copy i uses vertex ids i*n .. i*n+n-1."""
    deg = g.degrees()
    src = np.repeat(np.arange(g.n), deg)
    ss = np.concatenate([src + i * g.n for i in range(k)])
    dd = np.concatenate([g.col.astype(np.int64) + i * g.n for i in range(k)])
    ww = None if g.w is None else np.concatenate([g.w] * k)
    return from_edges(g.n * k, ss, dd, ww, name="%sx%d" % (g.name, k))


def boundary_path(n: int, back_edges: int, seed: int, hub_back: int = 0) -> Graph:
    """A directed path 0 -> 1 -> ... -> n-1 whose every edge weighs
    W = (2^31 - 2) // (n - 1), so that the last vertex lies at distance
    W * (n - 1) (2^31 - 2 = INT32_MAX - 1 when n - 1 divides it), plus
    `back_edges` random edges u -> v with u > v and weights uniform in [0, W],
    and `hub_back` more such edges out of the last vertex (distinct targets).
    Backward edges cannot shorten the path, so vertex i lies at distance
    i * W; their candidates from the far end exceed INT32_MAX."""
    W = (2 ** 31 - 2) // (n - 1)
    s = np.arange(n - 1)
    src = [s]
    dst = [s + 1]
    wts = [np.full(n - 1, W, np.int64)]
    a = uniform_ints(back_edges, n, seed, 0).astype(np.int64)
    b = uniform_ints(back_edges, n, seed, 1).astype(np.int64)
    keep = a != b
    hi, lo = np.maximum(a, b)[keep], np.minimum(a, b)[keep]
    src.append(hi)
    dst.append(lo)
    wts.append(uniform_ints(hi.size, W + 1, seed, 2).astype(np.int64))
    if hub_back:
        t = np.sort(np.random.Generator(np.random.Philox(seed)).choice(n - 1, size=min(hub_back, n - 1),
                                                                       replace=False))
        src.append(np.full(t.size, n - 1, np.int64))
        dst.append(t.astype(np.int64))
        wts.append(uniform_ints(t.size, W + 1, seed, 3).astype(np.int64))
    return from_edges(n, np.concatenate(src), np.concatenate(dst), np.concatenate(wts),
                      name="boundary_path%d" % n)


def hub_graph(n: int, hubs, deg_small: int, seed: int) -> Graph:
    """Vertices in `hubs` (dict vertex -> out-degree) point at distinct random
    targets; every other vertex gets about `deg_small` random out-edges."""
    rng = np.random.Generator(np.random.Philox(seed))
    src, dst = [], []
    for v, d in hubs.items():
        t = rng.choice(n, size=min(d, n), replace=False)
        src.append(np.full(t.size, v))
        dst.append(t)
    m_small = n * deg_small
    src.append(rng.integers(0, n, m_small))
    dst.append(rng.integers(0, n, m_small))
    return from_edges(n, np.concatenate(src), np.concatenate(dst), name="hub%d_s%d" % (n, seed))


# --------------------------------------------------------------------------
# The benchmark workloads (sizes and seeds of the configurations measured).
# --------------------------------------------------------------------------

_cache = {}


def workload(name: str) -> Graph:
    """Named workloads:
      rmat14      RMAT scale 14, ef 16, seed 1, unweighted (BFS from vertex 0)
      rmat22w     RMAT scale 22, ef 16, seed 1, weights U[1,100] seed 2 (SSSP
                  from the highest-degree vertex)
      zipf24      Zipf(1.9) out-degrees capped at 4,194,304, n = 2^24, seed 3
    Results are cached per process."""
    if name in _cache:
        return _cache[name]
    if name == "rmat14":
        g = rmat(14, 16, seed=1)
    elif name == "rmat22w":
        g = rmat(22, 16, seed=1).with_weights(2, 1, 100)
    elif name == "rmat22":
        g = rmat(22, 16, seed=1)
    elif name == "zipf24":
        g = zipf(1 << 24, 1.9, 4194304, seed=3)
    elif name.startswith("rmat") and name[4:].isdigit():
        g = rmat(int(name[4:]), 16, seed=1)
    else:
        raise KeyError(name)
    g.name = name
    _cache[name] = g
    return g


# --------------------------------------------------------------------------
# Query workloads: many graphs and many sources.
# --------------------------------------------------------------------------

def rmat_set(count: int = 64, lo: int = 12, hi: int = 20, seed: int = 7, edge_factor: int = 16,
             weighted: bool = True) -> list:
    """`count` RMAT graphs whose scales are drawn uniformly from lo..hi
    (stream `seed`); graph i uses RMAT seed 100 + i and, if weighted, weights
    U[1,100] with seed 1000 + i."""
    scales = uniform_ints(count, hi - lo + 1, seed) + lo
    out = []
    for i, s in enumerate(scales):
        g = rmat(int(s), edge_factor, seed=100 + i)
        if weighted:
            g = g.with_weights(1000 + i, 1, 100)
        out.append(g)
    return out


def query_sources(graphs: list, count: int, seed: int = 8):
    """`count` queries, query i on graph i mod len(graphs), each with a source
    of out-degree > 0 drawn uniformly; the sources on one graph are distinct
    while the graph has enough such vertices.  Returns (graph index, source)
    arrays."""
    k = len(graphs)
    members = np.arange(count, dtype=np.int32) % k
    sources = np.zeros(count, np.int32)
    for gi in range(k):
        qs = np.nonzero(members == gi)[0]
        if not len(qs):
            continue
        nz = np.nonzero(graphs[gi].degrees() > 0)[0].astype(np.int32)
        if not len(nz):
            nz = np.zeros(1, np.int32)
        picked, stream = [], 0
        while len(picked) < len(qs):
            for x in uniform_ints(4 * len(qs), len(nz), seed, stream=gi + k * stream):
                v = int(nz[x])
                if v not in picked or len(picked) >= len(nz):
                    picked.append(v)
                if len(picked) == len(qs):
                    break
            stream += 1
        sources[qs] = picked
    return members, sources


def serving_set(weighted: bool = True) -> list:
    """32 graphs for a serving workload: 30 RMAT graphs of scale 14 + (i mod 9)
    (RMAT seed 200 + i) and Zipf(1.9) out-degree graphs with 2^20 and 2^23
    vertices (degrees capped at n / 4, seeds 230, 231); weights U[1,100]
    with seed 2000 + i."""
    out = []
    for i in range(30):
        out.append(rmat(14 + i % 9, 16, seed=200 + i))
    out.append(zipf(1 << 20, 1.9, 1 << 18, seed=230))
    out.append(zipf(1 << 23, 1.9, 1 << 21, seed=231))
    if weighted:
        out = [g.with_weights(2000 + i, 1, 100) for i, g in enumerate(out)]
    return out


def poisson_arrivals(rate: float, count: int, seed: int = 9) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of `rate` per
    second: cumulative sums of exponential gaps -log(1 - U) / rate."""
    u = uniform_doubles(count, seed, stream=int(rate))
    return np.cumsum(-np.log1p(-u) / rate)

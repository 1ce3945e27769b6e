"""CPU oracle for the ALB hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it, and the two share no
code: the oracle is plain single-threaded C (oracle.c) implementing the
textbook definitions of what the path computes, plus the inspection, prefix
and distribution rules of Algorithms 1 and 2 and Section 4.1 of the paper.

Functions (each cites its passage in oracle.c):
  bfs(g, s)                 hop levels, INT32_MAX = unreachable     (Section 2, bfs in Section 5)
  sssp(g, s)                Dijkstra distances, INT32_MAX = unreachable (sssp, relaxation operator, Section 4.3)
  cc(g)                     weakly connected components, min-id labels (cc, Section 5)
  pagerank(g, d, iters)     fp64 synchronous power iteration         (pr, Section 5)
  inspect(...)              Algorithm 1 bins and the huge worklist
  prefix_work(...)          Section 4.1 prefixWork (exclusive scan of huge degrees)
  owner(...), lb_edges(...) Section 4.1 binary search and cyclic distribution

Parity status: every function is pinned by the CPU tests in
tests/test_oracle.py (brute force, closed forms, library routines,
invariants and the Figure 2 worked example).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

INF = np.iinfo(np.int32).max


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C; OpenMP only for the PageRank v-loop)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.oracle_bfs.restype = ctypes.c_int
        lib.oracle_bfs.argtypes = [i32, vp, vp, i32, vp]
        lib.oracle_sssp.restype = ctypes.c_int
        lib.oracle_sssp.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.oracle_cc.restype = ctypes.c_int
        lib.oracle_cc.argtypes = [i32, vp, vp, vp]
        lib.oracle_symmetrise.restype = i64
        lib.oracle_symmetrise.argtypes = [i32, vp, vp, vp, vp]
        lib.oracle_kcore.restype = ctypes.c_int
        lib.oracle_kcore.argtypes = [i32, vp, vp, i32, vp]
        lib.oracle_pagerank.restype = ctypes.c_int
        lib.oracle_pagerank.argtypes = [i32, vp, vp, dbl, i32, i32, vp]
        lib.oracle_inspect.restype = i64
        lib.oracle_inspect.argtypes = [i64, vp, vp, i64, i64, i64, vp, vp]
        lib.oracle_prefix_work.restype = None
        lib.oracle_prefix_work.argtypes = [i64, vp, vp, vp]
        lib.oracle_owner.restype = i64
        lib.oracle_owner.argtypes = [i64, vp, i64]
        lib.oracle_cyclic_thread.restype = i64
        lib.oracle_cyclic_thread.argtypes = [i64, i64]
        lib.oracle_blocked_thread.restype = i64
        lib.oracle_blocked_thread.argtypes = [i64, i64, i64]
        lib.oracle_lb_edges.restype = None
        lib.oracle_lb_edges.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp]
        _lib = lib
    return _lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def bfs(g, source: int) -> np.ndarray:
    off, col = _i32(g.off), _i32(g.col)
    out = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_bfs(g.n, _p(off), _p(col), int(source), _p(out))
    if rc != 0:
        raise ValueError("oracle_bfs failed: %d" % rc)
    return out


def sssp(g, source: int) -> np.ndarray:
    if g.w is None:
        raise ValueError("sssp needs weights")
    off, col, w = _i32(g.off), _i32(g.col), _i32(g.w)
    out = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_sssp(g.n, _p(off), _p(col), _p(w), int(source), _p(out))
    if rc != 0:
        raise ValueError("oracle_sssp failed: %d" % rc)
    return out


def cc(g) -> np.ndarray:
    off, col = _i32(g.off), _i32(g.col)
    out = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_cc(g.n, _p(off), _p(col), _p(out))
    if rc != 0:
        raise ValueError("oracle_cc failed: %d" % rc)
    return out


class _Csr:
    def __init__(self, n, off, col):
        self.n, self.off, self.col = n, off, col
        self.m = int(col.shape[0])


def symmetrised(g):
    """The undirected graph of g (both directions, no self-loops or
    duplicates, rows sorted), as an object with n, off, col."""
    off, col = _i32(g.off), _i32(g.col)
    off64 = np.empty(g.n + 1, dtype=np.int64)
    lib = _load()
    m = lib.oracle_symmetrise(g.n, _p(off), _p(col), _p(off64), None)
    if m < 0:
        raise MemoryError("oracle_symmetrise failed")
    if m >= 2 ** 31:
        raise ValueError("symmetrised graph too large")
    out = np.empty(max(m, 1), dtype=np.int32)
    lib.oracle_symmetrise(g.n, _p(off), _p(col), _p(off64), _p(out))
    return _Csr(g.n, off64.astype(np.int32), out[:m])


def kcore(g, k: int) -> np.ndarray:
    """k-core membership (1 in the core, 0 removed) of a symmetric CSR."""
    off, col = _i32(g.off), _i32(g.col)
    out = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_kcore(g.n, _p(off), _p(col), int(k), _p(out))
    if rc != 0:
        raise ValueError("oracle_kcore failed: %d" % rc)
    return out


def pagerank(g, damping: float = 0.85, iterations: int = 50, threads: int = 1) -> np.ndarray:
    off, col = _i32(g.off), _i32(g.col)
    out = np.empty(g.n, dtype=np.float64)
    rc = _load().oracle_pagerank(g.n, _p(off), _p(col), float(damping), int(iterations), int(threads), _p(out))
    if rc != 0:
        raise ValueError("oracle_pagerank failed: %d" % rc)
    return out


BIN_THREAD, BIN_WAVE, BIN_WG, BIN_HUGE = 0, 1, 2, 3


def inspect(frontier, off, threshold: int, warp_cutoff: int, cta_cutoff: int):
    """Algorithm 1: per-entry bin codes and the huge worklist in frontier order."""
    fr, off = _i32(frontier), _i32(off)
    nf = fr.shape[0]
    bins = np.empty(nf, dtype=np.int8)
    work = np.empty(max(nf, 1), dtype=np.int32)
    nw = _load().oracle_inspect(nf, _p(fr), _p(off), int(threshold), int(warp_cutoff), int(cta_cutoff),
                                _p(bins), _p(work))
    return bins, work[:nw].copy()


def prefix_work(work, off) -> np.ndarray:
    work, off = _i32(work), _i32(off)
    out = np.empty(work.shape[0] + 1, dtype=np.int64)
    _load().oracle_prefix_work(work.shape[0], _p(work), _p(off), _p(out))
    return out


def owner(prefix, k: int) -> int:
    prefix = np.ascontiguousarray(prefix, dtype=np.int64)
    return int(_load().oracle_owner(prefix.shape[0] - 1, _p(prefix), int(k)))


def cyclic_thread(k: int, p: int) -> int:
    return int(_load().oracle_cyclic_thread(int(k), int(p)))


def blocked_thread(k: int, w: int, p: int) -> int:
    return int(_load().oracle_blocked_thread(int(k), int(w), int(p)))


def lb_edges(work, prefix, off, p: int):
    """Algorithm 2 with the cyclic distribution: (src, pos, thread) per huge edge."""
    work, off = _i32(work), _i32(off)
    prefix = np.ascontiguousarray(prefix, dtype=np.int64)
    w = int(prefix[-1])
    src = np.empty(w, dtype=np.int32)
    pos = np.empty(w, dtype=np.int64)
    thr = np.empty(w, dtype=np.int64)
    if w:
        _load().oracle_lb_edges(work.shape[0], _p(work), _p(prefix), _p(off), int(p), _p(src), _p(pos), _p(thr))
    return src, pos, thr

"""Python binding of libalb.so (include/alb.h): argument marshalling only.

Every traversal step runs in the HIP kernels of libalb.so.  torch is used only
to hand over device buffers (a CUDA tensor's data_ptr) and streams.  If the
library is not built this module raises ImportError at import time: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ALB_LIBRARY: another build of the same library (the sanitizer builds)
LIB_PATH = os.environ.get("ALB_LIBRARY") or os.path.join(_HERE, "libalb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("%s is not built (python -m paper_1911_09135_amd.build); the ALB library has no CPU "
                      "fallback" % LIB_PATH)

# torch, where installed, is loaded before the library: its HIP runtime then
# serves the library as well.  Loaded the other way round, the library's
# runtime comes first and torch finds no GPU in the same process.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    pass

_lib = ctypes.CDLL(LIB_PATH)

ALB_OK, ALB_E_INVAL, ALB_E_NOMEM, ALB_E_DEVICE, ALB_E_RANGE, ALB_E_OVERFLOW, ALB_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
ALB_E_TIMEOUT, ALB_E_CANCELLED = -7, -8
ALB_SYMMETRIC, ALB_BUILD_SYMMETRIC, ALB_BUILD_TRANSPOSE = 1, 2, 4
# m / (20 * workgroups) within [64, 4096], lower in rounds smaller than the grid (BFS, k-core: 64; others: a
# quarter, at least 64); the launched thread count (the paper's rule); 64 in rounds smaller than the grid, else
# default
THRESHOLD_DEFAULT, THRESHOLD_LAUNCHED, THRESHOLD_ADAPTIVE = -1, -2, -3
GRID_ALL = -1  # grid_wgs: every resident workgroup (0 = automatic)
MODES = {"alb": 0, "twc": 1, "twc_only": 1, "lb_all": 2}
LAUNCHES = {"auto": 0, "host": 1, "host_loop": 1, "persistent": 2}
INF = np.iinfo(np.int32).max
BIN_THREAD, BIN_WAVE, BIN_WG, BIN_HUGE = 0, 1, 2, 3
ALGOS = {"bfs": 0, "sssp": 1}


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("mode", ctypes.c_int32),
        ("huge_threshold", ctypes.c_int64),
        ("wg_size", ctypes.c_int32),
        ("wave_cutoff", ctypes.c_int32),
        ("wg_cutoff", ctypes.c_int32),
        ("distribution", ctypes.c_int32),
        ("dedup", ctypes.c_int32),
        ("launch", ctypes.c_int32),
        ("grid_wgs", ctypes.c_int32),
        ("worklist_capacity", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("out_on_device", ctypes.c_uint32),
        ("visited_filter", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 6),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("rounds", ctypes.c_int32),
        ("kernel_launches", ctypes.c_int32),
        ("launched_threads", ctypes.c_int64),
        ("huge_threshold", ctypes.c_int64),
        ("frontier_vertices", ctypes.c_int64),
        ("edges_examined", ctypes.c_int64),
        ("huge_vertices", ctypes.c_int64),
        ("huge_edges", ctypes.c_int64),
        ("pushes", ctypes.c_int64),
        ("device_ms", ctypes.c_double),
        ("kernel_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i32, _i64, _u32, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float

# int32 (*)(void *user, int32 algo, int32 count, const int32 *members, const int32 *sources, int32 *const *outs,
#           int32 lane)
EXEC_FN = ctypes.CFUNCTYPE(_i32, _vp, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                           ctypes.POINTER(ctypes.POINTER(_i32)), _i32)


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("lanes", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("max_wait_us", ctypes.c_int32),
        ("hbm_budget", ctypes.c_int64),
        ("options", Options),
        ("executor", EXEC_FN),
        ("executor_user", ctypes.c_void_p),
        ("n_members", ctypes.c_int32),
        ("member_vertices", ctypes.POINTER(ctypes.c_int32)),
        ("whole_device_when_alone", ctypes.c_int32),
        ("join_running", ctypes.c_int32),
        ("join_idle_us", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("join_long_edges", ctypes.c_int64),
        ("reserved", ctypes.c_int32 * 2),
    ]


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("lane", ctypes.c_int32),
        ("algo", ctypes.c_int32),
        ("queue_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "timed_out", "cancelled",
                                              "rejected", "batches", "pending", "running")] + \
               [("busy_ms", ctypes.c_double), ("direct_outputs", ctypes.c_int64)]


class QueryTuning(ctypes.Structure):
    _fields_ = [("huge_threshold", ctypes.c_int64), ("wave_cutoff", ctypes.c_int32), ("wg_cutoff", ctypes.c_int32)]


class BatchRecord(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("lane", "algo", "batch_size", "status")] + \
               [(k, ctypes.c_double) for k in ("device_begin_ms", "device_end_ms", "host_begin_ms", "host_end_ms")]


_POpt, _PSt = ctypes.POINTER(Options), ctypes.POINTER(Stats)
_sig = {
    "alb_options_init": ([_POpt], ctypes.c_int),
    "alb_graph_create": ([_i32, _i64, _vp, _vp, _vp, _u32, ctypes.POINTER(_vp)], ctypes.c_int),
    "alb_graph_destroy": ([_vp], ctypes.c_int),
    "alb_graph_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                        ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "alb_bfs": ([_vp, _i32, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_sssp": ([_vp, _i32, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_sssp_noalloc": ([_vp, _i32, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_cc": ([_vp, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_pagerank": ([_vp, _f32, _i32, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_kcore": ([_vp, _i32, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_pagerank_pull": ([_vp, _f32, _i32, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_graph_create_set": ([_i32, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "alb_graph_members": ([_vp, ctypes.POINTER(_i32)], ctypes.c_int),
    "alb_graph_member_info": ([_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i32)],
                              ctypes.c_int),
    "alb_bfs_batch": ([_vp, _i32, _vp, _vp, _vp, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_sssp_batch": ([_vp, _i32, _vp, _vp, _vp, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_bfs_batch_tuned": ([_vp, _i32, _vp, _vp, _vp, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_sssp_batch_tuned": ([_vp, _i32, _vp, _vp, _vp, _vp, _POpt, _PSt], ctypes.c_int),
    "alb_batch_plan_create_tuned": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp, _POpt, ctypes.POINTER(_vp)], ctypes.c_int),
    "alb_autotune_batch_tuned": ([_vp, _i32, _i32, _vp, _vp, _POpt, _POpt, _vp, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "alb_batch_plan_create": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp, _POpt, ctypes.POINTER(_vp)], ctypes.c_int),
    "alb_batch_plan_run": ([_vp, _PSt], ctypes.c_int),
    "alb_batch_plan_destroy": ([_vp], ctypes.c_int),
    "alb_autotune": ([_vp, _i32, _i32, _i32, _vp, _POpt, _POpt, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "alb_autotune_batch": ([_vp, _i32, _i32, _vp, _vp, _POpt, _POpt, _vp], ctypes.c_int),
    "alb_autotune_reset": ([], ctypes.c_int),
    "alb_server_config_init": ([ctypes.POINTER(ServerConfig)], ctypes.c_int),
    "alb_server_create": ([_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)], ctypes.c_int),
    "alb_server_submit": ([_vp, _i32, _i32, _i32, _vp, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)],
                          ctypes.c_int),
    "alb_server_wait": ([_vp, ctypes.c_uint64, ctypes.POINTER(RequestInfo)], ctypes.c_int),
    "alb_server_cancel": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "alb_server_drain": ([_vp], ctypes.c_int),
    "alb_server_stats_get": ([_vp, ctypes.POINTER(ServerStats)], ctypes.c_int),
    "alb_server_destroy": ([_vp], ctypes.c_int),
    "alb_server_batch_log": ([_vp, _i32, ctypes.POINTER(BatchRecord), ctypes.POINTER(_i32)], ctypes.c_int),
    "alb_trace_round": ([_vp, _vp, _i64, _POpt, _vp, _vp, ctypes.POINTER(_i64), _vp, _vp, _vp, _vp,
                         ctypes.POINTER(_i64), _PSt], ctypes.c_int),
    "alb_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "alb_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class AlbError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = "%s: %s (%s)" % (where, _lib.alb_status_str(status).decode(), _lib.alb_last_error().decode())
        super().__init__(msg)


def _check(status: int, where: str) -> None:
    if status != ALB_OK:
        raise AlbError(status, where)


def make_options(mode: str = "alb", threshold: Optional[int] = None, wg_size: int = 0, wave_cutoff: int = 0,
                 wg_cutoff: int = 0, dedup: Optional[bool] = None, launch: str = "auto", grid_wgs: int = 0,
                 worklist_capacity: int = 0, stream=None, out_on_device: bool = False,
                 distribution: int = 0, visited_filter: Optional[bool] = None) -> Options:
    o = Options()
    _check(_lib.alb_options_init(ctypes.byref(o)), "alb_options_init")
    o.mode = MODES[mode]
    if threshold is None:
        o.huge_threshold = THRESHOLD_DEFAULT
    elif threshold == "launched":
        o.huge_threshold = THRESHOLD_LAUNCHED
    elif threshold == "adaptive":
        o.huge_threshold = THRESHOLD_ADAPTIVE
    else:
        o.huge_threshold = int(threshold)
    o.wg_size = int(wg_size)
    o.wave_cutoff = int(wave_cutoff)
    o.wg_cutoff = int(wg_cutoff)
    o.distribution = int(distribution)
    o.dedup = -1 if dedup is None else int(bool(dedup))
    o.launch = LAUNCHES[launch]
    o.grid_wgs = int(grid_wgs)
    o.worklist_capacity = int(worklist_capacity)
    o.stream = _stream_handle(stream)
    o.out_on_device = 1 if out_on_device else 0
    o.visited_filter = 0 if visited_filter is None else (1 if visited_filter else -1)
    return o


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # a torch.cuda.Stream


def _i32arr(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


class Graph:
    """Device-resident CSR graph (alb_graph_create)."""

    def __init__(self, off, col, weights=None, symmetric: bool = False, build_symmetric: bool = False,
                 build_transpose: bool = False):
        off, col = _i32arr(off), _i32arr(col)
        w = None if weights is None else _i32arr(weights)
        n = off.shape[0] - 1
        flags = (ALB_SYMMETRIC if symmetric else 0) | (ALB_BUILD_SYMMETRIC if build_symmetric else 0) | \
            (ALB_BUILD_TRANSPOSE if build_transpose else 0)
        h = _vp()
        _check(_lib.alb_graph_create(n, col.shape[0], off.ctypes.data, col.ctypes.data if col.size else None,
                                     None if w is None else w.ctypes.data, flags, ctypes.byref(h)),
               "alb_graph_create")
        self._h = h
        self.n = n
        n_, m_, md = _i32(), _i64(), _i32()
        _check(_lib.alb_graph_info(h, ctypes.byref(n_), ctypes.byref(m_), ctypes.byref(md), None), "alb_graph_info")
        self.m = m_.value
        self.max_out_degree = md.value

    @classmethod
    def from_csr(cls, g, **kw) -> "Graph":
        """From any object with .off, .col and optional .w (for example graphgen.Graph)."""
        return cls(g.off, g.col, getattr(g, "w", None), **kw)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph is closed")
        return self._h

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(_lib.alb_graph_info(self.handle, None, None, None, ctypes.byref(b)), "alb_graph_info")
        return b.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.alb_graph_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GraphSet(Graph):
    """Several CSR graphs held as one handle for query batches
    (alb_graph_create_set).  `graphs`: objects with .off, .col and, for SSSP,
    .w (for example graphgen.Graph).  members[i] = (n, m, vertex_base)."""

    def __init__(self, graphs, weighted: Optional[bool] = None):
        graphs = list(graphs)
        if weighted is None:
            weighted = all(getattr(g, "w", None) is not None for g in graphs)
        self._keep = []
        offs, cols, ws, ns, ms = [], [], [], [], []
        for g in graphs:
            off, col = _i32arr(g.off), _i32arr(g.col)
            w = _i32arr(g.w) if weighted else None
            self._keep += [off, col, w]
            ns.append(off.shape[0] - 1)
            ms.append(int(g.col.shape[0]))
            offs.append(off.ctypes.data)
            cols.append(col.ctypes.data if col.size else None)
            ws.append(w.ctypes.data if (w is not None and w.size) else None)
        k = len(graphs)
        P = _vp * max(k, 1)
        ns_a = np.asarray(ns, np.int32)
        ms_a = np.asarray(ms, np.int64)
        offs_p, cols_p, ws_p = P(*offs), P(*cols), P(*ws)
        h = _vp()
        _check(_lib.alb_graph_create_set(k, ns_a.ctypes.data, ms_a.ctypes.data, ctypes.cast(offs_p, _vp),
                                         ctypes.cast(cols_p, _vp), ctypes.cast(ws_p, _vp) if weighted else None,
                                         ctypes.byref(h)), "alb_graph_create_set")
        self._keep = None
        self._h = h
        n_, m_, md = _i32(), _i64(), _i32()
        _check(_lib.alb_graph_info(h, ctypes.byref(n_), ctypes.byref(m_), ctypes.byref(md), None), "alb_graph_info")
        self.n, self.m, self.max_out_degree = n_.value, m_.value, md.value
        cnt = _i32()
        _check(_lib.alb_graph_members(h, ctypes.byref(cnt)), "alb_graph_members")
        self.members = []
        for i in range(cnt.value):
            a, b, c = _i32(), _i64(), _i32()
            _check(_lib.alb_graph_member_info(h, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                   "alb_graph_member_info")
            self.members.append((a.value, b.value, c.value))


def _tuning_array(tuning, q: int):
    """A ctypes array of alb_query_tuning from a list of (threshold, wave cutoff, wg cutoff)."""
    if len(tuning) != q:
        raise ValueError("one tuning entry per query")
    arr = (QueryTuning * max(q, 1))()
    for i, (t, cw, cg) in enumerate(tuning):
        arr[i].huge_threshold, arr[i].wave_cutoff, arr[i].wg_cutoff = int(t), int(cw), int(cg)
    return arr


def _run_batch(fn, gs: GraphSet, members, sources, thresholds, outs, opts: dict, tuning=None):
    members = np.ascontiguousarray(members, np.int32)
    sources = np.ascontiguousarray(sources, np.int32)
    if members.shape != sources.shape or members.ndim != 1:
        raise ValueError("members and sources must be 1-D of one length")
    q = members.shape[0]
    outs, ptrs, dev = _batch_outputs(gs, members, outs)
    if dev and opts.get("stream") is None:
        import torch

        opts = dict(opts, stream=torch.cuda.current_stream())
    thr = None if thresholds is None else np.ascontiguousarray(thresholds, np.int64)
    if thr is not None and thr.shape != (q,):
        raise ValueError("one threshold per query")
    per_query = None
    if tuning is not None:
        per_query = ctypes.cast(_tuning_array(tuning, q), _vp)
    elif thr is not None:
        per_query = thr.ctypes.data
    ptr_arr = (_vp * max(q, 1))(*ptrs)
    o = make_options(out_on_device=dev, **opts)
    st = Stats()
    _check(fn(gs.handle, q, members.ctypes.data, sources.ctypes.data, ctypes.cast(ptr_arr, _vp), per_query,
              ctypes.byref(o), ctypes.byref(st)), fn.__name__)
    return outs, st.as_dict()


def _batch_outputs(gs: GraphSet, members, outs):
    """(outs, pointer list, on_device) for a batch's per-query outputs."""
    size = [gs.members[int(mb)][0] if 0 <= mb < len(gs.members) else 1 for mb in members]
    if outs is None:
        outs = [np.empty(n, np.int32) for n in size]
        return outs, [o.ctypes.data for o in outs], False
    outs = list(outs)
    if len(outs) != len(size):
        raise ValueError("one output per query")
    dev = not isinstance(outs[0], np.ndarray)
    ptrs = []
    for o, n in zip(outs, size):
        if dev:
            if not o.is_cuda or not o.is_contiguous() or o.numel() != n or o.dtype.itemsize != 4:
                raise ValueError("device outputs must be contiguous 32-bit CUDA tensors of the member's n")
            ptrs.append(o.data_ptr())
        else:
            if o.dtype != np.int32 or o.shape != (n,) or not o.flags.c_contiguous:
                raise ValueError("host outputs must be contiguous int32 arrays of the member's n")
            ptrs.append(o.ctypes.data)
    return outs, ptrs, dev


class BatchPlan:
    """A batch captured once into a HIP graph and replayed by run()
    (alb_batch_plan_create).  Outputs stay bound to the plan."""

    def __init__(self, gs: GraphSet, algo: str, members, sources, thresholds=None, outs=None, tuning=None,
                 **opts):
        members = np.ascontiguousarray(members, np.int32)
        sources = np.ascontiguousarray(sources, np.int32)
        if members.shape != sources.shape or members.ndim != 1:
            raise ValueError("members and sources must be 1-D of one length")
        self.outs, ptrs, dev = _batch_outputs(gs, members, outs)
        if dev and opts.get("stream") is None:
            import torch

            opts = dict(opts, stream=torch.cuda.current_stream())
        thr = None if thresholds is None else np.ascontiguousarray(thresholds, np.int64)
        self._ptrs = (_vp * max(len(ptrs), 1))(*ptrs)
        o = make_options(out_on_device=dev, **opts)
        h = _vp()
        if tuning is not None:
            tarr = _tuning_array(tuning, members.shape[0])
            _check(_lib.alb_batch_plan_create_tuned(gs.handle, ALGOS[algo], members.shape[0], members.ctypes.data,
                                                    sources.ctypes.data, ctypes.cast(self._ptrs, _vp),
                                                    ctypes.cast(tarr, _vp), ctypes.byref(o), ctypes.byref(h)),
                   "alb_batch_plan_create_tuned")
        else:
            _check(_lib.alb_batch_plan_create(gs.handle, ALGOS[algo], members.shape[0], members.ctypes.data,
                                              sources.ctypes.data, ctypes.cast(self._ptrs, _vp),
                                              None if thr is None else thr.ctypes.data, ctypes.byref(o),
                                              ctypes.byref(h)), "alb_batch_plan_create")
        self._h = h
        self._gs = gs  # the graph must outlive the plan

    def run(self):
        """Replay the batch; returns (outputs, stats)."""
        if self._h is None:
            raise ValueError("plan is closed")
        st = Stats()
        _check(_lib.alb_batch_plan_run(self._h, ctypes.byref(st)), "alb_batch_plan_run")
        return self.outs, st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.alb_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts_dict(o: Options) -> dict:
    thr = o.huge_threshold
    return {"threshold": None if thr == THRESHOLD_DEFAULT else thr, "wg_size": o.wg_size,
            "wave_cutoff": o.wave_cutoff, "wg_cutoff": o.wg_cutoff}


def autotune(g: Graph, algo: str, sources, member: int = 0, **opts):
    """Fastest settings for `algo` on graph g (or member `member` of a set),
    timed on the given sources.  Returns (options dict for the traversal
    calls, median ms of the winner)."""
    src = np.ascontiguousarray(sources, np.int32)
    base = make_options(**opts)
    tuned = Options()
    ms = ctypes.c_double()
    _check(_lib.alb_autotune(g.handle, ALGOS[algo], int(member), src.shape[0], src.ctypes.data, ctypes.byref(base),
                             ctypes.byref(tuned), ctypes.byref(ms)), "alb_autotune")
    return _opts_dict(tuned), ms.value


def autotune_batch(gs: GraphSet, algo: str, members, sources, **opts):
    """Launch-wide settings and per-query thresholds for a batch.  Returns
    (options dict, thresholds array) for bfs_batch / sssp_batch."""
    members = np.ascontiguousarray(members, np.int32)
    sources = np.ascontiguousarray(sources, np.int32)
    base = make_options(**opts)
    tuned = Options()
    thr = np.zeros(members.shape[0], np.int64)
    _check(_lib.alb_autotune_batch(gs.handle, ALGOS[algo], members.shape[0], members.ctypes.data,
                                   sources.ctypes.data, ctypes.byref(base), ctypes.byref(tuned), thr.ctypes.data),
           "alb_autotune_batch")
    d = _opts_dict(tuned)
    d.pop("threshold")
    return d, thr


def autotune_reset():
    _check(_lib.alb_autotune_reset(), "alb_autotune_reset")


def bfs_batch(gs: GraphSet, members, sources, thresholds=None, outs=None, **opts):
    """Query q: BFS levels of member members[q] from its vertex sources[q].
    Returns (list of per-query level arrays, stats), all queries in one launch."""
    return _run_batch(_lib.alb_bfs_batch, gs, members, sources, thresholds, outs, opts)


def sssp_batch(gs: GraphSet, members, sources, thresholds=None, outs=None, **opts):
    """Query q: SSSP distances of member members[q] from its vertex sources[q]."""
    return _run_batch(_lib.alb_sssp_batch, gs, members, sources, thresholds, outs, opts)


def bfs_batch_tuned(gs: GraphSet, members, sources, tuning, outs=None, **opts):
    """bfs_batch with per-query (threshold, wave cutoff, workgroup cutoff) triples."""
    return _run_batch(_lib.alb_bfs_batch_tuned, gs, members, sources, None, outs, opts, tuning=tuning)


def sssp_batch_tuned(gs: GraphSet, members, sources, tuning, outs=None, **opts):
    """sssp_batch with per-query (threshold, wave cutoff, workgroup cutoff) triples."""
    return _run_batch(_lib.alb_sssp_batch_tuned, gs, members, sources, None, outs, opts, tuning=tuning)


def autotune_batch_tuned(gs: GraphSet, algo: str, members, sources, **opts):
    """Per-query thresholds and TWC cutoffs for a batch (alb_autotune_batch_tuned).
    Returns (options dict, list of (threshold, wave cutoff, wg cutoff), best
    uniform-setting ms, tuned ms)."""
    members = np.ascontiguousarray(members, np.int32)
    sources = np.ascontiguousarray(sources, np.int32)
    q = members.shape[0]
    base = make_options(**opts)
    tuned = Options()
    arr = (QueryTuning * max(q, 1))()
    u_ms, t_ms = ctypes.c_double(), ctypes.c_double()
    _check(_lib.alb_autotune_batch_tuned(gs.handle, ALGOS[algo], q, members.ctypes.data, sources.ctypes.data,
                                         ctypes.byref(base), ctypes.byref(tuned), ctypes.cast(arr, _vp),
                                         ctypes.byref(u_ms), ctypes.byref(t_ms)), "alb_autotune_batch_tuned")
    d = _opts_dict(tuned)
    for k in ("threshold", "wave_cutoff", "wg_cutoff"):
        d.pop(k)
    return d, [(arr[i].huge_threshold, arr[i].wave_cutoff, arr[i].wg_cutoff) for i in range(q)], u_ms.value, t_ms.value


class Server:
    """Request loop over a graph set (alb_server_create).  submit() queues a
    BFS / SSSP request and returns its ticket; wait(ticket) blocks until the
    result is in the request's host array.

    `executor(algo, members, sources, outs, lane) -> status` replaces the
    device (outs are the requests' numpy arrays); it needs `member_vertices`
    when no graph set is given."""

    def __init__(self, gs: Optional[GraphSet] = None, lanes: int = 2, max_batch: int = 256, max_wait_us: int = 0,
                 hbm_budget: int = 0, executor=None, member_vertices=None, whole_device_when_alone: bool = True,
                 join_running: bool = False, join_idle_us: int = 0, join_long_edges: int = 0, **opts):
        cfg = ServerConfig()
        _check(_lib.alb_server_config_init(ctypes.byref(cfg)), "alb_server_config_init")
        cfg.lanes, cfg.max_batch, cfg.max_wait_us, cfg.hbm_budget = lanes, max_batch, max_wait_us, hbm_budget
        cfg.whole_device_when_alone = 1 if whole_device_when_alone else 0
        cfg.join_running = 1 if join_running else 0
        cfg.join_idle_us = int(join_idle_us)
        cfg.join_long_edges = int(join_long_edges)
        cfg.options = make_options(**opts)
        if gs is not None:
            self.member_n = [m[0] for m in gs.members]
        else:
            self.member_n = [int(x) for x in (member_vertices if member_vertices is not None else [])]
        self._mv = np.ascontiguousarray(self.member_n, np.int32)
        if executor is not None:
            member_n = self.member_n

            def trampoline(user, algo, count, members, sources, outs, lane):
                try:
                    mb = [members[i] for i in range(count)]
                    src = [sources[i] for i in range(count)]
                    arrs = [np.ctypeslib.as_array(outs[i], shape=(member_n[mb[i]],)) for i in range(count)]
                    return int(executor(algo, mb, src, arrs, lane))
                except Exception:  # an exception cannot cross the C boundary
                    return ALB_E_DEVICE

            self._cb = EXEC_FN(trampoline)
            cfg.executor = self._cb
            if gs is None:
                cfg.n_members = len(self.member_n)
                cfg.member_vertices = self._mv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        h = _vp()
        _check(_lib.alb_server_create(None if gs is None else gs.handle, ctypes.byref(cfg), ctypes.byref(h)),
               "alb_server_create")
        self._h = h
        self._gs = gs  # the graph must outlive the server
        self._outs = {}

    def submit(self, algo: str, member: int, source: int, out=None, timeout_ms: float = 0.0) -> int:
        if out is None:
            out = np.empty(self.member_n[member] if 0 <= member < len(self.member_n) else 1, np.int32)
        elif out.dtype != np.int32 or not out.flags.c_contiguous or out.shape != (self.member_n[member],):
            raise ValueError("out must be a contiguous int32 array of the member's vertex count")
        t = ctypes.c_uint64()
        _check(_lib.alb_server_submit(self._h, ALGOS[algo], int(member), int(source), out.ctypes.data,
                                      float(timeout_ms), ctypes.byref(t)), "alb_server_submit")
        self._outs[t.value] = out
        return t.value

    def wait(self, ticket: int):
        """(result array, info dict); raises AlbError for a failed, timed-out
        or cancelled request (the info is on the exception as .info)."""
        info = RequestInfo()
        st = _lib.alb_server_wait(self._h, ticket, ctypes.byref(info))
        out = self._outs.pop(ticket, None)
        d = {k: getattr(info, k) for k, _ in info._fields_}
        if st != ALB_OK:
            e = AlbError(st, "alb_server_wait")
            e.info = d
            raise e
        return out, d

    def cancel(self, ticket: int) -> None:
        _check(_lib.alb_server_cancel(self._h, ticket), "alb_server_cancel")

    def drain(self) -> None:
        _check(_lib.alb_server_drain(self._h), "alb_server_drain")

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.alb_server_stats_get(self._h, ctypes.byref(st)), "alb_server_stats_get")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def batch_log(self, max_records: int = 4096) -> list:
        """The most recent dispatched batches, oldest first (alb_server_batch_log)."""
        buf = (BatchRecord * max(max_records, 1))()
        n = _i32()
        _check(_lib.alb_server_batch_log(self._h, max_records, buf, ctypes.byref(n)), "alb_server_batch_log")
        return [{k: getattr(buf[i], k) for k, _ in BatchRecord._fields_} for i in range(n.value)]

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.alb_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _out_buffer(g: Graph, out, dtype):
    """Returns (pointer, result object, on_device)."""
    if out is None:
        arr = np.empty(g.n, dtype=dtype)
        return arr.ctypes.data, arr, False
    if isinstance(out, np.ndarray):
        if out.dtype != dtype or out.shape != (g.n,) or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous %s array of length n" % np.dtype(dtype).name)
        return out.ctypes.data, out, False
    # a torch tensor on the GPU
    if not out.is_cuda or not out.is_contiguous() or out.numel() != g.n:
        raise ValueError("out must be a contiguous CUDA tensor of length n")
    return out.data_ptr(), out, True


def _run(fn, g: Graph, out, dtype, opts: dict, *args):
    ptr, res, dev = _out_buffer(g, out, dtype)
    if dev and opts.get("stream") is None:
        import torch

        opts = dict(opts, stream=torch.cuda.current_stream())
    o = make_options(out_on_device=dev, **opts)
    st = Stats()
    _check(fn(g.handle, *args, ptr, ctypes.byref(o), ctypes.byref(st)), fn.__name__)
    return res, st.as_dict()


def bfs(g: Graph, source: int, out=None, **opts):
    """Levels from `source` (int32, INF unreachable) and the stats dict."""
    return _run(_lib.alb_bfs, g, out, np.int32, opts, int(source))


def sssp(g: Graph, source: int, out=None, **opts):
    return _run(_lib.alb_sssp, g, out, np.int32, opts, int(source))


def sssp_noalloc(g: Graph, source: int, out, **opts):
    """alb_sssp_noalloc: SSSP with the workspace in the library's device
    scratch array; `out` must be a contiguous int32 CUDA tensor of n."""
    if isinstance(out, np.ndarray) or out is None:
        raise ValueError("sssp_noalloc writes a device tensor (out)")
    return _run(_lib.alb_sssp_noalloc, g, out, np.int32, opts, int(source))


def cc(g: Graph, out=None, **opts):
    return _run(_lib.alb_cc, g, out, np.int32, opts)


def kcore(g: Graph, k: int, out=None, **opts):
    """k-core membership (int32 1/0) of a symmetric graph and the stats dict."""
    return _run(_lib.alb_kcore, g, out, np.int32, opts, int(k))


def pagerank_pull(g: Graph, damping: float = 0.85, iterations: int = 50, out=None, **opts):
    """PageRank by pull over the in-edges (graph built with build_transpose)."""
    return _run(_lib.alb_pagerank_pull, g, out, np.float32, opts, ctypes.c_float(damping), int(iterations))


def pagerank(g: Graph, damping: float = 0.85, iterations: int = 50, out=None, **opts):
    return _run(_lib.alb_pagerank, g, out, np.float32, opts, ctypes.c_float(damping), int(iterations))


def trace_round(g: Graph, frontier, off=None, **opts) -> dict:
    """One recorded round on an explicit frontier (alb_trace_round)."""
    fr = _i32arr(frontier)
    nf = fr.shape[0]
    bins = np.empty(nf, dtype=np.int8)
    work = np.empty(max(nf, 1), dtype=np.int32)
    prefix = np.empty(nf + 1, dtype=np.int64)
    hits = np.empty(max(g.m, 1), dtype=np.int32)
    thr = np.empty(max(g.m, 1), dtype=np.int32)
    if off is not None:
        cap = int(np.diff(_i32arr(off).astype(np.int64))[fr].sum())
    else:
        cap = g.m * nf  # upper bound when the caller gives no degrees
    nxt = np.empty(max(cap, nf, 1), dtype=np.int32)
    nwork, nnext = _i64(), _i64()
    o = make_options(**opts)
    st = Stats()
    _check(_lib.alb_trace_round(g.handle, fr.ctypes.data, nf, ctypes.byref(o), bins.ctypes.data, work.ctypes.data,
                                ctypes.byref(nwork), prefix.ctypes.data, hits.ctypes.data, thr.ctypes.data,
                                nxt.ctypes.data, ctypes.byref(nnext), ctypes.byref(st)), "alb_trace_round")
    k = nwork.value
    return {"bins": bins, "work": work[:k].copy(), "prefix": prefix[:k + 1].copy(), "edge_hits": hits[:g.m],
            "edge_thread": thr[:g.m], "next": nxt[:nnext.value].copy(), "stats": st.as_dict()}


def algorithmic_bytes(kind: str, stats: dict, n: int = 0, iterations: int = 0) -> int:
    """Bytes a push round must move whatever the schedule:
      bfs, cc, kcore: 16 B per active vertex (worklist entry, two offsets, label)
                 + 8 B per examined edge (column, destination label) + 4 B per push
      sssp:     16 B per active vertex + 12 B per examined edge (adds the weight) + 4 B per push
      pagerank: per iteration 8 B per edge (column, accumulator update) and 24 B per vertex
                (rank, offsets, accumulator read and clear, rank write)."""
    if kind in ("bfs", "cc", "kcore"):
        return 16 * stats["frontier_vertices"] + 8 * stats["edges_examined"] + 4 * stats["pushes"]
    if kind == "sssp":
        return 16 * stats["frontier_vertices"] + 12 * stats["edges_examined"] + 4 * stats["pushes"]
    if kind == "pagerank":
        return 8 * stats["edges_examined"] + 24 * n * iterations
    raise KeyError(kind)

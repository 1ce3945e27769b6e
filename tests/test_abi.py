"""CPU checks of the C ABI: the library loads, exports every declared symbol,
its structs match the C compiler's layout, and host-side validation rejects
bad input before any device call."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alb.h")


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(alb_[a-z_]+)\s*\(", text)))


def test_binding_covers_every_declared_symbol(alb):
    """The Python binding gives each C entry point a signature."""
    import inspect

    src = inspect.getsource(alb)
    for name in declared_functions():
        assert '"%s"' % name in src, name


def test_every_declared_symbol_is_exported(alb):
    names = declared_functions()
    assert len(names) >= 11
    lib = ctypes.CDLL(alb.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", alb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (alb_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(alb):
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "alb.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(alb_options), sizeof(alb_stats),
         offsetof(alb_options, stream), offsetof(alb_options, out_on_device),
         offsetof(alb_stats, device_ms), offsetof(alb_stats, pushes));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    O, S = alb.Options, alb.Stats
    assert vals == [ctypes.sizeof(O), ctypes.sizeof(S), O.stream.offset, O.out_on_device.offset,
                    S.device_ms.offset, S.pushes.offset]


def test_server_struct_layouts_match_c(alb):
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "alb.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(alb_server_config), offsetof(alb_server_config, options),
         offsetof(alb_server_config, executor), offsetof(alb_server_config, n_members),
         offsetof(alb_server_config, member_vertices), sizeof(alb_request_info),
         offsetof(alb_request_info, latency_ms), sizeof(alb_server_stats), offsetof(alb_server_stats, running),
         offsetof(alb_server_stats, busy_ms));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    C, R, S = alb.ServerConfig, alb.RequestInfo, alb.ServerStats
    assert vals == [ctypes.sizeof(C), C.options.offset, C.executor.offset, C.n_members.offset,
                    C.member_vertices.offset, ctypes.sizeof(R), R.latency_ms.offset, ctypes.sizeof(S),
                    S.running.offset, S.busy_ms.offset]


def test_options_init_defaults(alb):
    o = alb.make_options()
    assert o.struct_size == ctypes.sizeof(alb.Options)
    assert o.mode == 0 and o.huge_threshold == -1 and o.dedup == -1 and o.launch == 0


def _create(alb, n, off, col, w=None, flags=0):
    h = ctypes.c_void_p()
    off = np.ascontiguousarray(off, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    wp = None if w is None else np.ascontiguousarray(w, dtype=np.int32)
    st = alb._lib.alb_graph_create(n, col.shape[0], off.ctypes.data, col.ctypes.data if col.size else None,
                                   None if wp is None else wp.ctypes.data, flags, ctypes.byref(h))
    return st, alb._lib.alb_last_error().decode()


@pytest.mark.parametrize("case,expect", [
    (dict(n=0, off=[0], col=[]), -1),
    (dict(n=3, off=[1, 1, 2, 2], col=[0, 1]), -1),              # offsets[0] != 0
    (dict(n=3, off=[0, 2, 1, 2], col=[0, 1]), -1),              # decreasing
    (dict(n=3, off=[0, 1, 2, 3], col=[0, 1]), -1),              # offsets[n] != m
    (dict(n=3, off=[0, 1, 2, 2], col=[0, 3]), -1),              # column out of range
    (dict(n=3, off=[0, 1, 2, 2], col=[0, -1]), -1),             # negative column
    (dict(n=3, off=[0, 1, 2, 2], col=[1, 2], w=[1, -2]), -1),   # negative weight
    (dict(n=3, off=[0, 1, 2, 2], col=[1, 2], w=[1, 2**30]), -4),  # distance could overflow
    (dict(n=3, off=[0, 1, 2, 2], col=[1, 2], flags=8), -1),     # unknown flag
])
def test_create_validation(alb, case, expect):
    st, msg = _create(alb, case["n"], case["off"], case["col"], case.get("w"), case.get("flags", 0))
    assert st == expect, msg
    assert msg


def test_calls_reject_null_handles(alb):
    lvl = np.empty(4, dtype=np.int32)
    assert alb._lib.alb_bfs(None, 0, lvl.ctypes.data, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_sssp(None, 0, lvl.ctypes.data, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_cc(None, lvl.ctypes.data, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_pagerank(None, ctypes.c_float(0.85), 5, lvl.ctypes.data, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_kcore(None, 2, lvl.ctypes.data, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_pagerank_pull(None, ctypes.c_float(0.85), 5, lvl.ctypes.data, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_graph_info(None, None, None, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_graph_destroy(None) == alb.ALB_OK
    assert alb._lib.alb_options_init(None) == alb.ALB_E_INVAL


def _create_set(alb, members, weighted=False):
    keep = []
    k = len(members)
    P = ctypes.c_void_p * k
    offs, cols, ws = P(), P(), P()
    ns = np.array([len(o) - 1 for o, _, _ in members], np.int32)
    ms = np.array([len(c) for _, c, _ in members], np.int64)
    for i, (o, c, w) in enumerate(members):
        o, c = np.ascontiguousarray(o, np.int32), np.ascontiguousarray(c, np.int32)
        keep += [o, c]
        offs[i], cols[i] = o.ctypes.data, (c.ctypes.data if c.size else None)
        if w is not None:
            w = np.ascontiguousarray(w, np.int32)
            keep.append(w)
            ws[i] = w.ctypes.data if w.size else None
    h = ctypes.c_void_p()
    st = alb._lib.alb_graph_create_set(k, ns.ctypes.data, ms.ctypes.data, ctypes.cast(offs, ctypes.c_void_p),
                                       ctypes.cast(cols, ctypes.c_void_p),
                                       ctypes.cast(ws, ctypes.c_void_p) if weighted else None, ctypes.byref(h))
    return st, alb._lib.alb_last_error().decode()


@pytest.mark.parametrize("members,weighted", [
    ([([0, 1, 1], [1], None), ([0, 1, 2], [3, 0], None)], False),   # member 1: column out of range
    ([([0, 1, 1], [1], None), ([1, 1], [], None)], False),          # member 1: offsets[0] != 0
    ([([0, 1, 1], [1], [5]), ([0, 1, 1], [0], None)], True),        # member 1 has edges but no weights
    ([([0, 1, 1], [1], [-5])], True),                               # negative weight
])
def test_graph_set_validation(alb, members, weighted):
    st, msg = _create_set(alb, members, weighted)
    assert st == alb.ALB_E_INVAL, msg
    assert "member" in msg or "weight" in msg


def test_graph_set_rejects_empty_and_null(alb):
    h = ctypes.c_void_p()
    assert alb._lib.alb_graph_create_set(0, None, None, None, None, None, ctypes.byref(h)) == alb.ALB_E_INVAL
    assert alb._lib.alb_graph_create_set(1, None, None, None, None, None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_graph_members(None, None) == alb.ALB_E_INVAL
    assert alb._lib.alb_graph_member_info(None, 0, None, None, None) == alb.ALB_E_INVAL


def test_batch_calls_reject_null_handles(alb):
    mb = np.zeros(1, np.int32)
    st = alb.Stats()
    for fn in (alb._lib.alb_bfs_batch, alb._lib.alb_sssp_batch):
        assert fn(None, 1, mb.ctypes.data, mb.ctypes.data, mb.ctypes.data, None, None, ctypes.byref(st)) == \
            alb.ALB_E_INVAL
        assert st.rounds == 0


def test_status_strings(alb):
    for s, name in [(0, "ALB_OK"), (-1, "ALB_E_INVAL"), (-5, "ALB_E_OVERFLOW"), (-6, "ALB_E_UNSUPPORTED")]:
        assert alb._lib.alb_status_str(s).decode() == name


def test_binding_has_no_cpu_fallback():
    """The binding refuses to import when libalb.so is missing."""
    env = {k: v for k, v in os.environ.items() if k not in ("ALB_LIBRARY", "LD_PRELOAD")}
    with tempfile.TemporaryDirectory() as d:
        # a copy of the package without the library
        import shutil

        pkg = os.path.join(d, "paper_1911_09135_amd")
        shutil.copytree(os.path.join(ROOT, "paper_1911_09135_amd"), pkg,
                        ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
        code = "import sys; sys.path.insert(0, %r); import paper_1911_09135_amd.alb" % d
        r = subprocess.run(["python", "-c", code], capture_output=True, text=True, env=env)
    assert r.returncode != 0
    assert "not built" in r.stderr


def test_visited_filter_option_is_validated(alb):
    o = alb.make_options()
    assert o.visited_filter == 0  # automatic
    assert alb.make_options(visited_filter=True).visited_filter == 1
    assert alb.make_options(visited_filter=False).visited_filter == -1

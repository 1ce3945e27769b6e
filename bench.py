#!/usr/bin/env python3
"""Benchmark: SSSP on RMAT scale 22 (4,194,304 vertices, edge factor 16,
(a,b,c) = (0.57,0.19,0.19), self-loops and duplicates removed, int32 weights
uniform in [1,100]) from the highest-degree vertex, on one MI355X.

A step is one full SSSP query (label initialisation and every BSP round of
the adaptive load balancer) with the graph resident in HBM.  Reported: GTEPS
(edges of reached vertices / time), the same kernels with the huge-vertex
cyclic path disabled (TWC only), the roofline fraction of the traversal
kernel, and the CPU oracle (Dijkstra) on the host.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--threshold T] [--no-sweep]
                    [--workload sssp_rmat22|batch|serve|zipf24]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "GTEPS (SSSP/BFS, 1 MI355X) ALB vs TWC-only; % HBM roofline; queries/s + p99"
KERNEL_SOURCE = os.path.join(ROOT, "paper_1911_09135_amd", "csrc", "alb_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sssp_rmat22.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def run_steps(alb, dg, source, out, steps, opts):
    """Run `steps` queries back to back; returns (wall seconds, list of stats)."""
    import torch

    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st = alb.sssp(dg, source, out=out, **opts)
        stats.append(st)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--threshold", type=int, default=None,
                    help="huge-degree threshold for the ALB run (default: the library's, m / (20 x workgroups) "
                         "within [64, 4096])")
    ap.add_argument("--launch", default="auto")
    ap.add_argument("--no-sweep", action="store_true", help="skip the threshold sweep over powers of two")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only-alb", action="store_true", help="skip the TWC-only comparison (profiling runs)")
    ap.add_argument("--workload", default="sssp_rmat22", choices=["sssp_rmat22", "batch", "serve", "zipf24"],
                    help="batch: 256 SSSP queries over 64 RMAT graphs of scales 12..20 in one launch, "
                         "against the same queries one launch each; serve: Poisson streams of BFS/SSSP "
                         "requests over 32 graphs through the serving loop")
    ap.add_argument("--requests", type=int, default=5000, help="serve: requests per arrival rate")
    ap.add_argument("--rates", default="100,200,500,1000,2000,5000", help="serve: arrival rates per second")
    ap.add_argument("--join-long-edges", type=int, default=0,
                    help="serve: the joining server runs two lanes, requests on members with at least this many "
                         "edges on lane 0 and the rest on lane 1 (0: one lane with the whole device)")
    ap.add_argument("--tune", action="store_true",
                    help="batch: also run with autotuned per-query settings (always in the default line's summary)")
    ap.add_argument("--random-probe", action="store_true",
                    help="only measure plain random 8-byte gathers (the access pattern of the label reads)")
    ap.add_argument("--relax-probe", action="store_true",
                    help="only measure the edge-relaxation loop alone over RMAT-22's edges, labels in one array "
                         "or in eight per-XCD destination slices (what a label layout can gain)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: leave out the Zipf-2^24, batch and serving summaries")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed steps of each summary measurement")
    ap.add_argument("--parts", default="bfs,pagerank,pull,cc,kcore,grid",
                    help="zipf24: the parts to run (profiling runs take one)")
    ap.add_argument("--visited-filter", default="auto", choices=["auto", "on", "off"],
                    help="zipf24: the BFS/CC/k-core filter bitmap of the ALB runs (auto: the library's default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration << 18  # int32 elements
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                          "launches": max(args.steps, 1)}))
        return

    if args.random_probe:
        return random_probe(args)
    if args.relax_probe:
        return relax_probe(args)

    import graphgen as gg
    from paper_1911_09135_amd import alb

    if args.workload == "batch":
        bench_batch(args, alb, gg)
        return
    if args.workload == "serve":
        bench_serve(args, alb, gg)
        return
    if args.workload == "zipf24":
        bench_zipf24(args, alb, gg, cpu=not args.no_cpu, parts=args.parts)
        return

    t = time.perf_counter()
    g = gg.workload("rmat22w")
    src = g.max_degree_vertex()
    log("graph rmat22w: n=%d m=%d max_deg=%d (%.1fs)" % (g.n, g.m, g.degrees().max(), time.perf_counter() - t))
    dg = alb.Graph(g.off, g.col, g.w)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    base_opts = dict(launch=args.launch)

    def measure(opts, label):
        for _ in range(args.warmup):
            alb.sssp(dg, src, out=out, **opts)
        sec, stats = run_steps(alb, dg, src, out, args.steps, opts)
        log("%s: %.3f ms/query, rounds %d, huge v %d, kernel %.3f ms" % (
            label, 1e3 * sec / args.steps, stats[-1]["rounds"], stats[-1]["huge_vertices"],
            stats[-1]["kernel_ms"]))
        return sec, stats

    alb_opts = dict(base_opts, mode="alb", threshold=args.threshold)
    sec, stats = measure(alb_opts, "alb")
    dist = out.cpu().numpy()
    reached = dist < alb.INF
    m_reached = int(g.degrees()[reached].sum())
    if args.only_alb:
        twc_sec, twc_stats, twc_ok = sec, stats, None
    else:
        twc_sec, twc_stats = measure(dict(base_opts, mode="twc"), "twc_only")
        twc_ok = bool(np.array_equal(out.cpu().numpy(), dist))

    # roofline of the traversal kernel: algorithmic bytes of each launch over the
    # launch's own device time (HIP events recorded on the kernel's stream)
    bytes_per = [alb.algorithmic_bytes("sssp", s) for s in stats]
    kms = [s["kernel_ms"] for s in stats]
    achieved = float(np.mean([b / (k * 1e-3) for b, k in zip(bytes_per, kms)])) / 1e9
    # the work-efficient lower bound (each reached edge and vertex once), so that
    # redundant relaxations are not rewarded
    n_reached = int(reached.sum())
    we_bytes = 12 * m_reached + 20 * n_reached
    we_achieved = we_bytes / (float(np.mean(kms)) * 1e-3) / 1e9
    traffic = measured_traffic()

    paper_rule = None
    if not args.only_alb:
        s3, st3 = measure(dict(base_opts, mode="alb", threshold="launched"), "alb t=launched threads")
        paper_rule = {"value": round(args.steps * m_reached / s3 / 1e9, 3), "ms_per_step": round(1e3 * s3 / args.steps, 4),
                      "huge_threshold": st3[-1]["huge_threshold"], "huge_vertices": st3[-1]["huge_vertices"]}

    # the paper's threshold study (Section 6.1): 0 and powers of two, plus the
    # adaptive rule and LB for every vertex
    sweep = lb_all = blocked = None
    if not args.no_sweep and not args.only_alb:
        sweep = {}
        for thr in [0] + [1 << e for e in range(6, 21, 2)] + ["adaptive"]:
            s2, st2 = measure(dict(base_opts, mode="alb", threshold=thr), "alb t=%s" % thr)
            sweep[str(thr)] = round(args.steps * m_reached / s2 / 1e9, 3)
        s4, st4 = measure(dict(base_opts, mode="lb_all"), "lb_all")
        lb_all = {"value": round(args.steps * m_reached / s4 / 1e9, 3), "ms_per_step": round(1e3 * s4 / args.steps, 4)}
        # the blocked distribution of huge edges (Section 4.1) at the default threshold and at t = 64
        blocked = {}
        for thr in (None, 64):
            s5, _ = measure(dict(base_opts, mode="alb", threshold=thr, distribution=1), "blocked t=%s" % thr)
            blocked["default" if thr is None else str(thr)] = round(args.steps * m_reached / s5 / 1e9, 3)

    # the small BFS configuration: RMAT scale 14 from vertex 0, latency-bound
    bfs_small = None
    if not args.only_alb:
        g14 = gg.workload("rmat14")
        d14 = alb.Graph(g14.off, g14.col)
        o14 = torch.empty(g14.n, dtype=torch.int32, device="cuda")
        lv = {}
        for label, opts in (("alb", {}), ("twc_only", {"mode": "twc"})):
            for _ in range(5):
                alb.bfs(d14, 0, out=o14, **opts)
            ts = []
            for _ in range(20):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                alb.bfs(d14, 0, out=o14, **opts)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            lv[label] = float(np.median(ts))
        lev = o14.cpu().numpy()
        m14 = int(g14.degrees()[lev < alb.INF].sum())
        import oracle as _oracle

        bfs_small = {"workload": "bfs_rmat14_ef16_from0", "n": g14.n, "m": g14.m,
                     "latency_us": round(1e6 * lv["alb"], 1), "gteps": round(m14 / lv["alb"] / 1e9, 3),
                     "twc_only_latency_us": round(1e6 * lv["twc_only"], 1),
                     "bit_exact": bool(np.array_equal(lev, _oracle.bfs(g14, 0)))}
        d14.close()

    # a reference rate for the label accesses: plain 8-byte gathers at
    # uniform random indices from a table the size of the label array, as
    # many as the query examined edges (RMAT's destinations are skewed and
    # cache better than uniform ones, so this is a yardstick, not a bound)
    random_access = None
    if not args.only_alb:
        ex = int(np.mean([s["edges_examined"] for s in stats]))
        probe = gather_rate(g.n, ex)
        kernel_rate = ex / (float(np.mean(kms)) * 1e-3)
        # the same gathers at the graph's own destinations (every edge once,
        # in CSR order): the label reads alone, without atomics or balancing
        replay = gather_rate(g.n, 0, idx=torch.from_numpy(g.col.astype(np.int64)).cuda())
        random_access = {"probe": "torch index_select of int64 words at uniform random indices, table = label "
                                  "array (%d words), %d indices" % (g.n, ex),
                         "probe_reads_per_s_g": round(probe / 1e9, 2),
                         "kernel_edges_per_s_g": round(kernel_rate / 1e9, 2),
                         "frac": round(kernel_rate / probe, 3),
                         "csr_order_gather": "the same table gathered at every edge's destination in CSR order",
                         "csr_order_reads_per_s_g": round(replay / 1e9, 2),
                         "frac_of_csr_order": round(kernel_rate / replay, 3)}
        log("uniform random gathers: %.1f G reads/s; destinations in CSR order %.1f G reads/s; kernel %.1f G "
            "edges/s" % (probe / 1e9, replay / 1e9, kernel_rate / 1e9))

    cpu = None
    if not args.no_cpu:
        import oracle

        # the same query repeated until about 10 s of CPU work (at most 8 times),
        # the process pinned to one core meanwhile
        saved = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(saved)})
        reps, cpu_s = 0, 0.0
        try:
            while reps < 8 and (reps == 0 or cpu_s < 10.0):
                t0 = time.perf_counter()
                ref = oracle.sssp(g, src)
                cpu_s += time.perf_counter() - t0
                reps += 1
        finally:
            os.sched_setaffinity(0, saved)
        assert np.array_equal(ref, dist), "GPU result differs from the oracle"
        cpu = {"value": round(reps * m_reached / cpu_s / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "host_cpu": host_cpu_model(), "host_cores": os.cpu_count(),
               "sample": "%d full SSSP queries (binary-heap Dijkstra, single thread pinned to one core) on the "
                         "same graph and source, %.2f s in all" % (reps, cpu_s)}

    value = args.steps * m_reached / sec / 1e9
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "sssp_rmat22_ef16_w1-100", "n": g.n, "m": g.m, "source": src,
                   "m_reached": m_reached, "mode": "alb", "huge_threshold": stats[-1]["huge_threshold"],
                   "launched_threads": stats[-1]["launched_threads"], "rounds": stats[-1]["rounds"],
                   "kernel_launches": stats[-1]["kernel_launches"]},
        "twc_only": {"value": round(args.steps * m_reached / twc_sec / 1e9, 3),
                     "ms_per_step": round(1e3 * twc_sec / args.steps, 4), "same_result": twc_ok,
                     "kernel_ms": round(float(np.mean([s["kernel_ms"] for s in twc_stats])), 4)},
        "alb_paper_threshold_rule": paper_rule,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_persistent<256, OpSSSP>" if stats[-1]["kernel_launches"] == 1 else "host loop",
                     "algorithmic_bytes_per_launch": int(np.mean(bytes_per)),
                     "work_efficient_bytes": we_bytes, "work_efficient_gbs": round(we_achieved, 1),
                     "work_efficient_frac": round(we_achieved / HBM_PEAK_GBS, 4),
                     "kernel_ms": round(float(np.mean(kms)), 4)},
        "random_access": random_access,
        "cpu_baseline": cpu,
        "alb_stats": {k: stats[-1][k] for k in ("frontier_vertices", "edges_examined", "huge_vertices",
                                                  "huge_edges", "pushes")},
        # the paper's convention (median of the timed queries) and relaxations
        # (examined edges) per second of kernel time
        "median_ms_per_query_kernel": round(float(np.median(kms)), 4),
        "relaxations_per_s_g": round(float(np.mean([s["edges_examined"] for s in stats])) /
                                     (float(np.mean(kms)) * 1e-3) / 1e9, 2),
    }
    if sweep is not None:
        res["threshold_sweep_gteps"] = sweep
        res["lb_all"] = lb_all
        res["blocked_distribution_gteps"] = blocked
    if bfs_small is not None:
        res["bfs_small"] = bfs_small
    dg.close()
    del g
    if not args.only_alb and not args.no_extras:
        # the other configurations of the metric, each as a nested summary
        # with fewer timed steps (the headline above stays `value`)
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = args.extra_steps, 1
        t = time.perf_counter()
        res["zipf24"] = bench_zipf24(sub, alb, gg, emit=False, cpu=not args.no_cpu, kcore=False, grid=False)
        log("zipf24 summary: %.1fs" % (time.perf_counter() - t))
        t = time.perf_counter()
        res["batch"] = bench_batch(sub, alb, gg, emit=False)
        log("batch summary: %.1fs" % (time.perf_counter() - t))
        t = time.perf_counter()
        sub.requests = 1500
        sub.rates = "100,1000,2000"
        res["serve"] = bench_serve(sub, alb, gg, emit=False)
        log("serve summary: %.1fs" % (time.perf_counter() - t))
    print(json.dumps(res), flush=True)


def host_cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), for the baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gather_rate(words: int, n_idx: int, reps: int = 5, idx=None) -> float:
    """8-byte reads per second that torch's gather sustains from a table of
    `words` int64 words, at uniform random indices or at the given ones
    (event-timed)."""
    import torch

    table = torch.arange(words, dtype=torch.int64, device="cuda")
    if idx is None:
        idx = torch.randint(0, words, (n_idx,), dtype=torch.int64, device="cuda")
    n_idx = int(idx.numel())
    out = torch.empty(n_idx, dtype=torch.int64, device="cuda")
    for _ in range(2):
        torch.index_select(table, 0, idx, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.index_select(table, 0, idx, out=out)
    e1.record()
    torch.cuda.synchronize()
    rate = n_idx * reps / (e0.elapsed_time(e1) * 1e-3)
    del table, idx, out
    return rate


def random_probe(args):
    """What the device sustains for the label access pattern alone: torch's
    gather of 8-byte words at uniformly random indices from tables of the
    RMAT-22 label size (4,194,304 words, 33.5 MB), a quarter of it and 16x
    it, 128M indices per call, timed with events.  A reference point for
    the traversal's random-access rate, not part of it."""
    import torch

    res = {}
    n_idx = 1 << 27
    for words in (1 << 20, 1 << 22, 1 << 26):
        table = torch.arange(words, dtype=torch.int64, device="cuda")
        idx = torch.randint(0, words, (n_idx,), dtype=torch.int64, device="cuda")
        out = torch.empty(n_idx, dtype=torch.int64, device="cuda")
        for _ in range(2):
            torch.index_select(table, 0, idx, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.index_select(table, 0, idx, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        res[str(words * 8)] = {"ms": round(ms, 3), "random_reads_per_s_g": round(n_idx / ms / 1e6, 2),
                               "stream_gbs": round(16 * n_idx / ms / 1e6, 1)}
        log("table %d MB: %.3f ms, %.2f G random reads/s" % (words * 8 >> 20, ms, n_idx / ms / 1e6))
    print(json.dumps({"random_probe": res, "indices": n_idx}), flush=True)


def relax_probe(args):
    """The SSSP edge-relaxation loop alone (paper_1911_09135_amd/csrc/
    probe_relax.hip): every edge of RMAT-22 once in CSR order, balanced, with
    no inspection, bins, pushes or barriers; 8-byte label words with an atomic
    minimum (the traversal's), 8-byte gathers only, and the same with 4-byte
    labels; labels in one array ("flat") or split into eight destination
    slices with XCD x relaxing slice x ("sliced": vertex v goes to slice
    s(v) = the XOR of v's 3-bit digits, which balances RMAT's skewed ids, at
    index s(v) * ceil(n / 8) + (v >> 3)).  Labels start uniform in [0, 1000)
    and candidates are w + 880, so about 7 % of edges lower their label, as
    in the traversal.  Device time per launch (median of 5), G edges/s."""
    import ctypes

    import numpy as np
    import torch

    import graphgen as gg
    from paper_1911_09135_amd import build

    lib_path = build.PROBE_LIB
    if not os.path.exists(lib_path):
        build.build_probe()
    lib = ctypes.CDLL(lib_path)
    vp = ctypes.c_void_p
    lib.alb_probe_relax.argtypes = [ctypes.c_int, vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int, ctypes.c_int32, vp,
                                    vp, ctypes.c_int, vp]
    g = gg.workload("rmat22w")
    n, m = g.n, g.m
    v = np.arange(n, dtype=np.int64)
    s_of = np.zeros(n, np.int64)
    y = v.copy()
    while y.any():
        s_of ^= y & 7
        y >>= 3
    q = (n + 7) // 8
    idx = s_of * q + (v >> 3)  # a bijection onto [0, 8q): v = 8 (i mod q) + (s ^ digits-xor of (i mod q))
    col = g.col.astype(np.int64)
    order = np.argsort(s_of[col], kind="stable")
    cnt = np.bincount(s_of[col], minlength=8)
    list_off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    lab0 = np.random.default_rng(5).integers(0, 1000, n).astype(np.int64)
    dev = "cuda"
    flat = (torch.from_numpy(g.col.astype(np.int32)).to(dev), torch.from_numpy(g.w.astype(np.int32)).to(dev))
    sliced = (torch.from_numpy(idx[col[order]].astype(np.int32)).to(dev),
              torch.from_numpy(g.w[order].astype(np.int32)).to(dev))
    lo_d = torch.from_numpy(list_off).to(dev)
    perm = np.zeros(8 * q, np.int64)
    perm[idx] = lab0
    lab = {(0, 8): torch.from_numpy(lab0 << 32).to(dev), (0, 4): torch.from_numpy(lab0.astype(np.int32)).to(dev),
           (1, 8): torch.from_numpy(perm << 32).to(dev), (1, 4): torch.from_numpy(perm.astype(np.int32)).to(dev)}
    claim = torch.zeros(8 * 64 * 32, dtype=torch.int64, device=dev)
    lowered = torch.zeros(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    names = {0: "8-byte label, atomic min", 1: "8-byte gather only", 2: "4-byte label, atomic min",
             3: "4-byte gather only"}
    res = {}
    for variant in (0, 1, 2, 3):
        for sl in (0, 1):
            src = lab[(sl, 8 if variant < 2 else 4)]
            work = src.clone()
            c, w = sliced if sl else flat
            ts = []
            for it in range(7):
                work.copy_(src)
                claim.zero_()
                lowered.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                rc = lib.alb_probe_relax(variant, c.data_ptr(), w.data_ptr(), work.data_ptr(), m, lo_d.data_ptr(),
                                         sl, 880, claim.data_ptr(), lowered.data_ptr(), 1024, stream)
                e1.record()
                torch.cuda.synchronize()
                if rc != 0:
                    raise RuntimeError("probe launch failed: %d" % rc)
                if it >= 2:
                    ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            key = "%s, %s" % (names[variant], "sliced" if sl else "flat")
            res[key] = {"ms": round(ms, 4), "g_edges_per_s": round(m / ms / 1e6, 1), "lowered": int(lowered.item())}
            log("%-40s %.4f ms  %.1f G edges/s" % (key, ms, m / ms / 1e6))
    print(json.dumps({"relax_probe": res, "graph": "rmat22_ef16_w1-100", "edges": m,
                      "slice_edge_shares": [round(float(x) / m, 4) for x in cnt]}), flush=True)


def bench_batch(args, alb, gg, emit=True):
    """256 SSSP queries (query i on graph i mod 64, a random source of
    out-degree > 0) over 64 weighted RMAT graphs of scales drawn from 12..20,
    all resident in HBM.  A step runs every query once: batched = one
    alb_sssp_batch launch on the graph set; plan = the same batch captured
    once into a HIP graph and replayed (alb_batch_plan_run); one-at-a-time =
    256 alb_sssp calls on the graphs' own handles.  Reported: queries/s of the
    batched step, GTEPS over the edges of reached vertices, per-step latency
    percentiles of the batch and the plan and per-query percentiles of the
    single calls.  Returns the result line (printed when `emit`)."""
    import numpy as np
    import torch

    t = time.perf_counter()
    graphs = gg.rmat_set(64, 12, 20, seed=7)
    members, sources = gg.query_sources(graphs, 256, seed=8)
    log("64 graphs, %d edges in all, generated in %.1fs" % (sum(g.m for g in graphs), time.perf_counter() - t))
    gset = alb.GraphSet(graphs)
    handles = [alb.Graph(g.off, g.col, g.w) for g in graphs]
    outs = [torch.empty(graphs[int(m)].n, dtype=torch.int32, device="cuda") for m in members]
    single_outs = [torch.empty_like(o) for o in outs]
    q = len(members)
    edges = int(sum(graphs[int(m)].m for m in members))  # TEPS over each query's whole graph

    bopts = {} if args.threshold is None else {"threshold": args.threshold}

    def batched():
        return alb.sssp_batch(gset, members, sources, outs=outs, **bopts)[1]

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = batched()
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
    sec = time.perf_counter() - t0
    log("batched: %.3f ms/step, %d rounds, kernel %.3f ms" % (1e3 * sec / args.steps, st["rounds"], st["kernel_ms"]))
    # edges of the vertices each query reached (the GTEPS numerator)
    m_reached = 0
    for i, o in enumerate(outs):
        gi = graphs[int(members[i])]
        m_reached += int(gi.degrees()[o.cpu().numpy() < alb.INF].sum())

    # the same batch captured into a HIP graph once and replayed
    plan_outs = [torch.empty_like(o) for o in outs]
    plan = alb.BatchPlan(gset, "sssp", members, sources, outs=plan_outs, **bopts)
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    plan_s = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        plan.run()
        torch.cuda.synchronize()
        plan_s.append(time.perf_counter() - ts)
    psec = time.perf_counter() - t0
    plan_same = all(bool(torch.equal(a, b)) for a, b in zip(outs, plan_outs))
    plan.close()
    log("plan: %.3f ms/step" % (1e3 * psec / args.steps))

    tuned = None
    if args.tune or not emit:
        # the batch autotuner with per-query thresholds and TWC cutoffs: its
        # best single setting of the grid beside its per-query result
        t0 = time.perf_counter()
        topts, tuning, uniform_ms, tuned_ms = alb.autotune_batch_tuned(gset, "sssp", members, sources)
        tune_s = time.perf_counter() - t0
        tuned_outs = [torch.empty_like(o) for o in outs]
        for _ in range(args.warmup):
            alb.sssp_batch_tuned(gset, members, sources, tuning, outs=tuned_outs, **topts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, tst = alb.sssp_batch_tuned(gset, members, sources, tuning, outs=tuned_outs, **topts)
        torch.cuda.synchronize()
        tsec = time.perf_counter() - t0
        settings = {}
        for t in tuning:
            key = "t=%d,wave=%d,wg=%d" % t
            settings[key] = settings.get(key, 0) + 1
        tuned = {"value": round(args.steps * q / tsec, 1), "unit": "queries/s",
                 "ms_per_step": round(1e3 * tsec / args.steps, 4), "tuning_s": round(tune_s, 2),
                 "wg_size": topts["wg_size"], "settings": settings, "kernel_ms": round(tst["kernel_ms"], 4),
                 "tuner_best_uniform_ms": round(uniform_ms, 4), "tuner_per_query_ms": round(tuned_ms, 4),
                 "same_result": all(bool(torch.equal(a, b)) for a, b in zip(outs, tuned_outs))}
        log("autotuned: %.3f ms/step (tuning %.1fs), wg %d, best uniform %.3f ms, per-query %.3f ms, %s" % (
            1e3 * tsec / args.steps, tune_s, topts["wg_size"], uniform_ms, tuned_ms, settings))

    def one_at_a_time(lat):
        for i in range(q):
            ts = time.perf_counter()
            alb.sssp(handles[int(members[i])], int(sources[i]), out=single_outs[i])
            torch.cuda.synchronize()
            if lat is not None:
                lat.append(time.perf_counter() - ts)

    for _ in range(args.warmup):
        one_at_a_time(None)
    lat1 = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_at_a_time(lat1)
    sec1 = time.perf_counter() - t0
    log("one at a time: %.3f ms/step" % (1e3 * sec1 / args.steps))
    same = all(bool(torch.equal(a, b)) for a, b in zip(outs, single_outs))

    def pct(xs, p):
        return round(1e3 * float(np.percentile(np.asarray(xs), p)), 3)

    value = args.steps * q / sec
    res = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "sssp_batch_256q_64rmat_s12-20_ef16_w1-100", "queries": q, "graphs": len(graphs),
                   "vertices": int(sum(g.n for g in graphs)), "edges": int(sum(g.m for g in graphs)),
                   "rounds": st["rounds"], "launched_threads": st["launched_threads"],
                   "huge_threshold": st["huge_threshold"]},
        "gteps": round(args.steps * m_reached / sec / 1e9, 3),
        "m_reached": m_reached,
        "gteps_whole_graphs": round(args.steps * edges / sec / 1e9, 3),
        "latency_ms": {"p50": pct(step_s, 50), "p99": pct(step_s, 99), "per": "whole batch (256 queries)"},
        "plan": {"value": round(args.steps * q / psec, 1), "unit": "queries/s",
                 "ms_per_step": round(1e3 * psec / args.steps, 4),
                 "gteps": round(args.steps * m_reached / psec / 1e9, 3),
                 "latency_ms": {"p50": pct(plan_s, 50), "p99": pct(plan_s, 99), "per": "whole batch"},
                 "same_result": plan_same},
        "one_at_a_time": {"value": round(args.steps * q / sec1, 1), "unit": "queries/s",
                          "gteps": round(args.steps * m_reached / sec1 / 1e9, 3),
                          "latency_ms": {"p50": pct(lat1, 50), "p99": pct(lat1, 99), "per": "query"},
                          "same_result": same},
        "speedup_vs_one_at_a_time": round(sec1 / sec, 2),
        "autotuned": tuned,
        "batch_stats": {k: st[k] for k in ("frontier_vertices", "edges_examined", "huge_vertices", "huge_edges",
                                             "pushes", "kernel_ms")},
    }
    for h in handles:
        h.close()
    gset.close()
    if emit:
        print(json.dumps(res), flush=True)
    return res


def bench_zipf24(args, alb, gg, emit=True, cpu=False, kcore=True, grid=True, parts=None):
    """The extreme-skew graph: Zipf(1.9) out-degrees capped at 4,194,304,
    n = 2^24 (~372M edges).  BFS from the highest-degree vertex, CC and k-core
    (k = 8, 32) on the symmetrised graph, PageRank (0.85, 50 iterations) by
    push and by pull, each with the default balancer and TWC only; plus a
    2048 x 2048 undirected grid (low skew, high diameter) where the balancer
    should cost nothing.  Times are the traversal kernels' device time (median
    of the steps).  With `cpu`, the oracle's queue BFS on the same graph and
    source, single thread, as the CPU baseline (and the GPU levels checked
    against it).  Returns the result line (printed when `emit`)."""
    import numpy as np
    import torch

    def timed(fn, dg, out, opts, *a):
        for _ in range(max(1, args.warmup)):
            fn(dg, *a, out=out, **opts)
        ks, st = [], None
        for _ in range(args.steps):
            _, st = fn(dg, *a, out=out, **opts)
            ks.append(st["kernel_ms"])
        return float(np.median(ks)), st

    def rates(b, ms):
        return {"achieved_gbs": round(b / ms / 1e6, 1), "frac": round(b / ms / 1e6 / HBM_PEAK_GBS, 4)}

    parts = set((parts or "bfs,pagerank,pull,cc,kcore,grid").split(","))
    kcore = kcore and "kcore" in parts
    grid = grid and "grid" in parts
    res = {}
    t = time.perf_counter()
    g = gg.workload("zipf24")
    src = g.max_degree_vertex()
    deg = g.degrees()
    log("zipf24: n=%d m=%d max_deg=%d (%.1fs)" % (g.n, g.m, deg.max(), time.perf_counter() - t))
    dg = alb.Graph(g.off, g.col)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    alb_opts = {} if args.threshold is None else {"threshold": args.threshold}
    if args.visited_filter != "auto":
        alb_opts["visited_filter"] = args.visited_filter == "on"
    modes = (("alb", alb_opts),) if args.only_alb else (("alb", alb_opts), ("twc_only", {"mode": "twc"}))
    levels = None
    for label, opts in modes if "bfs" in parts else ():
        ms, st = timed(alb.bfs, dg, out, opts, src)
        lv = out.cpu().numpy()
        if levels is None:
            levels = lv
        m_r = int(deg[lv < alb.INF].sum())
        b = alb.algorithmic_bytes("bfs", st)
        res.setdefault("bfs", {})[label] = dict({"kernel_ms": round(ms, 4), "gteps": round(m_r / ms / 1e6, 3),
                                                 "huge_vertices": st["huge_vertices"]}, **rates(b, ms))
        log("bfs %s: %.3f ms" % (label, ms))
    if "bfs" in parts and not args.only_alb:
        # the reached-vertex filter (on by default at this size) switched off
        ms, _ = timed(alb.bfs, dg, out, dict(alb_opts, visited_filter=False), src)
        res["bfs"]["alb_without_filter"] = {"kernel_ms": round(ms, 4),
                                            "same_result": bool(np.array_equal(out.cpu().numpy(), levels))}
        log("bfs alb without the reached-vertex filter: %.3f ms" % ms)
    m_reached = None
    if "bfs" in parts:
        if not args.only_alb:
            res["bfs"]["twc_same_result"] = bool(np.array_equal(lv, levels))
            res["bfs"]["alb_over_twc"] = round(res["bfs"]["twc_only"]["kernel_ms"] / res["bfs"]["alb"]["kernel_ms"],
                                               2)
        m_reached = int(deg[levels < alb.INF].sum())
    cpu_line = None
    if cpu and "bfs" in parts:
        import oracle

        saved = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(saved)})
        reps, cpu_s = 0, 0.0
        try:
            while reps < 4 and (reps == 0 or cpu_s < 8.0):
                t0 = time.perf_counter()
                ref = oracle.bfs(g, src)
                cpu_s += time.perf_counter() - t0
                reps += 1
        finally:
            os.sched_setaffinity(0, saved)
        res["bfs"]["bit_exact"] = bool(np.array_equal(ref, levels))
        cpu_line = {"value": round(reps * m_reached / cpu_s / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
                    "host_cpu": host_cpu_model(), "host_cores": os.cpu_count(),
                    "sample": "%d full BFS queries (FIFO queue, single thread pinned to one core) on the same graph "
                              "and source, %.2f s in all" % (reps, cpu_s)}
        log("cpu oracle bfs: %.2f s per query" % (cpu_s / reps))
    outf = torch.empty(g.n, dtype=torch.float32, device="cuda")
    push_rank = None
    for label, opts in modes if "pagerank" in parts else ():
        ms, st = timed(alb.pagerank, dg, outf, opts, 0.85, 50)
        b = alb.algorithmic_bytes("pagerank", st, n=g.n, iterations=50)
        res.setdefault("pagerank", {})[label] = dict({"kernel_ms": round(ms, 3),
                                                      "gteps": round(50 * g.m / ms / 1e6, 3)}, **rates(b, ms))
        log("pagerank %s: %.3f ms" % (label, ms))
        push_rank = outf.cpu().numpy()
    dg.close()
    # the paper's pr: pull over the in-edges, classified by in-degree
    for label, opts in modes if "pull" in parts else ():
        if label == "alb":
            t = time.perf_counter()
            dt = alb.Graph(g.off, g.col, build_transpose=True)
            log("transposed (%.1fs)" % (time.perf_counter() - t))
        ms, st = timed(alb.pagerank_pull, dt, outf, opts, 0.85, 50)
        b = alb.algorithmic_bytes("pagerank", st, n=g.n, iterations=50)
        res.setdefault("pagerank_pull", {})[label] = dict({"kernel_ms": round(ms, 3),
                                                           "gteps": round(50 * g.m / ms / 1e6, 3),
                                                           "huge_vertices": st["huge_vertices"]}, **rates(b, ms))
        log("pagerank pull %s: %.3f ms" % (label, ms))
    if "pull" in parts:
        if push_rank is not None:
            res["pagerank_pull"]["equals_push"] = bool(np.array_equal(outf.cpu().numpy(), push_rank))
        dt.close()
    ds = None
    if "cc" in parts or kcore:
        t = time.perf_counter()
        ds = alb.Graph(g.off, g.col, build_symmetric=True)
        log("symmetrised: m=%d (%.1fs)" % (ds.m, time.perf_counter() - t))
    for label, opts in modes if "cc" in parts else ():
        ms, st = timed(lambda d, out=None, **o: alb.cc(d, out=out, **o), ds, out, opts)
        b = alb.algorithmic_bytes("cc", st)
        res.setdefault("cc", {})[label] = dict({"kernel_ms": round(ms, 3),
                                                "edges_per_s_g": round(st["edges_examined"] / ms / 1e6, 3),
                                                "gteps": round(ds.m / ms / 1e6, 3), "rounds": st["rounds"]},
                                               **rates(b, ms))
        log("cc %s: %.3f ms" % (label, ms))
    if "cc" in parts and not args.only_alb:
        res["cc"]["alb_over_twc"] = round(res["cc"]["twc_only"]["kernel_ms"] / res["cc"]["alb"]["kernel_ms"], 2)
        # the label-0 filter (on request only)
        lab_ref = out.cpu().numpy()
        ms, _ = timed(lambda d, out=None, **o: alb.cc(d, out=out, **o), ds, out, dict(alb_opts, visited_filter=True))
        res["cc"]["alb_with_label0_filter"] = {"kernel_ms": round(ms, 3),
                                               "same_result": bool(np.array_equal(out.cpu().numpy(), lab_ref))}
        log("cc alb with the label-0 filter: %.3f ms" % ms)
    # k-core (the paper's kcore) on the same symmetrised graph: peeling from
    # every vertex with fewer than k neighbours
    for k in ((8, 32) if kcore else ()):
        for label, opts in modes:
            ms, st = timed(lambda d, kk, out=None, **o: alb.kcore(d, kk, out=out, **o), ds, out, opts, k)
            b = alb.algorithmic_bytes("kcore", st)
            res.setdefault("kcore_k%d" % k, {})[label] = dict({
                "kernel_ms": round(ms, 3), "edges_per_s_g": round(st["edges_examined"] / ms / 1e6, 3),
                "rounds": st["rounds"], "core_vertices": int(out.sum().item())}, **rates(b, ms))
            log("kcore k=%d %s: %.3f ms" % (k, label, ms))
    if ds is not None:
        ds.close()
    del g
    if grid:
        gr = gg.grid(2048, 2048).with_weights(5)
        dgr = alb.Graph(gr.off, gr.col, gr.w)
        outg = torch.empty(gr.n, dtype=torch.int32, device="cuda")
        for kind, fn in (("bfs", alb.bfs), ("sssp", alb.sssp)):
            for label, opts in modes:
                ms, st = timed(fn, dgr, outg, opts, 0)
                res.setdefault("grid2048_" + kind, {})[label] = {"kernel_ms": round(ms, 3), "rounds": st["rounds"],
                                                                 "huge_vertices": st["huge_vertices"]}
                log("grid %s %s: %.3f ms" % (kind, label, ms))
        dgr.close()
    bfs = res["bfs"]["alb"] if "bfs" in res else {"gteps": None, "kernel_ms": None, "achieved_gbs": None,
                                                  "frac": None}
    line = {
        "metric": METRIC,
        "value": bfs["gteps"],
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bfs["kernel_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "zipf1.9_n2^24_cap4194304: bfs, cc, pagerank push and pull%s" %
                               ((", kcore" if kcore else "") + ("; grid2048 bfs, sssp" if grid else "")),
                   "source": src, "m_reached": m_reached},
        "roofline": {"bound": "hbm", "achieved": bfs["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bfs["frac"], "traffic": None},
        "cpu_baseline": cpu_line,
        "results": res,
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


class _BufferPool:
    """Reusable pinned host result arrays per graph, so that allocation and
    page faults do not land in the measured latency."""

    def __init__(self, sizes):
        import threading

        import torch

        self.torch = torch
        self.sizes = sizes
        self.free = {i: [] for i in range(len(sizes))}
        self.lock = threading.Lock()

    def get(self, m):
        with self.lock:
            if self.free[m]:
                return self.free[m].pop()
        # pinned (page-locked) memory: the device copies results at full speed
        a = self.torch.zeros(self.sizes[m], dtype=self.torch.int32, pin_memory=True).numpy()
        return a

    def put(self, m, a):
        with self.lock:
            self.free[m].append(a)


def serve_run(alb, srv, pool, reqs, arrivals, keep=()):
    """Submit reqs[i] at arrivals[i] seconds (None: all at once); returns
    (achieved queries/s, latencies ms, batch sizes, failures); the results of
    the requests whose indices are in `keep` are copied into srv.kept[i]."""
    import threading

    import numpy as np

    keep = set(keep)
    srv.kept = {}
    tickets = [None] * len(reqs)
    ready = threading.Semaphore(0)
    lat, sizes, fails = [], [], [0]
    done_t = [0.0]

    def waiter():
        for i in range(len(reqs)):
            ready.acquire()
            t, buf, m = tickets[i]
            try:
                _, info = srv.wait(t)
                lat.append(info["latency_ms"])
                sizes.append(info["batch_size"])
                if i in keep:
                    srv.kept[i] = np.array(buf, copy=True)
            except alb.AlbError:
                fails[0] += 1
            pool.put(m, buf)
        done_t[0] = time.perf_counter()

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for i, (a, m, s) in enumerate(reqs):
        if arrivals is not None:
            target = t0 + arrivals[i]
            while True:
                dt = target - time.perf_counter()
                if dt <= 0:
                    break
                if dt > 2e-3:
                    time.sleep(dt - 1e-3)
        buf = pool.get(m)
        tickets[i] = (srv.submit(a, m, s, out=buf), buf, m)
        ready.release()
    th.join()
    return len(reqs) / (done_t[0] - t0), np.asarray(lat), np.asarray(sizes), fails[0]


def bench_serve(args, alb, gg, emit=True):
    """Serving: 32 device-resident graphs (30 RMAT of scales 14..22 and Zipf
    graphs of 2^20 and 2^23 vertices, weights U[1,100]); requests BFS:SSSP
    1:1, graph uniform, source uniform over vertices with out-edges.  For each
    arrival rate a Poisson stream goes through the serving loop (2 lanes,
    batches up to 256), through the loop with continuous batching inside a
    launch (join_running: requests join a running launch between rounds) and,
    with fewer requests, through the loop with one request per batch on one
    lane (one launch per query).  Latency runs
    from submit to the result in host memory.  `value` is the batched loop's
    throughput with every request queued at once (its capacity)."""
    import numpy as np

    t = time.perf_counter()
    graphs = gg.serving_set()
    log("32 graphs, %d edges in all, generated in %.1fs" % (sum(g.m for g in graphs), time.perf_counter() - t))
    gset = alb.GraphSet(graphs)
    pool = _BufferPool([g.n for g in graphs])
    nz = [np.nonzero(g.degrees() > 0)[0] for g in graphs]

    def make_requests(count, seed):
        algo = gg.uniform_ints(count, 2, seed, stream=1)
        gi = gg.uniform_ints(count, len(graphs), seed, stream=2)
        u = gg.uniform_doubles(count, seed, stream=3)
        return [("bfs" if algo[i] == 0 else "sssp", int(gi[i]), int(nz[gi[i]][int(u[i] * len(nz[gi[i]]))]))
                for i in range(count)]

    def pct(x, p):
        return round(float(np.percentile(x, p)), 3) if len(x) else None

    batched = alb.Server(gset, lanes=2, max_batch=256, hbm_budget=32 << 30)
    single = alb.Server(gset, lanes=1, max_batch=1, hbm_budget=32 << 30)
    # continuous batching inside a launch: requests join a running launch of
    # their algorithm between rounds and leave when their traversal converges
    if args.join_long_edges > 0:  # long and short requests on lanes of their own
        join_cfg = dict(lanes=2, max_batch=512, join_running=True, join_long_edges=args.join_long_edges)
    else:
        join_cfg = dict(lanes=1, max_batch=512, join_running=True)
    joined = alb.Server(gset, hbm_budget=32 << 30, **join_cfg)
    warm = make_requests(200, 99)
    serve_run(alb, batched, pool, warm, None)
    serve_run(alb, single, pool, warm[:50], None)
    serve_run(alb, joined, pool, warm, None)

    # served results checked against the oracle: a sample of the capacity run's and each stream's
    # requests on the member graphs of at most 2M edges
    import oracle

    checked = {"requests": 0, "equal": 0}

    def sample(r, k=6):
        idx = [i for i, (_, m, _) in enumerate(r) if graphs[m].m <= (2 << 20)]
        return idx[:: max(1, len(idx) // k)][:k]

    def verify(srv, r):
        for i, got in srv.kept.items():
            a, m, src = r[i]
            want = oracle.bfs(graphs[m], src) if a == "bfs" else oracle.sssp(graphs[m], src)
            checked["requests"] += 1
            checked["equal"] += int(np.array_equal(got, want))

    reqs = make_requests(args.requests, 9)
    cap, lat, sizes, f = serve_run(alb, batched, pool, reqs, None, keep=sample(reqs))
    verify(batched, reqs)
    log("batched capacity: %.0f queries/s, p50 %.1f ms, p99 %.1f ms, mean batch %.1f" % (
        cap, pct(lat, 50), pct(lat, 99), sizes.mean()))
    n1 = min(args.requests, 2000)
    cap1, lat1, _, f1 = serve_run(alb, single, pool, reqs[:n1], None)
    log("one-at-a-time capacity: %.0f queries/s" % cap1)
    capj, latj, _, fj = serve_run(alb, joined, pool, reqs, None, keep=sample(reqs))
    verify(joined, reqs)
    log("joining capacity: %.0f queries/s, p50 %.1f ms, p99 %.1f ms" % (capj, pct(latj, 50), pct(latj, 99)))
    rates = []
    for rate in [float(x) for x in args.rates.split(",")]:
        arr = gg.poisson_arrivals(rate, args.requests, seed=9)
        r = make_requests(args.requests, 10 + int(rate))
        thr, l, sz, fb = serve_run(alb, batched, pool, r, arr, keep=sample(r))
        verify(batched, r)
        m1 = min(args.requests, max(200, int(rate * 10)), 2000)
        thr1, l1, _, fs = serve_run(alb, single, pool, r[:m1], arr[:m1])
        thrj, lj, _, fjr = serve_run(alb, joined, pool, r, arr, keep=sample(r))
        verify(joined, r)
        rates.append({"rate": rate, "requests": len(r), "achieved": round(thr, 1), "p50_ms": pct(l, 50),
                      "p99_ms": pct(l, 99), "mean_batch": round(float(sz.mean()), 2), "failed": fb,
                      "join_running": {"achieved": round(thrj, 1), "p50_ms": pct(lj, 50), "p99_ms": pct(lj, 99),
                                       "failed": fjr},
                      "one_at_a_time": {"requests": m1, "achieved": round(thr1, 1), "p50_ms": pct(l1, 50),
                                        "p99_ms": pct(l1, 99), "failed": fs}})
        log("rate %6.0f/s: batched %.0f/s p50 %.2f p99 %.2f ms (batch %.1f); joining %.0f/s p50 %.2f p99 %.2f; "
            "one-at-a-time %.0f/s p50 %.2f p99 %.2f" % (rate, thr, pct(l, 50), pct(l, 99), sz.mean(), thrj,
                                                       pct(lj, 50), pct(lj, 99), thr1, pct(l1, 50), pct(l1, 99)))
    st = batched.stats()
    stj = joined.stats()
    launches_j = len(joined.batch_log())
    batched.close()
    single.close()
    joined.close()
    res = {
        "metric": METRIC,
        "value": round(cap, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": len(warm),
        "ms_per_step": round(1e3 / cap, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "serve_bfs_sssp_32graphs_rmat14-22_zipf20_zipf23", "graphs": len(graphs),
                   "vertices": int(sum(g.n for g in graphs)), "edges": int(sum(g.m for g in graphs)),
                   "lanes": 2, "max_batch": 256},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "mean_batch": round(float(sizes.mean()), 2),
        "failed": f,
        "one_at_a_time": {"value": round(cap1, 1), "unit": "queries/s", "requests": n1,
                          "latency_ms": {"p50": pct(lat1, 50), "p99": pct(lat1, 99)}, "failed": f1},
        "join_running": {"value": round(capj, 1), "unit": "queries/s", "requests": len(reqs),
                         "latency_ms": {"p50": pct(latj, 50), "p99": pct(latj, 99)}, "failed": fj,
                         "launches": launches_j, "completed": stj["completed"],
                         "direct_outputs": stj["direct_outputs"],
                         "lanes": join_cfg["lanes"], "join_long_edges": join_cfg.get("join_long_edges", 0)},
        "poisson": rates,
        "results_checked_against_oracle": checked,
        "server_stats": st,
    }
    gset.close()
    if emit:
        print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()

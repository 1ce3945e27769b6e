"""Summaries of rocprofv3 CSV output (kernel trace statistics, PMC counters).

    python -m paper_1911_09135_amd.rocprof_summary stats DIR
    python -m paper_1911_09135_amd.rocprof_summary traffic --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --kernel k_persistent --out profiles/traffic_X.json
    python -m paper_1911_09135_amd.rocprof_summary overlap DIR --kernel k_persistent

`traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch, summed over the
counter's instances) into bytes per launch of the named kernel, each scaled by
what the same counter reads for a plain device copy of known size (bench.py
--copy-calibration), and records the hash of the kernel source the counters
were taken on (bench.py reports the traffic only while that hash matches).
`overlap` reads the kernel trace and reports, for the dispatches whose name
holds the given text, how long two or more of them ran at the same time on
the device (several serving lanes' launches on their own streams).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(_HERE, "csrc", "alb_kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    for name in sorted(os.listdir(d)):
        if name.endswith(suffix):
            return os.path.join(d, name)
    raise FileNotFoundError("%s/*%s" % (d, suffix))


def kernel_stats(d: str):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"]),
             float(r["Percentage"])) for r in rows]


def counter_per_dispatch(d: str, counter: str):
    """{kernel name: [value per dispatch, ...]} for one counter."""
    rows = list(csv.DictReader(open(_find(d, "counter_collection.csv"))))
    acc = collections.defaultdict(float)
    names = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = (r["Kernel_Name"], r["Dispatch_Id"])
        acc[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    out = collections.defaultdict(list)
    for key, v in acc.items():
        out[names[key]].append(v)
    return out


def _pick(per: dict, substr: str):
    hits = [k for k in per if substr in k]
    if len(hits) != 1:
        raise KeyError("kernel %r matches %s" % (substr, hits))
    return per[hits[0]]


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel, copy_kernel="copyBuffer",
            copy_bytes=1 << 30):
    fk = _pick(counter_per_dispatch(fetch_dir, "FETCH_SIZE"), kernel)
    wk = _pick(counter_per_dispatch(write_dir, "WRITE_SIZE"), kernel)
    fc = _pick(counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE"), copy_kernel)
    wc = _pick(counter_per_dispatch(copy_write_dir, "WRITE_SIZE"), copy_kernel)
    fetch_scale = copy_bytes / (sum(fc) / len(fc) * 1024.0)
    write_scale = copy_bytes / (sum(wc) / len(wc) * 1024.0)
    fetch_b = sum(fk) / len(fk) * 1024.0 * fetch_scale
    write_b = sum(wk) / len(wk) * 1024.0 * write_scale
    return {
        "kernel": kernel,
        "dispatches": [len(fk), len(wk)],
        "fetch_size_kib_per_dispatch": sum(fk) / len(fk),
        "write_size_kib_per_dispatch": sum(wk) / len(wk),
        "copy_calibration_bytes": copy_bytes,
        "fetch_scale": round(fetch_scale, 4),
        "write_scale": round(write_scale, 4),
        "fetch_bytes_per_launch": int(fetch_b),
        "write_bytes_per_launch": int(write_b),
        "bytes_per_launch": int(fetch_b + write_b),
        "kernel_sha256_16": kernel_hash(),
    }


def kernel_intervals(d: str, substr: str):
    """[(start ns, end ns, stream id), ...] of the traced dispatches whose
    kernel name contains `substr`, in start order."""
    rows = list(csv.DictReader(open(_find(d, "kernel_trace.csv"))))
    out = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), int(r["Stream_Id"])) for r in rows
           if substr in r["Kernel_Name"]]
    return sorted(out)


def overlap(intervals):
    """Time with at least one and with at least two of the intervals running,
    the most running at once, and the dispatches per stream (a sweep over the
    start and end points; an end at the same instant as a start counts first)."""
    ev = []
    for b, e, _ in intervals:
        if e > b:
            ev.append((b, 1))
            ev.append((e, -1))
    ev.sort(key=lambda x: (x[0], x[1]))
    busy = two = 0
    depth = peak = 0
    prev = None
    for t, d in ev:
        if prev is not None:
            if depth >= 1:
                busy += t - prev
            if depth >= 2:
                two += t - prev
        depth += d
        peak = max(peak, depth)
        prev = t
    per_stream = collections.Counter(s for _, _, s in intervals)
    return {"dispatches": len(intervals), "streams": dict(sorted(per_stream.items())),
            "kernel_ns_summed": sum(max(e - b, 0) for b, e, _ in intervals), "busy_ns": busy,
            "two_or_more_ns": two, "most_at_once": peak}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-mib", type=int, default=1024)
    t.add_argument("--out")
    o = sub.add_parser("overlap")
    o.add_argument("dir")
    o.add_argument("--kernel", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        print("| Kernel | Calls | Average ns | Min ns | Max ns | % |")
        print("|---|---|---|---|---|---|")
        for name, calls, avg, mn, mx, pct in kernel_stats(a.dir):
            print("| %s | %d | %.0f | %.0f | %.0f | %.2f |" % (name, calls, avg, mn, mx, pct))
    elif a.cmd == "overlap":
        print(json.dumps(overlap(kernel_intervals(a.dir, a.kernel)), indent=1))
    else:
        res = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.kernel, copy_bytes=a.copy_mib << 20)
        text = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
        print(text)


if __name__ == "__main__":
    main()

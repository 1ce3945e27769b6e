"""bench.py's command-line contract, on the CPU: more than one GPU is refused
with a message (there is no multi-GPU path), the roofline helpers read the
committed counter summary only when it was taken on the current kernel
source, and the algorithmic byte model adds up as documented."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_matches_the_kernel_source():
    import bench

    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    if t["kernel_sha256_16"] == bench.kernel_hash():
        assert bench.measured_traffic() == t["bytes_per_launch"]
    else:
        # counters taken on an older kernel source are not reported
        assert bench.measured_traffic() is None


def test_algorithmic_bytes_model():
    from paper_1911_09135_amd import alb

    st = {"frontier_vertices": 10, "edges_examined": 100, "pushes": 7}
    assert alb.algorithmic_bytes("sssp", st) == 16 * 10 + 12 * 100 + 4 * 7
    assert alb.algorithmic_bytes("bfs", st) == 16 * 10 + 8 * 100 + 4 * 7
    assert alb.algorithmic_bytes("kcore", st) == alb.algorithmic_bytes("cc", st) == alb.algorithmic_bytes("bfs", st)
    assert alb.algorithmic_bytes("pagerank", st, n=5, iterations=3) == 8 * 100 + 24 * 5 * 3


def test_rocprof_overlap_sweep():
    """The lane-overlap summary of a kernel trace: time with two or more of
    the dispatches running at once, on hand-made intervals."""
    from paper_1911_09135_amd import rocprof_summary as rs
    iv = [(0, 10, 1), (5, 15, 2), (15, 20, 1), (30, 40, 2), (32, 34, 1), (33, 35, 3)]
    r = rs.overlap(iv)
    assert r["busy_ns"] == 20 + 10
    assert r["two_or_more_ns"] == 5 + 3  # [5, 10) and [32, 35)
    assert r["most_at_once"] == 3
    assert r["streams"] == {1: 3, 2: 2, 3: 1}
    assert r["kernel_ns_summed"] == 10 + 10 + 5 + 10 + 2 + 2
    assert rs.overlap([])["busy_ns"] == 0

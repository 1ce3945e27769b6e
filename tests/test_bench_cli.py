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


def test_rocprof_traffic_scaling(tmp_path):
    """The HBM-traffic summary on hand-made counter files: per-dispatch sums
    over the counter's instances, averaged over dispatches, scaled by what
    the same counter read for a copy of known size."""
    from paper_1911_09135_amd import rocprof_summary as rs

    def write(d, kernel, counter, per_dispatch):
        d.mkdir()
        with open(d / "run_counter_collection.csv", "w") as f:
            f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
            for i, vals in enumerate(per_dispatch):
                for v in vals:  # one row per counter instance
                    f.write('%d,"%s","%s",%s\n' % (i + 1, kernel, counter, v))
        return str(d)

    gib = 1 << 30
    fk = write(tmp_path / "f", "k_persistent<256>", "FETCH_SIZE", [[100, 300], [200, 200]])  # 400 KiB each
    wk = write(tmp_path / "w", "k_persistent<256>", "WRITE_SIZE", [[50, 50], [30, 70]])  # 100 KiB each
    # the copy's FETCH_SIZE reads half its bytes (factor 2), WRITE_SIZE all of them (factor 1)
    fc = write(tmp_path / "cf", "copyBuffer", "FETCH_SIZE", [[gib / 1024 / 2]])
    wc = write(tmp_path / "cw", "copyBuffer", "WRITE_SIZE", [[gib / 1024]])
    r = rs.traffic(fk, wk, fc, wc, "k_persistent", copy_bytes=gib)
    assert r["dispatches"] == [2, 2]
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    assert r["fetch_bytes_per_launch"] == 400 * 1024 * 2
    assert r["write_bytes_per_launch"] == 100 * 1024
    assert r["bytes_per_launch"] == 400 * 1024 * 2 + 100 * 1024

"""The serving scheduler against a fake executor (no GPU): batching of
requests that arrive while a batch runs, algorithm grouping, max_batch, HBM
footprint admission, timeouts, cancellation, error propagation, concurrent
lanes and draining."""
import threading
import time

import numpy as np
import pytest


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


BYTES_PER_VERTEX, BYTES_PER_QUERY = 44, 64


class Fake:
    """Fills request q's array with algo * 10^6 + member * 1000 + source;
    can hold a batch until released; records every batch."""

    def __init__(self, hold=False, status=0, delay=0.0):
        self.batches = []
        self.lock = threading.Lock()
        self.entered = threading.Event()
        self.release = threading.Event()
        if not hold:
            self.release.set()
        self.status = status
        self.delay = delay

    def __call__(self, algo, members, sources, outs, lane):
        t0 = time.perf_counter()
        self.entered.set()
        self.release.wait(10)
        if self.delay:
            time.sleep(self.delay)
        for m, s, o in zip(members, sources, outs):
            o[:] = algo * 10**6 + m * 1000 + s
        with self.lock:
            self.batches.append((algo, list(zip(members, sources)), lane, t0, time.perf_counter()))
        return self.status


def marker(algo, m, s):
    return {"bfs": 0, "sssp": 1}[algo] * 10**6 + m * 1000 + s


def test_requests_complete_with_their_results(alb):
    f = Fake()
    with alb.Server(None, lanes=2, executor=f, member_vertices=[10, 20, 30]) as srv:
        reqs = []
        rng = np.random.default_rng(1)
        for i in range(60):
            algo = "bfs" if i % 3 else "sssp"
            m = int(rng.integers(3))
            s = int(rng.integers(srv.member_n[m]))
            reqs.append((srv.submit(algo, m, s), algo, m, s))
        for t, algo, m, s in reqs:
            out, info = srv.wait(t)
            assert out.shape == (srv.member_n[m],) and (out == marker(algo, m, s)).all()
            assert info["status"] == 0 and info["batch_size"] >= 1 and info["latency_ms"] >= info["queue_ms"] >= 0
        st = srv.stats()
        assert st["submitted"] == st["completed"] == 60 and st["pending"] == st["running"] == 0
        assert sum(len(b[1]) for b in f.batches) == 60


def test_arrivals_during_a_batch_join_the_next_batch_in_order(alb):
    f = Fake(hold=True)
    with alb.Server(None, lanes=1, max_batch=4, executor=f, member_vertices=[20]) as srv:
        first = srv.submit("bfs", 0, 0)
        assert f.entered.wait(5)
        later = [srv.submit("bfs", 0, s) for s in range(1, 11)]
        f.release.set()
        for t in [first] + later:
            srv.wait(t)
        sizes = [len(b[1]) for b in f.batches]
        assert sizes == [1, 4, 4, 2]
        order = [s for b in f.batches for _, s in b[1]]
        assert order == list(range(11))  # arrival order kept


def test_batches_hold_one_algorithm(alb):
    f = Fake(hold=True)
    with alb.Server(None, lanes=1, executor=f, member_vertices=[10]) as srv:
        t0 = srv.submit("sssp", 0, 9)
        assert f.entered.wait(5)
        ts = [srv.submit("bfs" if i % 2 == 0 else "sssp", 0, i) for i in range(8)]
        f.release.set()
        for t in [t0] + ts:
            srv.wait(t)
        algos = [(b[0], [s for _, s in b[1]]) for b in f.batches]
        assert algos == [(1, [9]), (0, [0, 2, 4, 6]), (1, [1, 3, 5, 7])]


def test_hbm_footprint_admission(alb):
    small, big = 1000, 100000
    lane_budget = 3 * (BYTES_PER_VERTEX * small + BYTES_PER_QUERY)
    f = Fake(hold=True)
    with alb.Server(None, lanes=2, hbm_budget=2 * lane_budget, executor=f, member_vertices=[small, big]) as srv:
        with pytest.raises(alb.AlbError) as e:
            srv.submit("bfs", 1, 0)  # alone larger than a lane's share
        assert e.value.status == alb.ALB_E_NOMEM
        ts = [srv.submit("bfs", 0, i) for i in range(10)]
        f.release.set()
        for t in ts:
            srv.wait(t)
        assert max(len(b[1]) for b in f.batches) <= 3
        assert srv.stats()["rejected"] == 1


def test_timeout_in_queue(alb):
    f = Fake(hold=True)
    with alb.Server(None, lanes=1, executor=f, member_vertices=[10]) as srv:
        a = srv.submit("bfs", 0, 0)
        assert f.entered.wait(5)
        b = srv.submit("bfs", 0, 1, timeout_ms=20)
        c = srv.submit("bfs", 0, 2, timeout_ms=60000)
        with pytest.raises(alb.AlbError) as e:
            srv.wait(b)
        assert e.value.status == alb.ALB_E_TIMEOUT and e.value.info["lane"] == -1
        f.release.set()
        srv.wait(a)
        out, info = srv.wait(c)
        assert (out == marker("bfs", 0, 2)).all()
        assert srv.stats()["timed_out"] == 1


def test_timeout_expired_by_the_dispatcher(alb):
    """A request whose deadline passes while nobody waits on it is completed
    as timed out when a lane next looks at the queue."""
    f = Fake(hold=True)
    with alb.Server(None, lanes=1, executor=f, member_vertices=[10]) as srv:
        a = srv.submit("bfs", 0, 0)
        assert f.entered.wait(5)
        b = srv.submit("bfs", 0, 1, timeout_ms=5)
        time.sleep(0.05)
        f.release.set()
        srv.wait(a)
        srv.drain()
        assert srv.stats()["timed_out"] == 1
        with pytest.raises(alb.AlbError) as e:
            srv.wait(b)
        assert e.value.status == alb.ALB_E_TIMEOUT
        assert all(s != 1 for b_ in f.batches for _, s in b_[1])


def test_cancel(alb):
    f = Fake(hold=True)
    with alb.Server(None, lanes=1, executor=f, member_vertices=[10]) as srv:
        a = srv.submit("bfs", 0, 0)
        assert f.entered.wait(5)
        b = srv.submit("bfs", 0, 1)
        srv.cancel(b)
        with pytest.raises(alb.AlbError) as e:
            srv.cancel(a)  # already running
        assert e.value.status == alb.ALB_E_INVAL
        f.release.set()
        srv.wait(a)
        with pytest.raises(alb.AlbError) as e:
            srv.wait(b)
        assert e.value.status == alb.ALB_E_CANCELLED
        with pytest.raises(alb.AlbError):
            srv.wait(b)  # each ticket once


def test_executor_error_reaches_every_request_of_the_batch(alb):
    f = Fake(status=-3)
    with alb.Server(None, lanes=1, executor=f, member_vertices=[10]) as srv:
        ts = [srv.submit("sssp", 0, i) for i in range(5)]
        for t in ts:
            with pytest.raises(alb.AlbError) as e:
                srv.wait(t)
            assert e.value.status == alb.ALB_E_DEVICE
        assert srv.stats()["failed"] == 5


def test_lanes_overlap(alb):
    f = Fake(delay=0.2)
    with alb.Server(None, lanes=2, max_batch=1, executor=f, member_vertices=[10]) as srv:
        ts = [srv.submit("bfs", 0, i) for i in range(2)]
        for t in ts:
            srv.wait(t)
    (_, _, l0, a0, b0), (_, _, l1, a1, b1) = f.batches
    assert l0 != l1
    assert max(a0, a1) < min(b0, b1)  # both batches in flight at once


def test_destroy_runs_what_is_queued(alb):
    f = Fake(delay=0.01)
    srv = alb.Server(None, lanes=1, max_batch=2, executor=f, member_vertices=[10])
    for i in range(7):
        srv.submit("bfs", 0, i)
    srv.close()
    assert sum(len(b[1]) for b in f.batches) == 7


def test_max_wait_gathers_a_batch(alb):
    f = Fake()
    with alb.Server(None, lanes=1, max_batch=8, max_wait_us=200000, executor=f, member_vertices=[10]) as srv:
        ts = []
        for i in range(8):
            ts.append(srv.submit("bfs", 0, i))
        for t in ts:
            srv.wait(t)
        assert [len(b[1]) for b in f.batches] == [8]


def test_bad_requests(alb):
    f = Fake()
    with alb.Server(None, lanes=1, executor=f, member_vertices=[10, 5]) as srv:
        for args in [("bfs", 2, 0), ("bfs", 1, 5), ("bfs", -1, 0), ("sssp", 0, -1)]:
            with pytest.raises(alb.AlbError) as e:
                srv.submit(*args)
            assert e.value.status == alb.ALB_E_INVAL
        with pytest.raises(alb.AlbError):
            srv.wait(12345)
    with pytest.raises(alb.AlbError):
        alb.Server(None, lanes=1)  # no graph and no executor
    with pytest.raises(alb.AlbError):
        alb.Server(None, lanes=17, executor=f, member_vertices=[10])


def test_batch_log_records_every_batch(alb):
    f = Fake(delay=0.02)
    with alb.Server(None, lanes=2, max_batch=4, executor=f, member_vertices=[10, 20]) as srv:
        tickets = [srv.submit("bfs" if i % 2 else "sssp", i % 2, 1) for i in range(24)]
        for t in tickets:
            srv.wait(t)
        log = srv.batch_log()
        assert srv.batch_log(3) == log[-3:]
        assert srv.batch_log(0) == []
    assert len(log) == len(f.batches)
    assert sum(r["batch_size"] for r in log) == 24
    assert all(r["device_begin_ms"] == 0 and r["status"] == 0 for r in log)  # no device with an executor
    assert all(0 <= r["host_begin_ms"] <= r["host_end_ms"] for r in log)
    assert {r["lane"] for r in log} == {0, 1}
    # the two lanes ran batches at the same time on the host
    assert any(a["lane"] != b["lane"] and a["host_begin_ms"] < b["host_end_ms"] and
               b["host_begin_ms"] < a["host_end_ms"] for a in log for b in log)


def test_join_running_needs_the_gpu(alb):
    with pytest.raises(alb.AlbError) as ei:
        alb.Server(None, lanes=1, executor=Fake(), member_vertices=[10], join_running=True)
    assert ei.value.status == alb.ALB_E_INVAL
    with pytest.raises(alb.AlbError):
        alb.Server(None, lanes=1, executor=Fake(), member_vertices=[10], join_idle_us=-1)


def test_bad_traversal_options_are_refused_at_create(alb):
    """The server validates its traversal options when it is created, not
    when its first batch runs."""
    with pytest.raises(alb.AlbError) as e:
        alb.Server(None, lanes=1, executor=Fake(), member_vertices=[10], wg_size=128)
    assert e.value.status == alb.ALB_E_UNSUPPORTED
    with pytest.raises(alb.AlbError) as e:
        alb.Server(None, lanes=1, executor=Fake(), member_vertices=[10], wave_cutoff=-3)
    assert e.value.status == alb.ALB_E_INVAL


def test_join_long_edges_needs_join_running_and_two_lanes(alb):
    with pytest.raises(alb.AlbError) as e:
        alb.Server(None, lanes=2, executor=Fake(), member_vertices=[10], join_long_edges=5)
    assert e.value.status == alb.ALB_E_INVAL
    with pytest.raises(alb.AlbError) as e:
        alb.Server(None, lanes=2, executor=Fake(), member_vertices=[10], join_long_edges=-1)
    assert e.value.status == alb.ALB_E_INVAL

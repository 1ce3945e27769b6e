"""alb_sssp_noalloc, the SSSP entry point for callers that cannot allocate:
its workspace lives in the library's per-GPU device scratch array.  Two
calls in a row through the C ABI, the second on a smaller graph (so the
scratch still holds the first call's larger state), each compared with
alb_sssp on the same inputs and with the oracle (int64 Dijkstra), bit for
bit; then a graph whose workspace exceeds the scratch is refused on the
host with ALB_E_NOMEM before any device work."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def alb():
    from paper_1911_09135_amd import alb as m

    return m


CONFIGS = [dict(), dict(threshold=64), dict(mode="twc"), dict(threshold=0, launch="host"),
           dict(threshold=64, wg_size=1024), dict(threshold=1, distribution=1)]


def _check_pair(alb, torch, g, source, cfg):
    dg = alb.Graph(g.off, g.col, g.w)
    try:
        ref_dev = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
        got_dev = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
        _, st_ref = alb.sssp(dg, source, out=ref_dev, **cfg)
        _, st = alb.sssp_noalloc(dg, source, got_dev, **cfg)
        torch.cuda.synchronize()
        ref, got = ref_dev.cpu().numpy(), got_dev.cpu().numpy()
    finally:
        dg.close()
    want = oracle.sssp(g, source)
    assert np.array_equal(ref, want), ("alb_sssp", cfg)
    assert np.array_equal(got, want), ("alb_sssp_noalloc", cfg)
    assert st["rounds"] >= 1 and st["edges_examined"] >= 1
    assert st["device_ms"] == 0.0  # not timed
    return st


def test_two_calls_second_smaller(alb):
    import torch

    big = gg.workload("rmat14").with_weights(2)
    small = gg.rmat(10, 16, seed=3).with_weights(4)
    for cfg in CONFIGS:
        print("noalloc", cfg, flush=True)
        st1 = _check_pair(alb, torch, big, big.max_degree_vertex(), cfg)
        st2 = _check_pair(alb, torch, small, 5, cfg)
        if cfg.get("threshold") in (0, 1, 64):
            assert st1["huge_vertices"] > 0 and st2["huge_vertices"] > 0


def test_larger_than_the_scratch_is_refused(alb):
    import torch

    g = gg.rmat(10, 16, seed=3).with_weights(4)
    dg = alb.Graph(g.off, g.col, g.w)
    try:
        out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
        # a worklist of 2^26 entries needs 1.6 GB of workspace
        with pytest.raises(alb.AlbError) as ei:
            alb.sssp_noalloc(dg, 0, out, worklist_capacity=1 << 26)
        assert ei.value.status == alb.ALB_E_NOMEM
        assert "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool((out == -7).all())  # nothing ran
        # the next call is served normally
        alb.sssp_noalloc(dg, 0, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.sssp(g, 0))
    finally:
        dg.close()

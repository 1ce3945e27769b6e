"""Loading the binding before torch leaves torch's GPU visible: the binding
loads torch first, so one HIP runtime serves both (the other way round torch
reported no GPU in the same process)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.gpu
def test_binding_first_then_torch_sees_the_gpu():
    code = ("from paper_1911_09135_amd import alb\n"
            "import numpy as np, torch\n"
            "assert torch.cuda.is_available()\n"
            "x = torch.zeros(4, dtype=torch.int32, pin_memory=True)\n"
            "g = alb.Graph(np.array([0, 1, 1], np.int32), np.array([1], np.int32))\n"
            "lv, _ = alb.bfs(g, 0)\n"
            "assert list(lv) == [0, 1], lv\n"
            "print('ok')\n")
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr

"""The host runtime under sanitizers, on the CPU: libalb.so's host C++
(argument validation, options, the serving scheduler and its dispatcher
threads) is rebuilt once with AddressSanitizer + UndefinedBehaviorSanitizer
and once with ThreadSanitizer (paper_1911_09135_amd/build.py --sanitize=...),
and the CPU tests of the C ABI and of the serving loop (fake executor) run
against each build with the sanitizer runtime preloaded; any report fails
the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

OPTS = {
    "address": {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
    "thread": {"TSAN_OPTIONS": "halt_on_error=1:report_signal_unsafe=0"},
}


@pytest.mark.parametrize("name", ["address", "thread"])
def test_host_runtime_under_sanitizer(name):
    from paper_1911_09135_amd import build

    lib = build.build(sanitize=name)
    env = dict(os.environ, ALB_LIBRARY=lib, LD_PRELOAD=build.sanitizer_runtime(name), **OPTS[name])
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_server.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out

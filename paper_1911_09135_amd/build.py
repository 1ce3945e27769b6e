"""Build libalb.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1911_09135_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libalb.so")
ARCH = os.environ.get("ALB_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
# device code: no packed-fp32 instructions
DEVICE = ["--offload-arch=%s" % ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# extra device-code defines, e.g. ALB_DEFINES="-DALB_WAVES_PER_EU=6"
DEVICE += os.environ.get("ALB_DEFINES", "").split()

SOURCES = [("alb_kernels.hip", DEVICE), ("alb_noalloc.hip", DEVICE), ("alb_api.cpp", []), ("alb_server.cpp", [])]


# Sanitizer builds of the host runtime (alb_api.cpp, alb_server.cpp): the
# host C++ files are compiled with the sanitizer, the device file as usual,
# into _build/libalb_<name>.so (never the product library).  Load it with
# ALB_LIBRARY=<path> and the sanitizer runtime preloaded (see sanitizer_env).
SANITIZERS = {"address": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
              "thread": ["-fsanitize=thread"]}
SAN_RUNTIME = {"address": "libclang_rt.asan-x86_64.so", "thread": "libclang_rt.tsan-x86_64.so"}


def sanitizer_runtime(name: str) -> str:
    """Path of the clang sanitizer runtime to preload for a sanitizer build."""
    res = subprocess.check_output(["/opt/rocm/llvm/bin/clang", "-print-resource-dir"], text=True).strip()
    for sub in ("lib/linux", "lib/x86_64-unknown-linux-gnu"):
        p = os.path.join(res, sub, SAN_RUNTIME[name])
        if os.path.exists(p):
            return p
    raise FileNotFoundError(SAN_RUNTIME[name])


def build(verbose: bool = False, sanitize: str = "") -> str:
    objdir = os.path.join(HERE, "_build", sanitize) if sanitize else os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    san = SANITIZERS[sanitize] + ["-g", "-fno-omit-frame-pointer"] if sanitize else []
    lib = os.path.join(HERE, "_build", "libalb_%s.so" % sanitize) if sanitize else LIB
    objs = []
    for src, extra in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        if sanitize and src.endswith(".hip"):
            plain = os.path.join(HERE, "_build", src + ".o")
            if os.path.exists(plain) and os.path.getmtime(plain) >= os.path.getmtime(os.path.join(CSRC, src)):
                objs.append(plain)  # device files are built without a sanitizer: reuse the product objects
                continue
        cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC] + COMMON + san + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                                            os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    link_san = (san[:1] + ["-shared-libsan"]) if sanitize else []
    cmd = [HIPCC, "--offload-arch=%s" % ARCH, "-shared", "-fPIC", "-o", tmp] + link_san + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


PROBE_LIB = os.path.join(HERE, "libalb_probe.so")


def build_probe(verbose: bool = False) -> str:
    """The measurement probe of the edge-relaxation loop (bench.py --relax-probe),
    a separate library: it is not part of the traversal."""
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + COMMON + DEVICE + ["-shared", os.path.join(CSRC, "probe_relax.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    san = ""
    for a in sys.argv[1:]:
        if a.startswith("--sanitize="):
            san = a.split("=", 1)[1]
    print(build(verbose="-v" in sys.argv, sanitize=san))

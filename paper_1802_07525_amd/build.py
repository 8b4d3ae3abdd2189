"""Build the HIP library ``_lbm.so`` for gfx950 in-tree.

Each source in ``csrc/`` is compiled by hipcc into ``_build/`` (in
parallel), then linked into ``paper_1802_07525_amd/_lbm.so``.  HIP code is
built with packed FP32 instructions disabled (``-packed-fp32-ops``).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "_lbm.so")
SOURCES = ["kernels.hip", "bio.hip", "geom.cpp", "solver.cpp", "biofilm.cpp", "api.cpp", "server.cpp", "trace.cpp",
           "noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# -ffp-contract=on: multiply-adds are fused per source expression, not
# after inlining, so every instance of a tile function (the single-domain
# kernels' tile shapes, the server's) rounds the same way
COMMON = ["-O3", "-std=c++17", "-ffp-contract=on", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + COMMON + DEVICE + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    lines = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(lines)))
    return obj, "\n".join(lines)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = list(SOURCES)
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    for obj, log in results:
        if verbose and log.strip():
            print(log, flush=True)
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-ldl", "-o", LIB + ".tmp"] + \
          [o for o, _ in results]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

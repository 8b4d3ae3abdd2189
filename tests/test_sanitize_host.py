"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two drivers are built with -fsanitize=address,undefined (no recovery, so a
report fails the run) and run: tests/sanitize/host_driver.cpp over the
library's integer geometry code (geom.cpp: electrodes, biofilm layers, link
masks and lists, percolation, flow domain, reference nodes, descriptor
words, growth picks, rejections), and tests/sanitize/oracle_driver.c over
the FP64 oracle (geometry, fixed steps and steady solves of both solvers in
2-D and 3-D, the stop rule, a short coupled loop).  The library's GPU code
is not built here; it runs under the GPU tests.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ROCM = "/opt/rocm"


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="no HIP headers")
def test_geometry_host_code_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_1802_07525_amd", "csrc")
    inc = ["-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"),
           "-I" + os.path.join(ROOT, "include"), "-I" + csrc]
    obj = str(tmp_path / "geom.o")
    exe = str(tmp_path / "host_driver")
    _run(["g++", "-std=c++17"] + SAN + inc + ["-c", os.path.join(csrc, "geom.cpp"), "-o", obj])
    _run(["g++", "-std=c++17"] + SAN + inc + [os.path.join(HERE, "sanitize", "host_driver.cpp"), obj,
          "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
          "-o", exe])
    assert _run([exe]).strip().endswith("ok")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c99"] + SAN + ["-ffp-contract=off", "-fopenmp", "-I" + os.path.join(ROOT, "oracle"),
          os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2")
    assert _run([exe], env=env).strip().endswith("ok")

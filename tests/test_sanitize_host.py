"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two drivers are built with -fsanitize=address,undefined (no recovery, so a
report fails the run) and run: tests/sanitize/host_driver.cpp over the
library's integer geometry code (geom.cpp: electrodes, biofilm layers, link
masks and lists, percolation, flow domain, reference nodes, descriptor
words, growth picks, rejections), and tests/sanitize/oracle_driver.c over
the FP64 oracle (geometry, fixed steps and steady solves of both solvers in
2-D and 3-D, the stop rule, a short coupled loop).  The library's GPU code
is not built here; it runs under the GPU tests.

The serving loop (server.cpp: submission, preparation threads, the worker's
admission, chunk, snapshot and retirement protocol, the solo lanes,
escalation, polling, draining, statistics) runs on the CPU against
tests/sanitize/server_emu.cpp, which stands in for the HIP runtime (streams
as threads, events, capture and graphs) and for the kernels (a stub stepper
with made-up residual histories); the solo lanes run the real single-domain
solver (solver.cpp, api.cpp) on those kernels.
It is run under ThreadSanitizer (clang's runtime: GCC 11's does not see the
mutex release inside condition-variable timed waits) for both served tile
forms, under AddressSanitizer with UndefinedBehaviorSanitizer, and plainly
several times over, since some interleavings are rare: the emulation found
requests lost at admission (a request prepared out of ticket order between
the worker's choice of the head of the ready queue and its removal), which
left a drain waiting forever, in about one run in thirty.  Two of its
streams inject a device failure (every HIP call fails after a given number
of queued operations): every accepted request must still come back once,
with its result or EDEVICE, and the drain must report the failure.  Under
AddressSanitizer that found a request freed by the caller while a
preparation thread was still building its mask, and, in the solver, a
staging allocation lost when clearing it failed.  Each run ends by
destroying servers with work in flight (queued, being prepared, stepped,
retiring, on the solo lanes, finished and unpolled, polled and unreleased)
and by three coupled biofilm loops at once (lbm_coupled_run: growth picks,
cell updates, warm re-solves of the real solver on the emulated kernels)
and two runs of the hourly model loop with the agent-based biofilm
(lbm_mfc_run: attachment, growth, spreading by random walks; biofilm.cpp).
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
    objs = [str(tmp_path / "geom.o"), str(tmp_path / "trace.o")]
    exe = str(tmp_path / "host_driver")
    for src, obj in zip(("geom.cpp", "trace.cpp"), objs):
        _run(["g++", "-std=c++17"] + SAN + inc + ["-c", os.path.join(csrc, src), "-o", obj])
    _run(["g++", "-std=c++17"] + SAN + inc + [os.path.join(HERE, "sanitize", "host_driver.cpp")] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
          "-ldl", "-o", exe])
    assert _run([exe]).strip().endswith("ok")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c99"] + SAN + ["-ffp-contract=off", "-fopenmp", "-I" + os.path.join(ROOT, "oracle"),
          os.path.join(HERE, "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
    env = dict(os.environ, OMP_NUM_THREADS="2")
    assert _run([exe], env=env).strip().endswith("ok")


CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
EMU_SRC = ["server.cpp", "solver.cpp", "api.cpp", "geom.cpp", "biofilm.cpp", "trace.cpp"]


def _emu_build(tmp_path, name, compiler, flags):
    csrc = os.path.join(ROOT, "paper_1802_07525_amd", "csrc")
    exe = str(tmp_path / name)
    _run([compiler, "-std=c++17", "-g"] + flags +
         ["-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
          "-I" + csrc] + [os.path.join(csrc, f) for f in EMU_SRC] +
         [os.path.join(HERE, "sanitize", "server_emu.cpp"), "-o", exe, "-lpthread", "-ldl"])
    return exe


def _emu_run(exe, scale, ty, extra_env=None):
    # ty 16: the FP32 forms may take 64 x 16 tiles; the server then switches
    # between the forms as its table crosses 12 such tiles
    env = dict(os.environ, EMU_SERVED_TILE_TY=str(ty), LBM_SERVED_WIDE_MIN_TILES="12", **(extra_env or {}))
    out = _run([exe, str(scale)], env=env, timeout=600)
    assert out.strip().endswith("ok"), out[-2000:]
    return out


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no clang")
@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="no HIP headers")
def test_server_emulation_under_tsan(tmp_path):
    """Both served tile forms: 64 x 4 paired launches only, and chunks that
    switch between those and the 64 x 16 four-step plan (two-step launches
    first when K / 4 is odd) as the table grows and shrinks."""
    exe = _emu_build(tmp_path, "emu_tsan", CLANG, ["-O1", "-fsanitize=thread"])
    # the second run opens roctx ranges on every thread (stub marker library)
    stub = str(tmp_path / "libroctx_stub.so")
    _run(["gcc", "-std=c99", "-O1", "-fPIC", "-shared", os.path.join(HERE, "sanitize", "roctx_stub.c"),
          "-o", stub, "-lpthread"])
    for ty, extra in ((4, {}), (16, {"LBM_ROCTX": stub})):
        _emu_run(exe, 2, ty, dict(TSAN_OPTIONS="halt_on_error=1:abort_on_error=1", **extra))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="no HIP headers")
def test_server_emulation_under_asan_ubsan(tmp_path):
    exe = _emu_build(tmp_path, "emu_asan", "g++", SAN)
    for ty in (4, 16):
        _emu_run(exe, 2, ty)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="no HIP headers")
def test_server_emulation_repeated(tmp_path):
    """Plain build, several runs of about 550 requests each: every request
    is returned once, with the steps, lane and fields its history gives."""
    exe = _emu_build(tmp_path, "emu_plain", "g++", ["-O1"])
    for k in range(4):
        _emu_run(exe, 4, 16 if k % 2 else 4)


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no g++/gcc")
@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="no HIP headers")
def test_roctx_ranges_balanced_on_every_thread(tmp_path):
    """roctx ranges (LBM_ROCTX) around the host phases, loaded by dlopen:
    the emulated serving loop, coupled loops and hourly model loop run with
    tests/sanitize/roctx_stub.c as the marker library.  Every phase's range
    opens, every push has its pop on its own thread, no thread ends with a
    range open; without LBM_ROCTX the marker library is never loaded."""
    stub = str(tmp_path / "libroctx_stub.so")
    _run(["gcc", "-std=c99", "-O1", "-fPIC", "-shared", os.path.join(HERE, "sanitize", "roctx_stub.c"),
          "-o", stub, "-lpthread"])
    exe = _emu_build(tmp_path, "emu_roctx", "g++", ["-O1"])
    out = str(tmp_path / "ranges.txt")
    _emu_run(exe, 1, 16, {"LBM_ROCTX": stub, "ROCTX_STUB_OUT": out})
    rec = {}
    names = {}
    for line in open(out):
        f = line.split()
        if f[0] == "range":
            names[f[1]] = int(f[2])
        else:
            rec[f[0]] = int(f[1])
    assert rec["pushes"] > 0 and rec["pushes"] == rec["pops"], rec
    assert rec["bad_pops"] == 0 and rec["unbalanced"] == 0, rec
    # the steady solves nest inside the served, coupled and hourly phases
    assert rec["max_depth"] >= 2, rec
    for n in ("lbm.fluid.steady", "lbm.ad.steady", "lbm.update_cells", "lbm.coupled.initial",
              "lbm.coupled.update", "lbm.mfc.hour", "lbm.biofilm.step", "lbm.srv.prepare", "lbm.srv.step",
              "lbm.srv.solo"):
        assert names.get(n, 0) > 0, (n, names)
    assert set(names) <= {"lbm.fluid.steady", "lbm.ad.steady", "lbm.update_cells", "lbm.coupled.initial",
                          "lbm.coupled.update", "lbm.mfc.hour", "lbm.biofilm.step", "lbm.srv.prepare",
                          "lbm.srv.step", "lbm.srv.solo", "lbm.srv.escalated", "lbm.geometry"}, names
    # a library that cannot be opened: one message, no ranges, the run unchanged
    env = dict(os.environ, LBM_ROCTX=str(tmp_path / "missing.so"), EMU_SERVED_TILE_TY="4")
    r = subprocess.run([exe, "1"], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stderr.count("cannot open the roctx library") == 1, r.stderr[-2000:]

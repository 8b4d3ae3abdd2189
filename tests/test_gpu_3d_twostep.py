"""Two steps per launch in 3-D: the z-marching kernels against single steps
and against the FP64 oracle (D3Q19 fluid, Sec. 2.1.1; D3Q7 substrate,
Sec. 2.1.2, on the 3-D extension of the anode).

A block owns a 32 x 8 column and marches along z over a segment of planes,
keeping the first step's results in LDS rings.  With FP32 storage (plain
and shifted) the intermediate state stays FP32 and every node runs the same
per-node code as a single step, so two-step launches give the states of two
single steps bit for bit, whatever the segment length.  That is checked
from seeded random states on ragged grids (partial columns in x and y, a
last segment shorter than the others, segments of one plane), and for
steady solves, whose residual checks the two-step kernel takes on its
second step: the same status, step count and state as single steps.  FP16
storage skips one rounding per launch and is held to the oracle at its
5e-3 field bound.

Single-step and segment-length forms are selected through the library's
tuning variables LBM_MAX_LAUNCH_STEPS and LBM_3D_PLANES_PER_BLOCK, read at
solver creation.
"""
import contextlib
import os

import numpy as np
import pytest

import oracle as O
from helpers import masks, rel_l2
from paper_1802_07525_amd import inputs

pytestmark = pytest.mark.gpu

FP32, FP32S, FP16S = 0, 1, 2
NAMES = {FP32: "fp32", FP32S: "fp32s", FP16S: "fp16s"}

C3 = inputs.WORKLOADS["c3"]
# ragged in x and y (45 = 32 + 13, 19 = 2 * 8 + 3); 13 planes
RAG = inputs.scaled(C3, 45, 19, 13, r_min=1, r_max=2, seed=21)
# one full 32 x 16 column (two 32 x 8 ones) over 34 planes
TALL = inputs.scaled(C3, 32, 16, 34, r_min=1, r_max=2, seed=22)


@contextlib.contextmanager
def _env(**kv):
    old = {k: os.environ.get(k) for k in kv}
    try:
        for k, v in kv.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = str(v)
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _solver(lbm, cls, w, storage, planes=None, max_steps=None, ty=None):
    with _env(LBM_3D_PLANES_PER_BLOCK=planes, LBM_MAX_LAUNCH_STEPS=max_steps, LBM_3D_TILE_Y=ty):
        return lbm.Solver(cls, tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"],
                          k_sink=w["k"], storage=storage)


def _random_state(lbm, s, cls, w, seed):
    """Seeded random populations near equilibrium for both solvers, and a
    seeded velocity for the substrate."""
    n = cls.size
    rng = np.random.default_rng(seed)
    u = np.zeros((3, n))
    u[0] = w["u_in"] * (1.0 + 0.5 * rng.random(n))
    u[1:] = 0.004 * (rng.random((2, n)) - 0.5)
    u[:, cls.ravel() != O.FLUID] = 0.0
    wf = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    wa = np.array([1 / 4] + [1 / 8] * 6)
    f = inputs.random_populations(19, n, seed + 1, scale=0.02, base=wf[:, None])
    g = inputs.random_populations(7, n, seed + 2, scale=0.02, base=wa[:, None] * w["c_in"])
    assert s.steps(lbm.LBM_SOLVER_FLUID, 0, cold=1)[0] == 0
    assert lbm.lbm_solver_put(s.h, lbm.LBM_FIELD_F, f) == 0
    assert lbm.lbm_solver_set_u(s.h, u) == 0
    assert s.steps(lbm.LBM_SOLVER_AD, 0, cold=1)[0] == 0
    assert lbm.lbm_solver_put(s.h, lbm.LBM_FIELD_G, g) == 0


def _advance_single(lbm, s, which, n):
    for _ in range(n):
        assert s.steps(which, 1)[0] == 0, s.error()


@pytest.mark.parametrize("ty", [8, 16])
@pytest.mark.parametrize("storage", [FP32, FP32S], ids=NAMES.get)
@pytest.mark.parametrize("w,planes", [(RAG, None), (RAG, 1), (RAG, 3), (RAG, 5), (RAG, 13),
                                      (TALL, None), (TALL, 7)],
                         ids=["rag-default", "rag-1", "rag-3", "rag-5", "rag-13",
                              "tall-default", "tall-7"])
def test_two_step_launches_equal_single_steps(gpu_lib, storage, w, planes, ty):
    lbm = gpu_lib
    cls = masks(w, lbm)
    n = 24
    with _solver(lbm, cls, w, storage, planes=planes, ty=ty) as a, \
            _solver(lbm, cls, w, storage, max_steps=1) as b:
        _random_state(lbm, a, cls, w, 5)
        _random_state(lbm, b, cls, w, 5)
        for which, field in ((lbm.LBM_SOLVER_FLUID, lbm.LBM_FIELD_F), (lbm.LBM_SOLVER_AD, lbm.LBM_FIELD_G)):
            st, _ = a.steps(which, n)          # n / 2 two-step launches
            assert st == 0, a.error()
            _advance_single(lbm, b, which, n)  # n single steps
            fa, fb = a.get(field), b.get(field)
            assert np.isfinite(fa).all()
            assert np.array_equal(fa, fb), (which, np.argwhere(fa != fb)[:5])


@pytest.mark.parametrize("ty", [8, 16])
@pytest.mark.parametrize("storage", [FP32, FP32S], ids=NAMES.get)
def test_two_step_steady_solves_equal_single_step_solves(gpu_lib, storage, ty):
    """Residual checks on the two-step kernel's second step: the stop, the
    step count and the state equal those of single-step launches."""
    lbm = gpu_lib
    w = RAG
    cls = masks(w, lbm)
    with _solver(lbm, cls, w, storage, ty=ty) as a, _solver(lbm, cls, w, storage, max_steps=1) as b:
        ra = a.fluid(2e-5, 40_000)
        rb = b.fluid(2e-5, 40_000)
        assert ra[0] == rb[0] == 0, (ra, rb)
        assert ra[1]["iters"] == rb[1]["iters"] and ra[1]["residual"] == rb[1]["residual"]
        assert np.array_equal(a.get(lbm.LBM_FIELD_F), b.get(lbm.LBM_FIELD_F))
        assert lbm.lbm_solver_export_u(a.h) == 0 and lbm.lbm_solver_export_u(b.h) == 0
        ra = a.ad(2e-5, 40_000)
        rb = b.ad(2e-5, 40_000)
        assert ra[0] == rb[0] == 0, (ra, rb)
        assert ra[1]["iters"] == rb[1]["iters"] and ra[1]["residual"] == rb[1]["residual"]
        assert ra[1]["sink_total"] == rb[1]["sink_total"]
        assert np.array_equal(a.get(lbm.LBM_FIELD_G), b.get(lbm.LBM_FIELD_G))


@pytest.mark.parametrize("storage", [FP32S, FP16S], ids=NAMES.get)
def test_two_step_fixed_steps_match_oracle(gpu_lib, storage):
    """Fixed steps from rest (fluid) and from equilibrium in the oracle's
    velocity (substrate) on the ragged grid, against the FP64 oracle."""
    lbm = gpu_lib
    w = RAG
    cls = masks(w, lbm)
    fl = cls.ravel() == O.FLUID
    act = np.isin(cls.ravel(), [O.FLUID, O.BIOFILM])
    tol = 1e-4 if storage == FP32S else 5e-3
    with _solver(lbm, cls, w, storage) as s:
        assert s.steps(lbm.LBM_SOLVER_FLUID, 300, cold=1)[0] == 0, s.error()
        f_or, _, _ = O.fluid_run(cls, O.fluid_init(cls), w["tau"], w["u_in"], 300)
        U_or, _ = O.fluid_moments(cls, f_or)
        assert rel_l2(s.get(lbm.LBM_FIELD_U), U_or, fl) < tol
        assert lbm.lbm_solver_set_u(s.h, U_or) == 0
        assert s.steps(lbm.LBM_SOLVER_AD, 300, cold=1)[0] == 0
        g_or, _ = O.ad_run(cls, O.ad_init(cls, U_or, w["c_in"]), U_or, w["D"], w["c_in"], w["k"], 300)
        C_or = O.ad_moment(cls, g_or, w["k"])
        assert rel_l2(s.get(lbm.LBM_FIELD_C), C_or, act) < tol


def test_fp16_checked_solve_plan_and_oracle(gpu_lib):
    """FP16 storage in 3-D: a chunk of K steps is (K - 2) / 2 two-step
    launches and two single steps (the check, with tile means over 64 x 4
    tiles of one plane, is a single step); FP16's default K is 1000.  A
    checked solve with tol 0 runs its 2000 steps; the fields stay within the
    FP16 bound of the oracle's 2000 steps."""
    lbm = gpu_lib
    w = RAG
    cls = masks(w, lbm)
    fl = cls.ravel() == O.FLUID
    with _solver(lbm, cls, w, FP16S) as s:
        st, info = s.fluid(0.0, 2000)
        assert st in (1, 2) and info["iters"] % 1000 == 0, (st, info)
        n = info["iters"]
        f_or, _, _ = O.fluid_run(cls, O.fluid_init(cls), w["tau"], w["u_in"], n)
        U_or, _ = O.fluid_moments(cls, f_or)
        assert rel_l2(s.get(lbm.LBM_FIELD_U), U_or, fl) < 5e-3
        assert info["launches"] == (n // 1000) * 501

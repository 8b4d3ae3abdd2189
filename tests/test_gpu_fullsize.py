"""Parity at the benchmark's full sizes and launch configuration.

The 1024 x 512 electrode (the single-solve benchmark) and the 256 x 128 x
128 fibre electrode, compared with the FP64 oracle element by element after
fixed steps, and the 1024 x 512 FP64 steady solve with a loose tolerance
(the residual checks, the stop decision and the iteration count).  On the
2-D grid FP32 storage runs the wide four-step kernels and FP64 the wide
two-step ones (64 x 16 tiles, 1024-thread blocks), FP16 four-step launches fused from
paired ones with its checks over 64 x 4 tiles -- the forms the
benchmark times; the 512 x 256 coupled-loop grid runs the same forms over
middle tiles (64 x 8, 512-thread blocks).
Tolerances as in the smaller parity tests: FP64 1e-12 absolute; FP32 1e-4
and FP16 5e-3 relative L2 on the fields.
"""
import numpy as np
import pytest

import oracle as O
from helpers import masks, rel_l2
from paper_1802_07525_amd import inputs

pytestmark = pytest.mark.gpu

FP32, FP32S, FP16S, FP64 = 0, 1, 2, 3
TOL = {FP64: 1e-12, FP32: 1e-4, FP32S: 1e-4, FP16S: 5e-3}
C2 = inputs.WORKLOADS["c2"]
C3 = inputs.WORKLOADS["c3"]


def _solver(lbm, cls, w, storage, ad9=False):
    return lbm.Solver(cls, tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"], k_sink=w["k"],
                      storage=storage, ad_lattice=1 if ad9 else 0)


def _fixed(lbm, w, storage, nf, na, ad9=False):
    cls = masks(w, lbm)
    print("full size %s storage %d ad9 %s: %d + %d steps" % (w["name"], storage, ad9, nf, na),
          flush=True)
    lat = O.D2Q9 if ad9 else None
    with _solver(lbm, cls, w, storage, ad9) as s:
        assert s.steps(0, nf, 1)[0] == 0, s.error()
        assert lbm.lbm_solver_export_u(s.h) == 0
        assert s.steps(1, na, 1)[0] == 0, s.error()
        U = s.get(lbm.LBM_FIELD_U)
        C = s.get(lbm.LBM_FIELD_C)
    f, _, _ = O.fluid_run(cls, O.fluid_init(cls), w["tau"], w["u_in"], nf)
    Uo, _ = O.fluid_moments(cls, f)
    g, _ = O.ad_run(cls, O.ad_init(cls, Uo, w["c_in"], lat=lat), Uo, w["D"], w["c_in"], w["k"], na,
                    lat=lat)
    Co = O.ad_moment(cls, g, w["k"], lat=lat)
    return cls, U, C, Uo.reshape(U.shape), Co


def _check(storage, cls, U, C, Uo, Co):
    act = np.isin(cls.reshape(-1), [O.FLUID, O.BIOFILM])
    if storage == FP64:
        assert np.abs(U - Uo).max() < TOL[FP64]
        assert np.abs(C - Co)[act].max() < TOL[FP64]
    else:
        assert rel_l2(U, Uo) < TOL[storage]
        assert rel_l2(C, Co, act) < TOL[storage]


@pytest.mark.parametrize("storage", [FP64, FP32S, FP16S], ids=["fp64", "fp32s", "fp16s"])
def test_c2_full_size_fixed_steps(gpu_lib, storage):
    cls, U, C, Uo, Co = _fixed(gpu_lib, C2, storage, 40, 40)
    _check(storage, cls, U, C, Uo, Co)


def test_c2_full_size_d2q9_substrate(gpu_lib):
    """The paper's D2Q9 substrate (its own words, the wide four-step kernel)."""
    cls, U, C, Uo, Co = _fixed(gpu_lib, C2, FP32S, 40, 40, ad9=True)
    _check(FP32S, cls, U, C, Uo, Co)


def test_c2_full_size_fp64_steady(gpu_lib):
    """The checks of the wide kernels (their 1024-thread block maxima)
    decide each stop at the oracle's step: fluid to 1e-2 (3 checks),
    substrate to 1e-3 (32 checks)."""
    lbm = gpu_lib
    cls = masks(C2, lbm)
    with _solver(lbm, cls, C2, FP64) as s:
        st, fi = s.fluid(1e-2, 20000)
        assert st == 0, s.error()
        U = s.get(lbm.LBM_FIELD_U)
        st, ai = s.ad(1e-3, 20000)
        assert st == 0, s.error()
        C = s.get(lbm.LBM_FIELD_C)
    fo = O.fluid_solve(cls, C2["tau"], C2["u_in"], 1e-2, 20000)
    assert fo["status"] == "OK" and fi["iters"] == fo["iters"]
    assert np.abs(U - fo["U"].reshape(U.shape)).max() < 1e-9
    ao = O.ad_solve(cls, fo["U"], C2["D"], C2["c_in"], C2["k"], 1e-3, 20000)
    assert ao["status"] == "OK" and ai["iters"] == ao["iters"]
    act = np.isin(cls.reshape(-1), [O.FLUID, O.BIOFILM])
    assert np.abs(C - ao["C"])[act].max() < 1e-9


def test_c2_full_size_fp32s_steady_iteration_matched(gpu_lib):
    """FP32 shifted storage takes the multi-step kernels on this grid
    (chunks of 100 steps: 25 four-step launches, the last carrying the
    check).  Fluid to 1e-2, substrate to 1e-3; the oracle then
    runs exactly the GPU's step counts and the fields agree to the FP32
    bound."""
    lbm = gpu_lib
    cls = masks(C2, lbm)
    with _solver(lbm, cls, C2, FP32S) as s:
        st, fi = s.fluid(1e-2, 20000)
        assert st == 0, s.error()
        U = s.get(lbm.LBM_FIELD_U)
        st, ai = s.ad(1e-3, 20000)
        assert st == 0, s.error()
        C = s.get(lbm.LBM_FIELD_C)
    f, _, _ = O.fluid_run(cls, O.fluid_init(cls), C2["tau"], C2["u_in"], fi["iters"])
    Uo, _ = O.fluid_moments(cls, f)
    assert fi["iters"] % 100 == 0 and fi["iters"] >= 200
    assert rel_l2(U, Uo.reshape(U.shape)) < TOL[FP32S]
    g, _ = O.ad_run(cls, O.ad_init(cls, Uo, C2["c_in"]), Uo, C2["D"], C2["c_in"], C2["k"], ai["iters"])
    act = np.isin(cls.reshape(-1), [O.FLUID, O.BIOFILM])
    assert ai["iters"] % 100 == 0 and ai["iters"] >= 200
    assert rel_l2(C, O.ad_moment(cls, g, C2["k"]), act) < TOL[FP32S]


@pytest.mark.parametrize("steps", [1, 2, 3, 4, 5, 6, 7, 8, 41])
def test_c2_three_step_planning_fixed_steps(gpu_lib, steps):
    """Step counts that end on each launch form (fours, threes, twos, a one)."""
    cls, U, C, Uo, Co = _fixed(gpu_lib, C2, FP32S, steps, 2)
    _check(FP32S, cls, U, C, Uo, Co)


def _paired_plan(n):
    """Launch sizes of the paired form for n steps: twos, a one only where
    two would leave a single step behind."""
    out = []
    while n:
        k = 2 if n >= 2 and n - 2 != 1 else 1
        out.append(k)
        n -= k
    return out


@pytest.mark.parametrize("steps", [8, 41])
@pytest.mark.parametrize("w", ["c2", "c5"], ids=["1024x512-wide", "512x256-middle"])
def test_fp16_fused_launches_equal_paired(gpu_lib, w, steps):
    """FP16 storage on the wide grid fuses paired launches into four-step
    ones, rounding in LDS as the paired store would.  Taking the same steps
    one paired launch per call (each call of one or two steps is a single
    launch) must give the same stored state bit for bit, for both solvers."""
    lbm = gpu_lib
    w = inputs.WORKLOADS[w]
    cls = masks(w, lbm)
    states = []
    for split in (False, True):
        print("fp16 fused vs paired, %s, %d steps, split %s" % (w["name"], steps, split), flush=True)
        with _solver(lbm, cls, w, FP16S) as s:
            for which in (0, 1):
                if which == 1:
                    assert lbm.lbm_solver_export_u(s.h) == 0
                plan = _paired_plan(steps) if split else [steps]
                for i, k in enumerate(plan):
                    assert s.steps(which, k, 1 if i == 0 else 0)[0] == 0, s.error()
            states.append(lbm.lbm_solver_get_state(s.h))
    assert np.array_equal(states[0], states[1])


# Grids whose sides are no multiples of the tile (1000 = 15 * 64 + 40, 530
# = 33 * 16 + 2; 1090 = 17 * 64 + 2, 483 = 30 * 16 + 3: over 512 tiles of
# 64 x 16; 530 x 250, 250 = 31 * 8 + 2: 288 tiles of 64 x 8), so the FP32
# forms take the multi-step kernels over wide or middle tiles: partial
# tiles whose halos leave the grid on the right and top edges.
RAGGED = [inputs.scaled(C2, 1000, 530, seed=23), inputs.scaled(C2, 1090, 483, seed=25),
          inputs.scaled(C2, 530, 250, seed=27)]


@pytest.mark.parametrize("steps", [4, 41])
@pytest.mark.parametrize("storage,ad9", [(FP32, False), (FP32S, False), (FP32S, True)],
                         ids=["fp32", "fp32s", "fp32s-d2q9"])
@pytest.mark.parametrize("w", RAGGED, ids=["1000x530", "1090x483", "530x250-middle"])
def test_ragged_wide_grid_multi_step(gpu_lib, w, storage, ad9, steps):
    """One four-step launch, and 41 steps (nine four-step launches, a three
    and a two), on each solver."""
    lbm = gpu_lib
    cls, U, C, Uo, Co = _fixed(lbm, w, storage, steps, steps, ad9)
    _check(storage, cls, U, C, Uo, Co)


def test_ragged_wide_grid_fp32s_steady(gpu_lib):
    """Steady solves on a ragged wide grid: the checks' per-block maxima
    cover partial tiles (fluid to 1e-2, substrate to 1e-3); the oracle then
    runs the GPU's step counts and the fields agree to the FP32 bound."""
    lbm = gpu_lib
    w = RAGGED[1]
    cls = masks(w, lbm)
    with _solver(lbm, cls, w, FP32S) as s:
        st, fi = s.fluid(1e-2, 20000)
        assert st == 0, s.error()
        U = s.get(lbm.LBM_FIELD_U)
        st, ai = s.ad(1e-3, 20000)
        assert st == 0, s.error()
        C = s.get(lbm.LBM_FIELD_C)
    fo = O.fluid_solve(cls, w["tau"], w["u_in"], 1e-2, 20000)
    # FP32 and FP64 residuals take the same stop decision unless one lies
    # within rounding of the tolerance
    assert abs(fi["iters"] - fo["iters"]) <= 100
    # 100-step chunks of four-step launches
    assert fi["iters"] == 4 * fi["launches"] and ai["iters"] == 4 * ai["launches"]
    f, _, _ = O.fluid_run(cls, O.fluid_init(cls), w["tau"], w["u_in"], fi["iters"])
    Uo, _ = O.fluid_moments(cls, f)
    assert rel_l2(U, Uo.reshape(U.shape)) < TOL[FP32S]
    g, _ = O.ad_run(cls, O.ad_init(cls, Uo, w["c_in"]), Uo, w["D"], w["c_in"], w["k"], ai["iters"])
    act = np.isin(cls.reshape(-1), [O.FLUID, O.BIOFILM])
    assert rel_l2(C, O.ad_moment(cls, g, w["k"]), act) < TOL[FP32S]


@pytest.mark.parametrize("storage", [FP64, FP32S], ids=["fp64", "fp32s"])
def test_c5_full_size_fixed_steps(gpu_lib, storage):
    """512 x 256, the coupled loop's grid: middle tiles (64 x 8, 512-thread
    blocks), four steps per launch in FP32, two in FP64."""
    cls, U, C, Uo, Co = _fixed(gpu_lib, inputs.WORKLOADS["c5"], storage, 60, 60)
    _check(storage, cls, U, C, Uo, Co)


def test_c3_full_size_fixed_steps(gpu_lib):
    cls, U, C, Uo, Co = _fixed(gpu_lib, C3, FP32S, 10, 10)
    _check(FP32S, cls, U, C, Uo, Co)

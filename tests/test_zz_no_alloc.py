"""The no-allocation steady fluid solve against the allocating one.

lbm_fluid_steady_dev_noalloc carves every device buffer of the solve from a
fixed device scratch array and runs the same kernels in the same order as
lbm_fluid_steady_dev, so status, step count and velocity field must be equal
bit for bit.  Two calls in a row (the second on a smaller grid, so that it
reuses the array the first one left behind), a 3-D grid (the two-step
z-marching kernels), and a grid too large for the array (a clear EINVAL).
"""
import numpy as np
import pytest

from helpers import masks
from paper_1802_07525_amd import inputs

pytestmark = pytest.mark.gpu

FP32S, FP64 = 1, 3
C1 = inputs.WORKLOADS["c1"]
C3 = inputs.WORKLOADS["c3"]


def _both(lbm, ctx, w, storage, tol=1e-5, max_iter=200000):
    import torch
    cls = masks(w, lbm)
    grid = (w["nx"], w["ny"], w["nz"])
    dim = 3 if w["nz"] > 1 else 2
    dcls = torch.from_numpy(np.ascontiguousarray(cls.reshape(-1))).cuda()
    ua = torch.zeros((dim, cls.size), dtype=torch.float64, device="cuda")
    ub = torch.full((dim, cls.size), 7.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    sa, ia = lbm.lbm_fluid_steady_dev(ctx, grid, dcls.data_ptr(), w["tau"], w["u_in"], tol, max_iter,
                                      ua.data_ptr(), storage)
    sb, ib = lbm.lbm_fluid_steady_dev_noalloc(ctx, grid, dcls.data_ptr(), w["tau"], w["u_in"], tol,
                                              max_iter, ub.data_ptr(), storage)
    torch.cuda.synchronize()
    return (sa, ia, ua.cpu().numpy()), (sb, ib, ub.cpu().numpy())


@pytest.mark.parametrize("storage", [FP32S, FP64], ids=["fp32s", "fp64"])
def test_noalloc_equals_allocating_solve_twice(gpu_lib, storage):
    lbm = gpu_lib
    ctx = lbm.lbm_ctx_create(0)
    try:
        for w in (inputs.scaled(C1, 256, 128, r_min=3, r_max=6, solid=0.3, seed=61),
                  inputs.scaled(C1, 96, 48, r_min=2, r_max=4, solid=0.25, seed=62)):
            (sa, ia, ua), (sb, ib, ub) = _both(lbm, ctx, w, storage)
            assert sa == 0 and sb == sa, (sa, sb, lbm.lbm_last_error(ctx))
            assert ib["iters"] == ia["iters"] and ib["residual"] == ia["residual"]
            assert ib["flux_in"] == ia["flux_in"] and ib["flux_out"] == ia["flux_out"]
            assert np.array_equal(ub, ua)
    finally:
        lbm.lbm_ctx_destroy(ctx)


def test_noalloc_3d_equals_allocating_solve(gpu_lib):
    lbm = gpu_lib
    ctx = lbm.lbm_ctx_create(0)
    try:
        w = inputs.scaled(C3, 64, 32, 24, r_min=1, r_max=2, seed=63)
        (sa, ia, ua), (sb, ib, ub) = _both(lbm, ctx, w, FP32S)
        assert sa == 0 and sb == sa, (sa, sb, lbm.lbm_last_error(ctx))
        assert ib["iters"] == ia["iters"]
        assert np.array_equal(ub, ua)
    finally:
        lbm.lbm_ctx_destroy(ctx)


def test_noalloc_rejects_a_grid_beyond_the_scratch(gpu_lib):
    import torch
    lbm = gpu_lib
    ctx = lbm.lbm_ctx_create(0)
    try:
        # 2048 x 1024 nodes need ~190 MB: beyond the 64 MiB array
        w = inputs.scaled(C1, 2048, 1024, r_min=4, r_max=8, solid=0.3, seed=64)
        cls = masks(w, lbm)
        dcls = torch.from_numpy(np.ascontiguousarray(cls.reshape(-1))).cuda()
        u = torch.zeros((2, cls.size), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        st, _ = lbm.lbm_fluid_steady_dev_noalloc(ctx, (w["nx"], w["ny"], 1), dcls.data_ptr(), w["tau"],
                                                 w["u_in"], 1e-5, 1000, u.data_ptr(), FP32S)
        assert st == lbm.LBM_EINVAL
        assert "scratch" in lbm.lbm_last_error(ctx)
        # and a call that fits still works afterwards
        w2 = inputs.scaled(C1, 96, 48, r_min=2, r_max=4, solid=0.25, seed=62)
        (sa, ia, ua), (sb, ib, ub) = _both(lbm, ctx, w2, FP32S)
        assert sa == sb == 0 and np.array_equal(ub, ua)
    finally:
        lbm.lbm_ctx_destroy(ctx)

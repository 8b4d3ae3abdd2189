"""The one-shot steady solves of the C ABI (host and device-pointer forms).

lbm_fluid_steady against the oracle's steady fluid solve (FP64: the same
step count, fields to 1e-9); lbm_ad_steady in a seeded random velocity
field shared by both sides, against the oracle's substrate solve; the
device-pointer forms (torch tensors as device memory) equal to the host
forms bit for bit.
"""
import numpy as np
import pytest

import oracle as O
from helpers import masks
from paper_1802_07525_amd import inputs

pytestmark = pytest.mark.gpu

FP32S, FP64 = 1, 3
W = inputs.scaled(inputs.WORKLOADS["c1"], 96, 48, seed=41)


def _velocity(cls):
    """Seeded velocity, zero on nodes the substrate solve does not read."""
    u = inputs.random_velocity(2, cls.size, seed=42, amp=0.01)
    act = np.isin(cls.reshape(-1), [O.FLUID, O.BIOFILM])
    bio = cls.reshape(-1) == O.BIOFILM
    return np.where(act & ~bio, u, 0.0)


def test_fluid_steady_matches_oracle(gpu_lib):
    lbm = gpu_lib
    cls = masks(W, lbm)
    ctx = lbm.lbm_ctx_create(0)
    try:
        st, U, info = lbm.lbm_fluid_steady(ctx, cls, W["tau"], W["u_in"], 1e-8, 100000, FP64)
    finally:
        lbm.lbm_ctx_destroy(ctx)
    assert st == 0
    fo = O.fluid_solve(cls, W["tau"], W["u_in"], 1e-8, 100000)
    assert fo["status"] == "OK" and info["iters"] == fo["iters"]
    assert np.abs(U - fo["U"]).max() < 1e-9


def test_ad_steady_matches_oracle(gpu_lib):
    lbm = gpu_lib
    cls = masks(W, lbm)
    u = _velocity(cls)
    ctx = lbm.lbm_ctx_create(0)
    try:
        st, C, info = lbm.lbm_ad_steady(ctx, cls, u, W["D"], W["c_in"], W["k"], 1e-9, 200000,
                                        storage=FP64)
    finally:
        lbm.lbm_ctx_destroy(ctx)
    assert st == 0
    ao = O.ad_solve(cls, u, W["D"], W["c_in"], W["k"], 1e-9, 200000)
    assert ao["status"] == "OK" and info["iters"] == ao["iters"]
    act = np.isin(cls.reshape(-1), [O.FLUID, O.BIOFILM])
    assert np.abs(C - ao["C"])[act].max() < 1e-9


@pytest.mark.parametrize("storage", [FP32S, FP64], ids=["fp32s", "fp64"])
def test_device_pointer_forms_equal_host_forms(gpu_lib, storage):
    import torch
    lbm = gpu_lib
    cls = masks(W, lbm)
    grid = (cls.shape[1], cls.shape[0], 1)
    u_in = _velocity(cls)
    ctx = lbm.lbm_ctx_create(0)
    try:
        sf, U, fi = lbm.lbm_fluid_steady(ctx, cls, W["tau"], W["u_in"], 1e-6, 400000, storage)
        assert sf >= 0
        sa, C, ai = lbm.lbm_ad_steady(ctx, cls, u_in, W["D"], W["c_in"], W["k"], 1e-6, 400000,
                                      storage=storage)
        assert sa >= 0
        dcls = torch.from_numpy(np.ascontiguousarray(cls.reshape(-1))).cuda()
        dU = torch.zeros((2, cls.size), dtype=torch.float64, device="cuda")
        du = torch.from_numpy(np.ascontiguousarray(u_in)).cuda()
        dC = torch.zeros(cls.size, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        sf2, fi2 = lbm.lbm_fluid_steady_dev(ctx, grid, dcls.data_ptr(), W["tau"], W["u_in"], 1e-6,
                                            400000, dU.data_ptr(), storage)
        sa2, ai2 = lbm.lbm_ad_steady_dev(ctx, grid, dcls.data_ptr(), du.data_ptr(), W["D"],
                                         W["c_in"], W["k"], 1e-6, 400000, dC.data_ptr(),
                                         storage=storage)
        assert sf2 == sf and sa2 == sa
        U2, C2 = dU.cpu().numpy(), dC.cpu().numpy()
    finally:
        lbm.lbm_ctx_destroy(ctx)
    assert fi2["iters"] == fi["iters"] and ai2["iters"] == ai["iters"]
    assert np.array_equal(U2, U) and np.array_equal(C2, C)

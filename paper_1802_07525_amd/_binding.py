"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every ``lbm_*`` function here has the name of the C entry point it calls and
does nothing but convert numpy arrays and Python numbers to C arguments and
results back; all lattice work runs in the HIP library ``_lbm.so``.  The
library must be built (``__graft_entry__.build()`` or
``python paper_1802_07525_amd/build.py``); ``load()`` raises if it is not:
there is no fallback.

Masks are uint8 numpy arrays shaped [ny, nx] (2-D) or [nz, ny, nx] (3-D);
flat fields use the linear index n = x + nx*(y + ny*z).
"""
import ctypes as ct
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lbm.so")

LBM_OK, LBM_NOT_CONVERGED, LBM_STALLED = 0, 1, 2
LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_EBUSY, LBM_ENOTFOUND = -1, -2, -3, -4, -5, -6
LBM_FP32, LBM_FP32_SHIFTED, LBM_FP16_SHIFTED, LBM_FP64, LBM_FP32_SHIFTED_F64 = 0, 1, 2, 3, 4
LBM_FLUID, LBM_SOLID, LBM_WALL, LBM_BIOFILM = 0, 1, 2, 3
LBM_OUT_ZERO_GRADIENT, LBM_OUT_DIRICHLET = 0, 1
LBM_SOLVER_FLUID, LBM_SOLVER_AD = 0, 1
LBM_LANE_BATCH, LBM_LANE_SOLO, LBM_LANE_ESCALATED = 0, 1, 2
(LBM_FIELD_U, LBM_FIELD_RHO, LBM_FIELD_C, LBM_FIELD_CLASS, LBM_FIELD_LINKS_F, LBM_FIELD_LINKS_C,
 LBM_FIELD_F, LBM_FIELD_G, LBM_FIELD_U_DEVICE, LBM_FIELD_DESC) = range(10)

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "STALLED", -1: "EINVAL", -2: "ENOMEM",
                -3: "EDEVICE", -4: "EDIVERGED", -5: "EBUSY", -6: "ENOTFOUND"}


class lbm_grid(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32)]


class lbm_params(ct.Structure):
    _fields_ = [("tau", ct.c_double), ("u_in", ct.c_double), ("D", ct.c_double),
                ("c_in", ct.c_double), ("k_sink", ct.c_double), ("outlet", ct.c_int32),
                ("c_out", ct.c_double), ("storage", ct.c_int32), ("check_every", ct.c_int32),
                ("stall_checks", ct.c_int32), ("k_half", ct.c_double), ("ad_lattice", ct.c_int32)]


class lbm_info(ct.Structure):
    _fields_ = [("iters", ct.c_int64), ("residual", ct.c_double), ("checks", ct.c_int64),
                ("active_nodes", ct.c_int64), ("seconds", ct.c_double),
                ("kernel_ms", ct.c_double), ("launches", ct.c_int64), ("mlups", ct.c_double),
                ("gbps", ct.c_double), ("flux_in", ct.c_double), ("flux_out", ct.c_double),
                ("sink_total", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_disc_params(ct.Structure):
    _fields_ = [("r_min", ct.c_int32), ("r_max", ct.c_int32), ("solid_frac", ct.c_double),
                ("overlap", ct.c_int32)]


class lbm_fibre_params(ct.Structure):
    _fields_ = [("r_min", ct.c_int32), ("r_max", ct.c_int32), ("solid_frac", ct.c_double)]


class lbm_server_cfg(ct.Structure):
    _fields_ = [("pool_bytes", ct.c_size_t), ("max_slots", ct.c_int32), ("storage", ct.c_int32),
                ("check_every", ct.c_int32), ("stall_checks", ct.c_int32),
                ("inflight", ct.c_int32),
                ("prep_threads", ct.c_int32), ("direct_launch", ct.c_int32),
                ("escalate", ct.c_int32), ("solo_nodes", ct.c_int64),
                ("solo_lanes", ct.c_int32)]


class lbm_request(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("cls", ct.c_void_p),
                ("discs", lbm_disc_params), ("seed", ct.c_uint64), ("layer", ct.c_int32),
                ("tau", ct.c_double), ("u_in", ct.c_double), ("D", ct.c_double),
                ("c_in", ct.c_double), ("k_sink", ct.c_double), ("outlet", ct.c_int32),
                ("c_out", ct.c_double), ("tol", ct.c_double), ("max_iter", ct.c_int64),
                ("user", ct.c_uint64), ("k_half", ct.c_double)]


class lbm_result(ct.Structure):
    _fields_ = [("ticket", ct.c_uint64), ("user", ct.c_uint64), ("status", ct.c_int32),
                ("status_fluid", ct.c_int32), ("status_ad", ct.c_int32), ("nx", ct.c_int32),
                ("ny", ct.c_int32), ("iters_fluid", ct.c_int64), ("iters_ad", ct.c_int64),
                ("residual_fluid", ct.c_double), ("residual_ad", ct.c_double),
                ("flux", ct.c_double * 5), ("active_fluid", ct.c_int64),
                ("active_ad", ct.c_int64), ("t_submit", ct.c_double), ("t_admit", ct.c_double),
                ("t_finish", ct.c_double), ("u", ct.POINTER(ct.c_float)),
                ("c", ct.POINTER(ct.c_float)), ("message", ct.c_char * 96),
                ("lane", ct.c_int32), ("first_status", ct.c_int32),
                ("first_iters_fluid", ct.c_int64), ("first_iters_ad", ct.c_int64)]


class lbm_server_stats_t(ct.Structure):
    _fields_ = [("submitted", ct.c_int64), ("finished", ct.c_int64), ("rejected", ct.c_int64),
                ("active", ct.c_int64), ("queued", ct.c_int64), ("chunks", ct.c_int64),
                ("pool_bytes", ct.c_uint64), ("pool_used", ct.c_uint64),
                ("pool_peak", ct.c_uint64), ("lattice_updates", ct.c_double),
                ("busy_seconds", ct.c_double), ("clock", ct.c_double),
                ("solo", ct.c_int64), ("escalated", ct.c_int64), ("chunks_wide", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_bio_params(ct.Structure):
    _fields_ = [(k, ct.c_double) for k in (
        "q_max", "K_s", "M_total", "K_Mox", "Y", "gamma", "m", "I0", "E0", "R_ext", "R_int",
        "A_a", "V_a", "T", "eps", "C0_bio", "c_scale", "dt_hours")]


class lbm_bio_out(ct.Structure):
    _fields_ = [(k, ct.c_double) for k in (
        "I_cell", "V_cell", "V_total", "n_conc", "n_act", "M_ox", "M_red", "biomass",
        "q_total")] + [("n_cells", ct.c_int32), ("root_iters", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


LBM_BIO_CBIO, LBM_BIO_MOX = 0, 1


class lbm_biofilm_params(ct.Structure):
    _fields_ = [("k_ata", ct.c_int32), ("C_max", ct.c_double), ("fr_spr", ct.c_double),
                ("max_walk", ct.c_int32), ("Y_bio", ct.c_double)]


class lbm_biofilm_stats(ct.Structure):
    _fields_ = [("attached", ct.c_int32), ("spread", ct.c_int32), ("walks", ct.c_int32),
                ("abandoned", ct.c_int32), ("new_biofilm", ct.c_int32), ("cells", ct.c_int32),
                ("biomass", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_mfc_interval(ct.Structure):
    _fields_ = [("status_fluid", ct.c_int32), ("status_ad", ct.c_int32),
                ("iters_fluid", ct.c_int64), ("iters_ad", ct.c_int64),
                ("nodes_fluid", ct.c_int64), ("nodes_ad", ct.c_int64),
                ("seconds_solves", ct.c_double), ("seconds_bio", ct.c_double),
                ("seconds_film", ct.c_double),
                ("bio", lbm_bio_out), ("film", lbm_biofilm_stats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_[:9]}
        d.update(bio=self.bio.as_dict(), film=self.film.as_dict())
        return d

P, I32, I64, U64, D, SZ = (ct.c_void_p, ct.c_int, ct.c_int64, ct.c_uint64, ct.c_double,
                           ct.c_size_t)
G = lbm_grid
_SIGS = {
    "lbm_status_str": (ct.c_char_p, [I32]),
    "lbm_version": (ct.c_char_p, []),
    "lbm_ctx_create": (I32, [I32, P, P]),
    "lbm_ctx_destroy": (None, [P]),
    "lbm_last_error": (ct.c_char_p, [P]),
    "lbm_ctx_stream": (P, [P]),
    "lbm_geom_discs": (I32, [G, P, U64, P, P]),
    "lbm_geom_fibres": (I32, [G, P, U64, P, P]),
    "lbm_biofilm_layer": (I32, [G, P]),
    "lbm_links": (I32, [G, P, I32, P]),
    "lbm_link_list": (I64, [G, P, I32, P, I64]),
    "lbm_percolates": (I32, [G, P]),
    "lbm_flow_domain": (I32, [G, P, P]),
    "lbm_growth_pick": (I64, [G, P, P, D]),
    "lbm_splitmix64": (None, [U64, I64, P]),
    "lbm_fluid_steady": (I32, [P, G, P, D, D, D, I64, I32, P, P]),
    "lbm_ad_steady": (I32, [P, G, P, P, D, D, D, I32, D, D, I64, I32, P, P]),
    "lbm_fluid_steady_dev": (I32, [P, G, P, D, D, D, I64, I32, P, P]),
    "lbm_ad_steady_dev": (I32, [P, G, P, P, D, D, D, I32, D, D, I64, I32, P, P]),
    "lbm_fluid_steady_dev_noalloc": (I32, [P, G, P, D, D, D, I64, I32, P, P]),
    "lbm_solver_create": (I32, [P, G, P, P, P]),
    "lbm_solver_destroy": (None, [P]),
    "lbm_solver_fluid": (I32, [P, D, I64, I32, P]),
    "lbm_solver_ad": (I32, [P, D, I64, I32, P]),
    "lbm_solver_steps": (I32, [P, I32, I64, I32, P]),
    "lbm_solver_time_steps": (I32, [P, I32, I32, P]),
    "lbm_solver_export_u": (I32, [P]),
    "lbm_solver_set_u": (I32, [P, P]),
    "lbm_solver_get": (I32, [P, I32, P]),
    "lbm_solver_put": (I32, [P, I32, P]),
    "lbm_solver_device_ptr": (I32, [P, I32, P, P]),
    "lbm_solver_fluxes": (I32, [P, P]),
    "lbm_solver_update_cells": (I32, [P, P, P, I64]),
    "lbm_solver_state_size": (I32, [P, P]),
    "lbm_solver_get_state": (I32, [P, P, SZ]),
    "lbm_solver_put_state": (I32, [P, P, SZ]),
    "lbm_coupled_run": (I32, [P, I32, P, D, I64, P, P, P, P, P]),
    "lbm_bio_create": (I32, [P, P, P, P, P]),
    "lbm_bio_step": (I32, [P, P]),
    "lbm_bio_get": (I32, [P, I32, P]),
    "lbm_bio_set": (I32, [P, P, P, P, I64]),
    "lbm_bio_destroy": (None, [P]),
    "lbm_biofilm_step": (I32, [P, P, U64, P]),
    "lbm_mfc_run": (I32, [P, P, I32, U64, D, I64, P]),
    "lbm_copy_bandwidth": (I32, [P, SZ, I32, P, P]),
    "lbm_server_footprint": (SZ, [I32, I32, I32]),
    "lbm_server_create": (I32, [P, P, P]),
    "lbm_server_submit": (I32, [P, P, P]),
    "lbm_server_poll": (I32, [P, P, I32, P, D]),
    "lbm_result_release": (None, [P, P]),
    "lbm_server_drain": (I32, [P, D]),
    "lbm_server_stats": (I32, [P, P]),
    "lbm_server_error": (ct.c_char_p, [P]),
    "lbm_server_destroy": (None, [P]),
}

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
        lib = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _grid(cls):
    if cls.ndim == 2:
        return lbm_grid(cls.shape[1], cls.shape[0], 1)
    return lbm_grid(cls.shape[2], cls.shape[1], cls.shape[0])


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def status_name(st):
    return STATUS_NAMES.get(int(st), str(st))


class LBMError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__("%s%s" % (status_name(status), (": " + msg) if msg else ""))
        self.status = status


# ------------------------------------------------------------- geometry
def lbm_geom_discs(nx, ny, r_min, r_max, solid_frac, overlap, seed):
    cls = np.zeros((ny, nx), np.uint8)
    ach = ct.c_double()
    p = lbm_disc_params(r_min, r_max, solid_frac, overlap)
    st = load().lbm_geom_discs(lbm_grid(nx, ny, 1), ct.byref(p), ct.c_uint64(seed), _p(cls),
                               ct.byref(ach))
    return st, cls, ach.value


def lbm_geom_fibres(nx, ny, nz, r_min, r_max, solid_frac, seed):
    cls = np.zeros((nz, ny, nx), np.uint8)
    ach = ct.c_double()
    p = lbm_fibre_params(r_min, r_max, solid_frac)
    st = load().lbm_geom_fibres(lbm_grid(nx, ny, nz), ct.byref(p), ct.c_uint64(seed), _p(cls),
                                ct.byref(ach))
    return st, cls, ach.value


def lbm_biofilm_layer(cls):
    out = _u8(cls).copy()
    st = load().lbm_biofilm_layer(_grid(out), _p(out))
    if st:
        raise LBMError(st)
    return out


def lbm_links(cls, which):
    cls = _u8(cls)
    dt = np.uint8 if which == LBM_SOLVER_AD else (np.uint32 if cls.ndim == 3 else np.uint16)
    out = np.zeros(cls.shape, dt)
    st = load().lbm_links(_grid(cls), _p(cls), int(which), _p(out))
    if st:
        raise LBMError(st)
    return out


def lbm_link_list(cls, which):
    cls = _u8(cls)
    n = load().lbm_link_list(_grid(cls), _p(cls), int(which), None, 0)
    if n < 0:
        raise LBMError(n)
    out = np.zeros((max(n, 1), 2), np.int64)
    load().lbm_link_list(_grid(cls), _p(cls), int(which), _p(out), n)
    return out[:n]


def lbm_percolates(cls):
    cls = _u8(cls)
    r = load().lbm_percolates(_grid(cls), _p(cls))
    if r < 0:
        raise LBMError(r)
    return bool(r)


def lbm_flow_domain(cls):
    """Nodes the fluid solver updates: FLUID nodes linked to the outlet
    column.  Returns a bool array of the shape of cls."""
    cls = _u8(cls)
    out = np.zeros(cls.shape, np.uint8)
    st = load().lbm_flow_domain(_grid(cls), _p(cls), _p(out))
    if st:
        raise LBMError(st)
    return out.astype(bool)


def lbm_growth_pick(cls, C, xi):
    cls = _u8(cls)
    return int(load().lbm_growth_pick(_grid(cls), _p(cls), _p(_f64(C)), float(xi)))


def lbm_splitmix64(seed, count):
    out = np.zeros(count, np.uint64)
    load().lbm_splitmix64(ct.c_uint64(seed), int(count), _p(out))
    return out


# ------------------------------------------------------------- contexts
def lbm_ctx_create(device=0, stream=None):
    h = ct.c_void_p()
    st = load().lbm_ctx_create(int(device), stream, ct.byref(h))
    if st:
        raise LBMError(st, "lbm_ctx_create")
    return h


def lbm_ctx_destroy(ctx):
    load().lbm_ctx_destroy(ctx)


def lbm_last_error(ctx):
    return load().lbm_last_error(ctx).decode()


def lbm_fluid_steady(ctx, cls, tau, u_in, tol, max_iter, storage=LBM_FP32_SHIFTED):
    cls = _u8(cls)
    dim = 3 if cls.ndim == 3 else 2
    u = np.zeros((dim, cls.size))
    info = lbm_info()
    st = load().lbm_fluid_steady(ctx, _grid(cls), _p(cls), float(tau), float(u_in), float(tol),
                                 int(max_iter), int(storage), _p(u), ct.byref(info))
    return st, u, info.as_dict()


def lbm_ad_steady(ctx, cls, u, D, c_in, k_sink, tol, max_iter, outlet=LBM_OUT_ZERO_GRADIENT,
                  c_out=0.0, storage=LBM_FP32_SHIFTED):
    cls = _u8(cls)
    C = np.zeros(cls.size)
    info = lbm_info()
    st = load().lbm_ad_steady(ctx, _grid(cls), _p(cls), _p(_f64(u)), float(D), float(c_in),
                              float(k_sink), int(outlet), float(c_out), float(tol), int(max_iter),
                              int(storage), _p(C), ct.byref(info))
    return st, C, info.as_dict()


def lbm_fluid_steady_dev(ctx, grid, cls_ptr, tau, u_in, tol, max_iter, u_ptr,
                         storage=LBM_FP32_SHIFTED):
    """Device-pointer form: grid (nx, ny, nz); cls_ptr and u_ptr are device
    addresses (e.g. tensor.data_ptr()) of uint8 [N] and float64 [dim][N]."""
    info = lbm_info()
    st = load().lbm_fluid_steady_dev(ctx, lbm_grid(*grid), ct.c_void_p(cls_ptr), float(tau),
                                     float(u_in), float(tol), int(max_iter), int(storage),
                                     ct.c_void_p(u_ptr), ct.byref(info))
    return st, info.as_dict()


def lbm_fluid_steady_dev_noalloc(ctx, grid, cls_ptr, tau, u_in, tol, max_iter, u_ptr,
                                 storage=LBM_FP32_SHIFTED):
    """No-allocation form of lbm_fluid_steady_dev (same arguments)."""
    info = lbm_info()
    st = load().lbm_fluid_steady_dev_noalloc(ctx, lbm_grid(*grid), ct.c_void_p(cls_ptr), float(tau),
                                             float(u_in), float(tol), int(max_iter), int(storage),
                                             ct.c_void_p(u_ptr), ct.byref(info))
    return st, info.as_dict()


def lbm_ad_steady_dev(ctx, grid, cls_ptr, u_ptr, D, c_in, k_sink, tol, max_iter, c_ptr,
                      outlet=LBM_OUT_ZERO_GRADIENT, c_out=0.0, storage=LBM_FP32_SHIFTED):
    """Device-pointer form of lbm_ad_steady (device addresses as above;
    c_ptr: float64 [N])."""
    info = lbm_info()
    st = load().lbm_ad_steady_dev(ctx, lbm_grid(*grid), ct.c_void_p(cls_ptr), ct.c_void_p(u_ptr),
                                  float(D), float(c_in), float(k_sink), int(outlet), float(c_out),
                                  float(tol), int(max_iter), int(storage), ct.c_void_p(c_ptr),
                                  ct.byref(info))
    return st, info.as_dict()


def lbm_copy_bandwidth(ctx, nbytes, reps=20):
    g, ms = ct.c_double(), ct.c_double()
    st = load().lbm_copy_bandwidth(ctx, ct.c_size_t(nbytes), int(reps), ct.byref(g), ct.byref(ms))
    if st:
        raise LBMError(st, lbm_last_error(ctx))
    return g.value, ms.value


# --------------------------------------------------------------- solver
def make_params(tau=0.8, u_in=0.01, D=0.1, c_in=1.0, k_sink=0.0, outlet=LBM_OUT_ZERO_GRADIENT,
                c_out=0.0, storage=LBM_FP32_SHIFTED, check_every=0, stall_checks=0, k_half=0.0,
                ad_lattice=0):
    return lbm_params(float(tau), float(u_in), float(D), float(c_in), float(k_sink), int(outlet),
                      float(c_out), int(storage), int(check_every), int(stall_checks), float(k_half),
                      int(ad_lattice))


def lbm_solver_create(ctx, cls, params):
    cls = _u8(cls)
    h = ct.c_void_p()
    st = load().lbm_solver_create(ctx, _grid(cls), _p(cls), ct.byref(params), ct.byref(h))
    if st:
        raise LBMError(st, lbm_last_error(ctx))
    return h


def lbm_solver_destroy(s):
    load().lbm_solver_destroy(s)


def lbm_solver_fluid(s, tol, max_iter, warm=0):
    info = lbm_info()
    st = load().lbm_solver_fluid(s, float(tol), int(max_iter), int(warm), ct.byref(info))
    return st, info.as_dict()


def lbm_solver_ad(s, tol, max_iter, warm=0):
    info = lbm_info()
    st = load().lbm_solver_ad(s, float(tol), int(max_iter), int(warm), ct.byref(info))
    return st, info.as_dict()


def lbm_solver_steps(s, which, nsteps, cold=0):
    ms = ct.c_double()
    st = load().lbm_solver_steps(s, int(which), int(nsteps), int(cold), ct.byref(ms))
    return st, ms.value


def lbm_solver_time_steps(s, which, nsteps):
    ms = ct.c_double()
    st = load().lbm_solver_time_steps(s, int(which), int(nsteps), ct.byref(ms))
    return st, ms.value


def lbm_solver_export_u(s):
    return load().lbm_solver_export_u(s)


def lbm_solver_set_u(s, u):
    return load().lbm_solver_set_u(s, _p(_f64(u)))


_FIELD_SHAPES = {LBM_FIELD_U: ("dim", np.float64), LBM_FIELD_RHO: (1, np.float64),
                 LBM_FIELD_C: (1, np.float64), LBM_FIELD_CLASS: (1, np.uint8),
                 LBM_FIELD_LINKS_C: (1, np.uint8), LBM_FIELD_F: ("qf", np.float64),
                 LBM_FIELD_G: ("qa", np.float64), LBM_FIELD_DESC: (1, np.uint32)}


def lbm_solver_get(s, field, grid, qa=None):
    """grid = (nx, ny, nz).  Returns the field as a numpy array.  qa: the
    substrate lattice's direction count where it is not the default (9 for
    the D2Q9 substrate)."""
    nx, ny, nz = grid
    N = nx * ny * nz
    dim = 3 if nz > 1 else 2
    if field == LBM_FIELD_LINKS_F:
        out = np.zeros(N, np.uint32 if nz > 1 else np.uint16)
    else:
        rows, dt = _FIELD_SHAPES[field]
        rows = {"dim": dim, "qf": 19 if nz > 1 else 9,
                "qa": qa or (7 if nz > 1 else 5)}.get(rows, rows)
        out = np.zeros((rows, N) if rows != 1 else N, dt)
    st = load().lbm_solver_get(s, int(field), _p(out))
    if st:
        raise LBMError(st)
    return out


def lbm_solver_put(s, field, arr):
    return load().lbm_solver_put(s, int(field), _p(_f64(arr)))


def lbm_solver_device_ptr(s, field=LBM_FIELD_U_DEVICE):
    ptr, nb = ct.c_void_p(), ct.c_size_t()
    st = load().lbm_solver_device_ptr(s, int(field), ct.byref(ptr), ct.byref(nb))
    if st:
        raise LBMError(st)
    return ptr.value, nb.value


def lbm_solver_fluxes(s):
    out = np.zeros(5)
    st = load().lbm_solver_fluxes(s, _p(out))
    if st:
        raise LBMError(st)
    return out


def lbm_solver_update_cells(s, idx, new_cls):
    idx = np.ascontiguousarray(idx, np.int64)
    new_cls = _u8(new_cls)
    return load().lbm_solver_update_cells(s, _p(idx), _p(new_cls), len(idx))


def lbm_solver_get_state(s):
    n = ct.c_size_t()
    load().lbm_solver_state_size(s, ct.byref(n))
    buf = np.zeros(n.value, np.uint8)
    st = load().lbm_solver_get_state(s, _p(buf), n.value)
    if st:
        raise LBMError(st)
    return buf


def lbm_solver_put_state(s, buf):
    buf = np.ascontiguousarray(buf, np.uint8)
    return load().lbm_solver_put_state(s, _p(buf), buf.size)


def lbm_coupled_run(s, xi, tol, max_iter):
    xi = _f64(xi)
    M = len(xi)
    picked = np.zeros(M, np.int64)
    J = np.zeros(M + 1)
    itf = np.zeros(M + 1, np.int64)
    ita = np.zeros(M + 1, np.int64)
    acc = ct.c_double()
    st = load().lbm_coupled_run(s, M, _p(xi), float(tol), int(max_iter), _p(picked), _p(J),
                                ct.byref(acc), _p(itf), _p(ita))
    return st, dict(picked=picked, J=J, J_accum=acc.value, iters_fluid=itf, iters_ad=ita)


# ------------------------------------------------- bio-electrochemistry
def make_bio_params(c_scale, **kw):
    """Parameters of the bio-electrochemical model (Sec. 2.2).  Defaults:
    Table 1, with T = 298.15 K, eps = 0.01 M_total, A_a = 48 x 65 mm^2 and
    V_a = 17 x 60 x 65 mm^3; c_scale is mg/L per lattice concentration unit."""
    M_total = kw.pop("M_total", 0.05)
    v = dict(q_max=8.48, K_s=20.0, M_total=M_total, K_Mox=0.02 * M_total, Y=0.5687,
             gamma=663400.0, m=2.0, I0=1e-3, E0=0.7, R_ext=360.0, R_int=360.0,
             A_a=48e-3 * 65e-3, V_a=17 * 60 * 65 * 1e-6, T=298.15, eps=0.01 * M_total,
             C0_bio=450.0, c_scale=float(c_scale), dt_hours=1.0)
    for k, x in kw.items():
        if k not in v:
            raise KeyError(k)
        v[k] = float(x)
    return lbm_bio_params(**v)


def lbm_bio_create(s, params, c_bio=None, m_ox=None, ctx=None):
    h = ct.c_void_p()
    cb = None if c_bio is None else _f64(np.asarray(c_bio).reshape(-1))
    mo = None if m_ox is None else _f64(np.asarray(m_ox).reshape(-1))
    st = load().lbm_bio_create(s, ct.byref(params), _p(cb), _p(mo), ct.byref(h))
    if st:
        raise LBMError(st, lbm_last_error(ctx) if ctx else "")
    return h


def lbm_bio_step(b):
    o = lbm_bio_out()
    st = load().lbm_bio_step(b, ct.byref(o))
    return st, o.as_dict()


def lbm_bio_get(b, field, n_nodes):
    out = np.zeros(int(n_nodes))
    st = load().lbm_bio_get(b, int(field), _p(out))
    if st:
        raise LBMError(st)
    return out


def lbm_bio_set(b, nodes, c_bio, m_ox):
    nodes = np.ascontiguousarray(nodes, np.int64)
    c_bio, m_ox = _f64(c_bio), _f64(m_ox)
    return load().lbm_bio_set(b, _p(nodes), _p(c_bio), _p(m_ox), len(nodes))


def lbm_bio_destroy(b):
    load().lbm_bio_destroy(b)


def make_biofilm_params(k_ata=200, C_max=512.5, fr_spr=0.4, max_walk=10000, Y_bio=1.0):
    """Biofilm formation parameters (Sec. 2.3); defaults from Table 1, and
    Y_bio = 1 (not in Table 1: growth rate per unit biomass = q_a)."""
    return lbm_biofilm_params(int(k_ata), float(C_max), float(fr_spr), int(max_walk),
                              float(Y_bio))


def lbm_biofilm_step(b, params, seed):
    o = lbm_biofilm_stats()
    st = load().lbm_biofilm_step(b, ct.byref(params), ct.c_uint64(int(seed)), ct.byref(o))
    return st, o.as_dict()


def lbm_mfc_run(b, params, n_hours, seed, tol, max_iter):
    """The model loop; returns (status, list of per-interval dicts)."""
    arr = (lbm_mfc_interval * max(int(n_hours), 1))()
    st = load().lbm_mfc_run(b, ct.byref(params), int(n_hours), ct.c_uint64(int(seed)),
                            float(tol), int(max_iter), arr)
    return st, [arr[h].as_dict() for h in range(int(n_hours))]


class Solver:
    """Owning wrapper of an lbm_solver handle (and, if none is given, of its
    context)."""

    def __init__(self, cls, ctx=None, **params):
        self.cls = _u8(cls)
        self.own_ctx = ctx is None
        self.ctx = lbm_ctx_create() if ctx is None else ctx
        g = _grid(self.cls)
        self.grid = (g.nx, g.ny, g.nz)
        self.params = make_params(**params)
        self.h = lbm_solver_create(self.ctx, self.cls, self.params)

    def close(self):
        if self.h:
            lbm_solver_destroy(self.h)
            self.h = None
        if self.own_ctx and self.ctx:
            lbm_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fluid(self, tol, max_iter, warm=0):
        return lbm_solver_fluid(self.h, tol, max_iter, warm)

    def ad(self, tol, max_iter, warm=0):
        return lbm_solver_ad(self.h, tol, max_iter, warm)

    def steps(self, which, nsteps, cold=0):
        return lbm_solver_steps(self.h, which, nsteps, cold)

    def get(self, field):
        return lbm_solver_get(self.h, field, self.grid, qa=9 if self.params.ad_lattice == 1 else None)

    def error(self):
        return lbm_last_error(self.ctx)


# -------------------------------------------------------------- serving
def lbm_server_footprint(nx, ny, storage):
    return int(load().lbm_server_footprint(int(nx), int(ny), int(storage)))


def make_server_cfg(pool_bytes, max_slots=32, storage=LBM_FP16_SHIFTED, check_every=0,
                    stall_checks=0, inflight=0, prep_threads=0, direct_launch=0, escalate=0,
                    solo_nodes=0, solo_lanes=0):
    return lbm_server_cfg(int(pool_bytes), int(max_slots), int(storage), int(check_every),
                          int(stall_checks), int(inflight), int(prep_threads),
                          int(direct_launch), int(escalate), int(solo_nodes), int(solo_lanes))


def make_request(nx, ny, cls=None, r_min=3, r_max=6, solid_frac=0.3, overlap=1, seed=0, layer=0,
                 tau=0.8, u_in=0.01, D=0.2 / 3, c_in=1.0, k_sink=0.0,
                 outlet=LBM_OUT_ZERO_GRADIENT, c_out=0.0, tol=1e-6, max_iter=1000000, user=0,
                 k_half=0.0):
    """Request struct; a given mask is referenced, not copied, until submit
    (the returned pair keeps the array alive)."""
    arr = None if cls is None else _u8(cls)
    r = lbm_request(int(nx), int(ny), None if arr is None else arr.ctypes.data,
                    lbm_disc_params(int(r_min), int(r_max), float(solid_frac), int(overlap)),
                    int(seed), int(layer), float(tau), float(u_in), float(D), float(c_in),
                    float(k_sink), int(outlet), float(c_out), float(tol), int(max_iter), int(user),
                    float(k_half))
    return r, arr


def lbm_server_create(ctx, cfg):
    h = ct.c_void_p()
    st = load().lbm_server_create(ctx, ct.byref(cfg), ct.byref(h))
    if st:
        raise LBMError(st, lbm_last_error(ctx))
    return h


def lbm_server_submit(srv, req):
    """req: (lbm_request, keep-alive) from make_request.  Returns (status, ticket)."""
    r, _keep = req
    t = ct.c_uint64()
    st = load().lbm_server_submit(srv, ct.byref(r), ct.byref(t))
    return st, t.value


def _result_dict(r):
    N = r.nx * r.ny
    d = {k: getattr(r, k) for k, _ in r._fields_ if k not in ("u", "c", "flux", "message")}
    d["flux"] = np.array(r.flux[:])
    d["message"] = r.message.decode(errors="replace")
    d["u"] = np.ctypeslib.as_array(r.u, (2, N)).copy() if r.u else None
    d["c"] = np.ctypeslib.as_array(r.c, (N,)).copy() if r.c else None
    return d


def lbm_server_poll(srv, max_results=64, wait_s=0.0):
    """Finished results as dicts (arrays copied; the server's copies are
    released)."""
    buf = (lbm_result * max_results)()
    n = ct.c_int()
    st = load().lbm_server_poll(srv, buf, int(max_results), ct.byref(n), float(wait_s))
    if st:
        raise LBMError(st)
    out = []
    for k in range(n.value):
        out.append(_result_dict(buf[k]))
        load().lbm_result_release(srv, ct.byref(buf[k]))
    return out


def lbm_server_drain(srv, timeout_s=0.0):
    return load().lbm_server_drain(srv, float(timeout_s))


def lbm_server_stats(srv):
    o = lbm_server_stats_t()
    st = load().lbm_server_stats(srv, ct.byref(o))
    if st:
        raise LBMError(st)
    return o.as_dict()


def lbm_server_error(srv):
    return load().lbm_server_error(srv).decode()


def lbm_server_destroy(srv):
    load().lbm_server_destroy(srv)

"""Python view of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark import this module.  It wraps ``liboracle.so`` (built from
``oracle.c`` by ``oracle/build.py``) with ctypes and numpy; every function
returns plain float64 / integer numpy arrays.  No code here is shared with
the HIP library.

Layouts: grid index n = x + nx*(y + ny*z); populations are [q][N];
velocities [dim][N].  2-D grids use nz = 1.
"""
import ctypes as ct
import os

import numpy as np

from . import build as _build

D2Q9, D2Q5, D3Q19, D3Q7 = 0, 1, 2, 3
FLUID, SOLID, WALL, BIOFILM = 0, 1, 2, 3
STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "STALLED", -1: "EINVAL", -4: "EDIVERGED"}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ct.CDLL(_build.LIB)
        P = ct.c_void_p
        I, I64, D, U64 = ct.c_int, ct.c_int64, ct.c_double, ct.c_uint64
        sig = {
            "orc_lattice_tables": (I, [I, P, P, P, P, P]),
            "orc_feq": (None, [I, D, P, P]),
            "orc_geq": (None, [I, D, P, P]),
            "orc_fluid_init": (I, [I, I, I, I, P, P]),
            "orc_fluid_step": (I, [I, I, I, I, P, D, D, P, P, P, P, P, P]),
            "orc_fluid_moments": (I, [I, I, I, I, P, P, P, P, P]),
            "orc_fluid_fluxes": (I, [I, I, I, I, P, D, P, P, P]),
            "orc_fluid_solve": (I, [I, I, I, I, P, D, D, D, I64, I, I, P, P, P, P]),
            "orc_ad_init": (I, [I, I, I, I, P, D, P, P]),
            "orc_ad_step": (I, [I, I, I, I, P, D, D, D, D, I, D, P, P, P, P, P]),
            "orc_ad_moment": (I, [I, I, I, I, P, D, D, P, P]),
            "orc_ad_fluxes": (I, [I, I, I, I, P, D, D, D, I, D, P, P, P, P, P]),
            "orc_ad_solve": (I, [I, I, I, I, P, P, D, D, D, D, I, D, D, I64, I, I, P, P, P, P]),
            "orc_splitmix64": (None, [U64, I64, P]),
            "orc_geom_discs": (I, [I, I, I, I, D, I, U64, P, P]),
            "orc_geom_fibres": (I, [I, I, I, I, I, D, U64, P, P]),
            "orc_biofilm_layer": (I, [I, I, I, P]),
            "orc_links": (I, [I, I, I, P, I, P]),
            "orc_percolates": (I, [I, I, I, P]),
            "orc_flow_domain": (I, [I, I, I, P, P]),
            "orc_growth_pick": (I64, [I, I, I, P, P, D]),
            "orc_fluid_run": (I, [I, I, I, I, P, D, D, P, P, I64, P, P, P]),
            "orc_ad_run": (I, [I, I, I, I, P, D, D, D, D, I, D, P, P, I64, P, P]),
            "orc_coupled_run": (I, [I, I, I, P, D, D, D, D, D, D, I, D, I64, I, I, I, P,
                                    P, P, P, P, P, P, P]),
            "orc_stall_rule": (I, [P, P, I, D, I, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _shape(cls_shape):
    """(nx, ny, nz) of a class array given as [ny, nx] or [nz, ny, nx]."""
    if len(cls_shape) == 2:
        return cls_shape[1], cls_shape[0], 1
    return cls_shape[2], cls_shape[1], cls_shape[0]


def fluid_lattice(nz):
    return D3Q19 if nz > 1 else D2Q9


def ad_lattice(nz):
    return D3Q7 if nz > 1 else D2Q5


def lattice_tables(lat):
    q = ct.c_int()
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    cs2 = ct.c_double()
    lib().orc_lattice_tables(lat, ct.byref(q), _p(c), _p(w), _p(opp), ct.byref(cs2))
    n = q.value
    return c[:n].copy(), w[:n].copy(), opp[:n].copy(), cs2.value


def feq(lat, rho, u):
    u3 = np.zeros(3)
    u3[: len(u)] = u
    out = np.zeros(19)
    lib().orc_feq(lat, float(rho), _p(u3), _p(out))
    return out[: lattice_tables(lat)[0].shape[0]]


def geq(lat, C, u):
    u3 = np.zeros(3)
    u3[: len(u)] = u
    out = np.zeros(19)
    lib().orc_geq(lat, float(C), _p(u3), _p(out))
    return out[: lattice_tables(lat)[0].shape[0]]


def _q(lat):
    return {D2Q9: 9, D2Q5: 5, D3Q19: 19, D3Q7: 7}[lat]


def _dim(lat):
    return 3 if lat in (D3Q19, D3Q7) else 2


# ----------------------------------------------------------------- fluid
def fluid_init(cls, lat=None):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = fluid_lattice(nz) if lat is None else lat
    f = np.zeros((_q(lat), cls.size))
    lib().orc_fluid_init(lat, nx, ny, nz, _p(cls), _p(f))
    return f


def fluid_step(cls, f, tau, u_in, periodic=(0, 0, 0), force=(0.0, 0.0, 0.0), lat=None):
    """One step; returns (f_next, U [dim][N], rho [N])."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = fluid_lattice(nz) if lat is None else lat
    f = _f64(f)
    out = np.empty_like(f)
    U = np.empty((_dim(lat), cls.size))
    rho = np.empty(cls.size)
    per = np.asarray(periodic, np.int32)
    fo = _f64(list(force) + [0.0] * (3 - len(force)))
    lib().orc_fluid_step(lat, nx, ny, nz, _p(cls), float(tau), float(u_in), _p(per),
                         _p(fo), _p(f), _p(out), _p(U), _p(rho))
    return out, U, rho


def fluid_run(cls, f, tau, u_in, nsteps, periodic=(0, 0, 0), force=(0.0, 0.0, 0.0), lat=None):
    """nsteps fixed steps from state f (not modified); returns (f, U of the
    last step, rho of the last step)."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = fluid_lattice(nz) if lat is None else lat
    f = _f64(f).copy()
    U = np.zeros((_dim(lat), cls.size))
    rho = np.zeros(cls.size)
    per = np.asarray(periodic, np.int32)
    fo = _f64(list(force) + [0.0] * (3 - len(force)))
    lib().orc_fluid_run(lat, nx, ny, nz, _p(cls), float(tau), float(u_in), _p(per), _p(fo),
                        int(nsteps), _p(f), _p(U), _p(rho))
    return f, U, rho


def fluid_moments(cls, f, force=(0.0, 0.0, 0.0), lat=None):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = fluid_lattice(nz) if lat is None else lat
    U = np.empty((_dim(lat), cls.size))
    rho = np.empty(cls.size)
    fo = _f64(list(force) + [0.0] * (3 - len(force)))
    lib().orc_fluid_moments(lat, nx, ny, nz, _p(cls), _p(fo), _p(_f64(f)), _p(U), _p(rho))
    return U, rho


def fluid_fluxes(cls, f, u_in, lat=None):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = fluid_lattice(nz) if lat is None else lat
    a, b = ct.c_double(), ct.c_double()
    lib().orc_fluid_fluxes(lat, nx, ny, nz, _p(cls), float(u_in), _p(_f64(f)),
                           ct.byref(a), ct.byref(b))
    return a.value, b.value


STALL_CHECKS = 1000


def stall_rule(r, tol, window, umax=None):
    """The solves' stop rule applied to a sequence of check residuals r (and
    the largest |u| at each check): (status, index of the deciding check),
    or ("NOT_CONVERGED", len(r)) when no check stops it."""
    r = _f64(r)
    um = None if umax is None else _f64(umax)
    at = ct.c_int()
    st = lib().orc_stall_rule(_p(r), None if um is None else _p(um), len(r), float(tol),
                              int(window), ct.byref(at))
    return STATUS.get(st, st), at.value


def fluid_solve(cls, tau, u_in, tol, max_iter, check_every=100, f=None, lat=None,
                stall_checks=STALL_CHECKS):
    """Steady solve (cold if f is None).  Returns dict(status, iters,
    residual, f, U)."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = fluid_lattice(nz) if lat is None else lat
    f = fluid_init(cls, lat) if f is None else _f64(f).copy()
    U = np.empty((_dim(lat), cls.size))
    it, res = ct.c_int64(), ct.c_double()
    st = lib().orc_fluid_solve(lat, nx, ny, nz, _p(cls), float(tau), float(u_in), float(tol),
                               int(max_iter), int(check_every), int(stall_checks), _p(f),
                               _p(U), ct.byref(it), ct.byref(res))
    return dict(status=STATUS.get(st, st), iters=it.value, residual=res.value, f=f, U=U)


# -------------------------------------------------------------------- AD
def ad_init(cls, u, c_init, lat=None):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = ad_lattice(nz) if lat is None else lat
    g = np.zeros((_q(lat), cls.size))
    lib().orc_ad_init(lat, nx, ny, nz, _p(cls), float(c_init), _p(_f64(u)), _p(g))
    return g


def ad_step(cls, g, u, D, c_in, k_sink, outlet=0, c_out=0.0, periodic=(0, 0, 0), lat=None,
            k_half=0.0):
    """One step; returns (g_next, C of this step).  k_half > 0 selects the
    Monod sink k C / (C + k_half) in place of k C."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = ad_lattice(nz) if lat is None else lat
    g = _f64(g)
    out = np.empty_like(g)
    C = np.empty(cls.size)
    per = np.asarray(periodic, np.int32)
    lib().orc_ad_step(lat, nx, ny, nz, _p(cls), float(D), float(c_in), float(k_sink),
                      float(k_half), int(outlet), float(c_out), _p(per), _p(_f64(u)), _p(g), _p(out), _p(C))
    return out, C


def ad_run(cls, g, u, D, c_in, k_sink, nsteps, outlet=0, c_out=0.0, periodic=(0, 0, 0), lat=None,
           k_half=0.0):
    """nsteps fixed steps from state g (not modified); returns (g, C of the
    last step)."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = ad_lattice(nz) if lat is None else lat
    g = _f64(g).copy()
    C = np.zeros(cls.size)
    per = np.asarray(periodic, np.int32)
    lib().orc_ad_run(lat, nx, ny, nz, _p(cls), float(D), float(c_in), float(k_sink),
                     float(k_half), int(outlet), float(c_out), _p(per), _p(_f64(u)), int(nsteps), _p(g), _p(C))
    return g, C


def ad_moment(cls, g, k_sink, lat=None, k_half=0.0):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = ad_lattice(nz) if lat is None else lat
    C = np.empty(cls.size)
    lib().orc_ad_moment(lat, nx, ny, nz, _p(cls), float(k_sink), float(k_half), _p(_f64(g)), _p(C))
    return C


def ad_fluxes(cls, g, c_in, k_sink, outlet=0, c_out=0.0, lat=None, k_half=0.0, u=None):
    """Inflow, outflow and consumption per step of a stored substrate state.
    u (the frozen velocity) enters the Dirichlet faces of the second-order
    form; None is u = 0."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = ad_lattice(nz) if lat is None else lat
    a, b, s = ct.c_double(), ct.c_double(), ct.c_double()
    lib().orc_ad_fluxes(lat, nx, ny, nz, _p(cls), float(c_in), float(k_sink), float(k_half), int(outlet),
                        float(c_out), None if u is None else _p(_f64(u)), _p(_f64(g)), ct.byref(a),
                        ct.byref(b), ct.byref(s))
    return a.value, b.value, s.value


def ad_solve(cls, u, D, c_in, k_sink, tol, max_iter, outlet=0, c_out=0.0, check_every=100,
             g=None, lat=None, stall_checks=STALL_CHECKS, k_half=0.0):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    lat = ad_lattice(nz) if lat is None else lat
    u = _f64(u)
    g = ad_init(cls, u, c_in, lat) if g is None else _f64(g).copy()
    C = np.empty(cls.size)
    it, res = ct.c_int64(), ct.c_double()
    st = lib().orc_ad_solve(lat, nx, ny, nz, _p(cls), _p(u), float(D), float(c_in),
                            float(k_sink), float(k_half), int(outlet), float(c_out), float(tol),
                            int(max_iter),
                            int(check_every), int(stall_checks), _p(g), _p(C), ct.byref(it),
                            ct.byref(res))
    return dict(status=STATUS.get(st, st), iters=it.value, residual=res.value, g=g, C=C)


# -------------------------------------------------------------- geometry
def splitmix64(seed, count):
    out = np.zeros(count, np.uint64)
    lib().orc_splitmix64(ct.c_uint64(seed), count, _p(out))
    return out


def geom_discs(nx, ny, r_min, r_max, solid_frac, overlap, seed):
    cls = np.zeros((ny, nx), np.uint8)
    ach = ct.c_double()
    st = lib().orc_geom_discs(nx, ny, r_min, r_max, float(solid_frac), int(overlap),
                              ct.c_uint64(seed), _p(cls), ct.byref(ach))
    return STATUS.get(st, st), cls, ach.value


def geom_fibres(nx, ny, nz, r_min, r_max, solid_frac, seed):
    cls = np.zeros((nz, ny, nx), np.uint8)
    ach = ct.c_double()
    st = lib().orc_geom_fibres(nx, ny, nz, r_min, r_max, float(solid_frac),
                               ct.c_uint64(seed), _p(cls), ct.byref(ach))
    return STATUS.get(st, st), cls, ach.value


def biofilm_layer(cls):
    cls = _u8(cls).copy()
    nx, ny, nz = _shape(cls.shape)
    lib().orc_biofilm_layer(nx, ny, nz, _p(cls))
    return cls


def links(cls, which):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    dt = np.uint8 if which == 1 else (np.uint32 if nz > 1 else np.uint16)
    out = np.zeros(cls.shape, dt)
    lib().orc_links(nx, ny, nz, _p(cls), int(which), _p(out))
    return out


def percolates(cls):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    return bool(lib().orc_percolates(nx, ny, nz, _p(cls)))


def flow_domain(cls):
    """FLUID nodes linked to the outlet column (bool mask, shape of cls): the
    nodes the fluid solver updates; closed pores and inlet-only pockets carry
    no steady flow (reading of Sec. 2.1.1 on the Sec. 3 pore space)."""
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    out = np.zeros(cls.shape, np.uint8)
    lib().orc_flow_domain(nx, ny, nz, _p(cls), _p(out))
    return out.astype(bool)


def growth_pick(cls, C, xi):
    cls = _u8(cls)
    nx, ny, nz = _shape(cls.shape)
    return int(lib().orc_growth_pick(nx, ny, nz, _p(cls), _p(_f64(C)), float(xi)))


def coupled_run(cls, tau, u_in, D, c_in, k_sink, tol, max_iter, xi, check_every=100,
                stall_checks=STALL_CHECKS, k_half=0.0, lat_ad=None):
    cls = _u8(cls).copy()
    nx, ny, nz = _shape(cls.shape)
    xi = _f64(xi)
    M = len(xi)
    picked = np.zeros(M, np.int64)
    J = np.zeros(M + 1)
    itf = np.zeros(M + 1, np.int64)
    ita = np.zeros(M + 1, np.int64)
    acc = ct.c_double()
    U = np.zeros((3 if nz > 1 else 2, cls.size))
    C = np.zeros(cls.size)
    st = lib().orc_coupled_run(nx, ny, nz, _p(cls), float(tau), float(u_in), float(D),
                               float(c_in), float(k_sink), float(k_half),
                               -1 if lat_ad is None else int(lat_ad), float(tol), int(max_iter),
                               int(check_every), int(stall_checks), M, _p(xi), _p(picked), _p(J), ct.byref(acc),
                               _p(itf), _p(ita), _p(U), _p(C))
    return dict(status=STATUS.get(st, st), cls=cls, picked=picked, J=J, J_accum=acc.value,
                iters_fluid=itf, iters_ad=ita, U=U, C=C)

"""Pins of the FP64 oracle to facts other than itself (CPU only).

Each test checks the oracle against something the paper or mathematics fixes:
lattice identities (Sec. 2.1, Eqs. 1-3, 5-8, 11), Table 1's tau_D / D pair,
Poiseuille flow (exact at the magic relaxation time, second order otherwise:
Sec. 2.1.1), exact mass conservation, exact moment recurrences and the
continuum Gaussian for the advection-diffusion LBM (Sec. 2.1.2, Eqs. 12-13),
the exact discrete two-mode solution of the steady 1-D advection-diffusion-
sink problem, flux balances at steady state, uniform flow and uniform
substrate as exact fixed points of the inlet and outlet rules, and an
independent push-form brute force on tiny grids; most of them on the 3-D
lattices (D3Q19, D3Q7) as well as the 2-D ones.  A plausible mistake in the
oracle (a wrong weight, sign, opposite index, equilibrium term, inlet/outlet
rule or sink form) fails at least one of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ lattice
@pytest.mark.parametrize("lat", [O.D2Q9, O.D2Q5, O.D3Q19, O.D3Q7])
def test_lattice_isotropy(lat):
    c, w, opp, cs2 = O.lattice_tables(lat)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs((w[:, None] * c).sum(0)).max() < 1e-16
    second = np.einsum("i,ia,ib->ab", w, c, c)
    dim = 3 if lat in (O.D3Q19, O.D3Q7) else 2
    assert np.allclose(second[:dim, :dim], cs2 * np.eye(dim), atol=1e-15, rtol=0)
    for i in range(len(w)):
        assert (c[opp[i]] == -c[i]).all()
        assert w[opp[i]] == w[i]


def test_d2q9_matches_equations_1_to_8_and_11():
    c, w, opp, cs2 = O.lattice_tables(O.D2Q9)
    # Eqs. 6-8: 4/9 rest, 1/9 axes, 1/36 diagonals (exact rationals)
    exact = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    assert [float(e) for e in exact] == list(w)
    assert sum(exact) == 1
    # Eqs. 1-3: c0 rest, c1/c3 = (+-1,0), c2/c4 = (0,+-1), c5..c8 diagonals
    assert tuple(c[0]) == (0, 0, 0)
    assert {tuple(c[1][:2]), tuple(c[3][:2])} == {(1, 0), (-1, 0)}
    assert {tuple(c[2][:2]), tuple(c[4][:2])} == {(0, 1), (0, -1)}
    assert all(abs(c[i][0]) == 1 and abs(c[i][1]) == 1 for i in range(5, 9))
    # Eq. 11 (south boundary): the unknowns 5, 2, 6 move north and take the
    # values of 7, 4, 8 -> those are their opposites.
    for a, b in [(5, 7), (2, 4), (6, 8)]:
        assert opp[a] == b and c[a][1] == 1
    assert cs2 == 1.0 / 3.0


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_equilibrium_moments(lat):
    c, w, opp, cs2 = O.lattice_tables(lat)
    rng = np.random.default_rng(7)
    dim = 3 if lat == O.D3Q19 else 2
    for _ in range(20):
        rho = 0.8 + 0.4 * rng.random()
        u = np.zeros(3)
        u[:dim] = 0.1 * (rng.random(dim) - 0.5)
        f = O.feq(lat, rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.abs((c * f[:, None]).sum(0) - rho * u).max() < 1e-16
        P = np.einsum("i,ia,ib->ab", f, c, c)
        want = rho * (cs2 * np.eye(3) + np.outer(u, u))
        assert np.abs(P[:dim, :dim] - want[:dim, :dim]).max() < 1e-15


@pytest.mark.parametrize("lat", [O.D2Q5, O.D3Q7])
def test_ad_equilibrium_moments(lat):
    c, w, opp, cs2 = O.lattice_tables(lat)
    u = np.array([0.03, -0.02, 0.01 if lat == O.D3Q7 else 0.0])
    g = O.geq(lat, 0.7, u)
    assert abs(g.sum() - 0.7) < 1e-15
    assert np.abs((c * g[:, None]).sum(0) - 0.7 * u).max() < 1e-16


def test_ad_second_order_equilibrium_moments():
    """D2Q9 substrate equilibrium (Eq. 5 with C for rho): zeroth, first and
    second moments C, C u and C (c_s^2 I + u u)."""
    c, w, opp, cs2 = O.lattice_tables(O.D2Q9)
    u = np.array([0.04, -0.025, 0.0])
    C = 0.7
    g = O.geq(O.D2Q9, C, u)
    assert abs(g.sum() - C) < 1e-15
    assert np.abs((c * g[:, None]).sum(0) - C * u).max() < 1e-16
    Pi = np.einsum("ia,ib,i->ab", c[:, :2].astype(float), c[:, :2].astype(float), g)
    want = C * (cs2 * np.eye(2) + np.outer(u[:2], u[:2]))
    assert np.abs(Pi - want).max() < 1e-15


def test_table1_tau_d_and_diffusivity_consistent():
    """Table 1: tau_D = 0.5036 and D = 0.0012 mm^2/s satisfy
    D = c_s^2 (tau_D - 1/2) dx^2/dt with the oracle's D2Q5 c_s^2 = 1/3,
    dx = 1 mm (60 x 65 lattice on 60 x 65 mm) and dt = 1 s."""
    vals = {}
    with open(os.path.join(HERE, "golden", "table1_lbm.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v, _ = line.split()
            vals[k] = float(v)
    cs2 = O.lattice_tables(O.D2Q5)[3]
    assert abs(cs2 * (vals["tau_D"] - 0.5) - vals["D"]) < 1e-15


# ------------------------------------------------------------------ fluid
def _poiseuille_error(H, tau, g=1e-6, steps=None):
    ny, nx = H + 2, 4
    cls = np.zeros((ny, nx), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    nu = (tau - 0.5) / 3
    steps = steps or int(25 * H * H / nu)
    f, U, _ = O.fluid_run(cls, O.fluid_init(cls), tau, 0.0, steps, periodic=(1, 0, 0),
                          force=(g, 0.0, 0.0))
    y = np.arange(ny)
    exact = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    ux = U[0].reshape(ny, nx)[:, 1]
    return np.abs(ux[1:-1] - exact[1:-1]).max() / exact.max()


@pytest.mark.parametrize("H", [8, 16])
def test_poiseuille_exact_at_magic_tau(H):
    """BGK + half-way bounce-back put the wall exactly half-way when
    (tau - 1/2)^2 = 3/16: the parabola is reproduced to round-off."""
    assert _poiseuille_error(H, (2.0 + math.sqrt(3.0)) / 4.0) < 1e-10


def test_poiseuille_second_order():
    """Sec. 2.1.1 claims second-order accuracy: the error falls ~4x per
    doubling of the channel height."""
    e8, e16 = _poiseuille_error(8, 0.8), _poiseuille_error(16, 0.8)
    assert 3.6 < e8 / e16 < 4.4
    assert e16 < 3e-3


def _poiseuille3d_error(H, tau, axis, g=1e-6):
    """D3Q19 plane Poiseuille flow between two walls normal to y or to z
    (periodic in the other two directions), driven by a body force in x."""
    n = H + 2
    shape, per = ((n, 4, 4), (1, 1, 0)) if axis == "z" else ((4, n, 4), (1, 0, 1))
    cls = np.zeros(shape, np.uint8)
    if axis == "z":
        cls[0] = O.WALL
        cls[-1] = O.WALL
    else:
        cls[:, 0] = O.WALL
        cls[:, -1] = O.WALL
    nu = (tau - 0.5) / 3
    f, U, _ = O.fluid_run(cls, O.fluid_init(cls), tau, 0.0, int(25 * H * H / nu), periodic=per,
                          force=(g, 0.0, 0.0))
    k = np.arange(n)
    exact = g / (2 * nu) * (k - 0.5) * (n - 1.5 - k)
    ux = U[0].reshape(shape)
    prof = ux[:, 1, 1] if axis == "z" else ux[1, :, 1]
    return np.abs(prof[1:-1] - exact[1:-1]).max() / exact.max(), np.abs(U[1:]).max()


@pytest.mark.parametrize("axis", ["y", "z"])
def test_poiseuille_3d_exact_at_magic_tau_and_second_order(axis):
    """The 3-D lattice (D3Q19) with half-way bounce-back on walls normal to
    y and to z: the parabola to round-off at (tau - 1/2)^2 = 3/16, no
    cross-flow, and second order (error ~4x smaller per doubling) at
    tau = 0.8 -- the properties the 2-D pins fix for D2Q9."""
    e, cross = _poiseuille3d_error(8, (2.0 + math.sqrt(3.0)) / 4.0, axis)
    assert e < 1e-10 and cross < 1e-14
    e8, e16 = _poiseuille3d_error(8, 0.8, axis)[0], _poiseuille3d_error(16, 0.8, axis)[0]
    assert 3.6 < e8 / e16 < 4.4
    assert e16 < 3e-3


def test_channel_inlet_outlet_develops_parabola():
    """Production boundaries (velocity inlet, pressure outlet): the
    mid-length momentum profile j = rho u of a long empty channel is the
    parabola carrying the injected mass flux (rho itself rises along the
    channel with the driving pressure), and inflow equals outflow at steady
    state."""
    nx, ny, tau, uin = 200, 18, 0.8, 0.01
    cls = np.zeros((ny, nx), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    r = O.fluid_solve(cls, tau, uin, 1e-8, 100000)
    assert r["status"] == "OK"
    U, rho = O.fluid_moments(cls, r["f"])
    ux = (rho * U[0]).reshape(ny, nx)[1:-1, nx // 2]
    y = np.arange(1, ny - 1)
    shape = (y - 0.5) * (ny - 1.5 - y)
    par = shape * (uin * (ny - 2)) / shape.sum()
    assert np.abs(ux - par).max() / par.max() < 1e-2
    fin, fout = O.fluid_fluxes(cls, r["f"], uin)
    assert fin == pytest.approx(uin * (ny - 2), rel=1e-14)   # exactly u_in per inlet node
    assert abs(fout - fin) / fin < 1e-6   # residual level: tol 1e-8 per step over ~200 columns


@pytest.mark.parametrize("lat,shape,periodic", [(O.D2Q9, (6, 12), (0, 1, 0)),
                                                 (O.D3Q19, (4, 5, 10), (0, 1, 1))])
def test_uniform_plug_flow_is_exact_fixed_point_of_inlet_and_outlet(lat, shape, periodic):
    """Production boundaries on an open duct (periodic across the flow, no
    walls): the uniform equilibrium at rho = 1, u = (u_in, 0, 0) is an exact
    fixed point of the whole step.  BGK leaves an equilibrium unchanged;
    the moving-wall inlet (reading 5) holds because f_i^eq - f_opp^eq is
    twice the odd part 3 w_i c_i.u; the anti-bounce-back outlet at rho_out = 1
    (reading 6) holds because f_i^eq + f_opp^eq is twice the even part
    w_i (1 + 9/2 (c_i.u)^2 - 3/2 u^2).  The equilibrium is built here from
    the textbook weights and Eqs. 5-8, not from the oracle; a dropped u^2
    term or a wrong factor in either boundary moves f by O(w u^2) ~ 1e-4."""
    c = O.lattice_tables(lat)[0]
    wts = {9: {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}, 19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}}[c.shape[0]]
    w = np.array([wts[int(k)] for k in (c ** 2).sum(1)])
    uin = 0.05
    cu = c[:, 0] * uin
    fe = w * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uin ** 2)
    cls = np.zeros(shape, np.uint8)
    f0 = np.repeat(fe[:, None], cls.size, axis=1)
    f, U, rho = O.fluid_run(cls, f0, 0.8, uin, 50, periodic=periodic)
    assert np.abs(f - f0).max() < 1e-14
    assert np.abs(rho - 1.0).max() < 1e-14
    assert np.abs(U[0] - uin).max() < 1e-14 and np.abs(U[1:]).max() < 1e-14


@pytest.mark.parametrize("lat,shape,periodic,outlet", [(O.D2Q5, (6, 12), (0, 1, 0), 0),
                                                        (O.D2Q5, (6, 12), (0, 1, 0), 1),
                                                        (O.D2Q9, (6, 12), (0, 1, 0), 0),
                                                        (O.D3Q7, (4, 5, 10), (0, 1, 1), 0),
                                                        (O.D3Q7, (4, 5, 10), (0, 1, 1), 1)])
def test_uniform_substrate_is_exact_fixed_point_of_inlet_and_outlet(lat, shape, periodic, outlet):
    """Substrate boundaries on an open duct in uniform flow: the uniform
    equilibrium at C = c_in is an exact fixed point of the substrate step.
    The Dirichlet inlet (anti-bounce-back with the equilibrium's even part)
    holds because g_i^eq + g_opp^eq is twice that even part; the
    zero-gradient outlet copies the node's own state; the Dirichlet outlet
    at c_out = c_in holds as the inlet does.  Equilibria from the textbook:
    w_i C (1 + c_i.u / c_s^2) with c_s^2 = 1/3 (D2Q5: 1/3, 1/6) and 1/4 (D3Q7:
    1/4, 1/8), and the second-order Eq. 5 form on D2Q9."""
    c = O.lattice_tables(lat)[0]
    q = c.shape[0]
    uin, c_in = 0.05, 0.8
    cu = c[:, 0] * uin
    if q == 9:
        wts = {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}
        w = np.array([wts[int(k)] for k in (c ** 2).sum(1)])
        ge = w * c_in * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uin ** 2)
    else:
        w0, cs2 = (1 / 3, 1 / 3) if q == 5 else (1 / 4, 1 / 4)
        w = np.where((c ** 2).sum(1) == 0, w0, (1 - w0) / (q - 1))
        ge = w * c_in * (1 + cu / cs2)
    cls = np.zeros(shape, np.uint8)
    dim = 3 if len(shape) == 3 else 2
    U = np.zeros((dim, cls.size))
    U[0] = uin
    g0 = np.repeat(ge[:, None], cls.size, axis=1)
    D = 0.05
    g, C = O.ad_run(cls, g0, U, D, c_in, 0.0, 50, outlet=outlet, c_out=c_in, periodic=periodic, lat=lat)
    assert np.abs(g - g0).max() < 1e-14
    assert np.abs(C - c_in).max() < 1e-14


def _porous(nx, ny, seed, frac=0.3):
    st, cls, _ = O.geom_discs(nx, ny, 2, 4, frac, 0, seed)
    assert st == "OK"
    return cls


def test_mass_conservation_periodic_porous_fluid():
    cls = _porous(64, 32, 11)
    f0 = O.fluid_init(cls)
    f1, _, _ = O.fluid_run(cls, f0, 0.7, 0.0, 1, periodic=(1, 0, 0), force=(2e-6, 0, 0))
    f, _, _ = O.fluid_run(cls, f0, 0.7, 0.0, 3000, periodic=(1, 0, 0), force=(2e-6, 0, 0))
    M0, M1 = f0.sum(), f.sum()
    # round-off only: well under 1e-15 per step, accumulated
    assert abs(f1.sum() - M0) / M0 < 1e-14
    assert abs(M1 - M0) / M0 < 1e-11
    U, _ = O.fluid_moments(cls, f, force=(2e-6, 0, 0))
    assert U[0].max() > 1e-5          # the flow did develop


def test_mass_conservation_3d_periodic():
    st, cls, _ = O.geom_fibres(24, 12, 12, 1, 2, 0.2, 5)
    assert st == "OK"
    f0 = O.fluid_init(cls)
    f, _, _ = O.fluid_run(cls, f0, 0.8, 0.0, 300, periodic=(1, 0, 0), force=(1e-5, 0, 0))
    assert abs(f.sum() - f0.sum()) / f0.sum() < 1e-13


def test_ad_closed_box_sink_removes_exactly_kC():
    """Periodic box with biofilm nodes: each step removes k * sum(C) over
    the biofilm, to round-off."""
    cls = O.biofilm_layer(_porous(48, 24, 3))
    nx, ny = 48, 24
    rng = np.random.default_rng(1)
    u = np.zeros((2, nx * ny))
    u[0] = 0.02 * (cls.ravel() == O.FLUID)
    g = O.ad_init(cls, u, 1.0) * (1.0 + 0.1 * rng.random((5, nx * ny)))
    k = 2e-3
    bf = cls.ravel() == O.BIOFILM
    for _ in range(5):
        g2, C = O.ad_step(cls, g, u, 0.05, 1.0, k, periodic=(1, 0, 0))
        dM = g2.sum() - g.sum()
        assert abs(dM - (-k * C[bf].sum())) < 1e-13 * g.sum()
        g = g2


def test_ad_closed_box_monod_sink_removes_exactly_q():
    """The Monod form of the consumption rate (Eq. 16, mediator factor in
    k): in a periodic box each step removes sum over biofilm nodes of
    k C / (C + K), C the concentration the step collides with."""
    cls = O.biofilm_layer(_porous(48, 24, 3))
    nx, ny = 48, 24
    rng = np.random.default_rng(2)
    u = np.zeros((2, nx * ny))
    u[0] = 0.02 * (cls.ravel() == O.FLUID)
    g = O.ad_init(cls, u, 1.0) * (1.0 + 0.1 * rng.random((5, nx * ny)))
    k, K = 3e-3, 0.4
    bf = cls.ravel() == O.BIOFILM
    for _ in range(5):
        g2, C = O.ad_step(cls, g, u, 0.05, 1.0, k, periodic=(1, 0, 0), k_half=K)
        dM = g2.sum() - g.sum()
        q = k * C[bf] / (C[bf] + K)
        assert abs(dM - (-q.sum())) < 1e-13 * g.sum()
        g = g2


@pytest.mark.parametrize("K", [0.0, 0.4])
def test_ad_closed_box_sink_removes_exactly_q_3d(K):
    """D3Q7 on a periodic fibre box with its biofilm layer: each step
    removes the sum over biofilm nodes of k C (K = 0) or k C / (C + K)
    (the Monod form), C the concentration the step collides with."""
    st, cls, _ = O.geom_fibres(24, 12, 12, 1, 2, 0.2, 8)
    assert st == "OK"
    cls = O.biofilm_layer(cls)
    bf = cls.ravel() == O.BIOFILM
    assert bf.any()
    rng = np.random.default_rng(9)
    u = np.zeros((3, cls.size))
    u[0] = 0.02 * (cls.ravel() == O.FLUID)
    g = O.ad_init(cls, u, 1.0) * (1.0 + 0.1 * rng.random((7, cls.size)))
    k = 3e-3
    for _ in range(5):
        g2, C = O.ad_step(cls, g, u, 0.05, 1.0, k, periodic=(1, 0, 0), k_half=K)
        q = k * C[bf] if K == 0.0 else k * C[bf] / (C[bf] + K)
        assert abs((g2.sum() - g.sum()) + q.sum()) < 1e-13 * g.sum()
        g = g2


def test_monod_uniform_biofilm_decay_recurrence():
    """A closed, uniform biofilm-filled box at rest: C follows
    C <- C - k C / (C + K) exactly, and each stored state gives back the
    concentration of the step that produced it (the sink is inverted)."""
    nx, ny = 12, 8
    cls = np.full((ny, nx), O.BIOFILM, np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    u = np.zeros((2, nx * ny))
    g = O.ad_init(cls, u, 2.0)
    k, K = 0.02, 0.7
    act = cls.ravel() == O.BIOFILM
    c = 2.0
    for _ in range(60):
        g, C = O.ad_step(cls, g, u, 0.1, 2.0, k, periodic=(1, 0, 0), k_half=K)
        assert np.abs(C[act] - c).max() < 1e-13 * c
        Cm = O.ad_moment(cls, g, k, k_half=K)
        assert np.abs(Cm[act] - c).max() < 1e-13 * c
        c = c - k * c / (c + K)
    assert c < 1.2    # the decay did happen


def test_monod_tends_to_first_order():
    """K -> infinity with k / K fixed: the Monod sink tends to the first-
    order sink with rate k / K, the gap shrinking like C / K."""
    cls = O.biofilm_layer(_porous(40, 20, 5))
    nx, ny = 40, 20
    u = np.zeros((2, nx * ny))
    u[0] = 0.01 * (cls.ravel() == O.FLUID)
    r = 2e-3
    g1, _ = O.ad_run(cls, O.ad_init(cls, u, 1.0), u, 0.05, 1.0, r, 300)
    gaps = []
    for K in (10.0, 100.0, 1000.0):
        gm, _ = O.ad_run(cls, O.ad_init(cls, u, 1.0), u, 0.05, 1.0, r * K, 300, k_half=K)
        gaps.append(np.abs(gm - g1).max())
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[1] / gaps[0] < 0.15 and gaps[2] / gaps[1] < 0.15


def _gauss_setup(nx, ny, tau, ux, s0, x0, y0):
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    C0 = np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * s0 ** 2)).ravel()
    c, w, opp, cs2 = O.lattice_tables(O.D2Q5)
    g = np.array([w[i] * C0 * (1 + c[i, 0] * ux / cs2) for i in range(5)])
    u = np.zeros((2, nx * ny))
    u[0] = ux
    return X.ravel(), Y.ravel(), C0, g, u, cs2


def test_gaussian_pulse_exact_moment_recurrences():
    """From the linear moment recurrences of the D2Q5 BGK map (started at
    equilibrium, uniform u): the centroid moves exactly u per step and the
    central second moment V obeys
        V(t+1) - V(t) = 2 s_t + (c_s^2 - u^2) M,
        s_t = (1-w)(c_s^2 - u^2) M / w * (1 - (1-w)^t),  w = 1/tau_D."""
    nx, ny, tau, ux, T = 300, 64, 0.8, 0.05, 300
    X, Y, C0, g, u, cs2 = _gauss_setup(nx, ny, tau, ux, 6.0, 80.0, 32.0)
    D = (tau - 0.5) * cs2
    _, C = O.ad_run(np.zeros((ny, nx), np.uint8), g, u, D, 1.0, 0.0, T, periodic=(1, 1, 0))
    M0, M = C0.sum(), C.sum()
    assert abs(M - M0) / M0 < 1e-13
    X0 = (X * C0).sum() / M0
    assert abs((X * C).sum() / M - X0 - ux * T) < 1e-10
    om = 1.0 / tau
    V0 = (X * X * C0).sum() - (X * C0).sum() ** 2 / M0
    pred = V0 + sum(2 * (1 - om) * (cs2 - ux ** 2) * M0 / om * (1 - (1 - om) ** t)
                    + (cs2 - ux ** 2) * M0 for t in range(T))
    V = (X * X * C).sum() - (X * C).sum() ** 2 / M
    assert abs(V - pred) / pred < 1e-11


def test_gaussian_pulse_d3q7_exact_moment_recurrences():
    """The same recurrences on the 3-D substrate lattice (D3Q7, linear
    equilibrium, textbook weights 1/4 and 1/8, c_s^2 = 1/4): along the flow
    with c_s^2 - u^2, across it (u_z = 0) with c_s^2; the centroid moves
    exactly u per step along x and stays put along z."""
    nx, ny, nz, tau, ux, T = 160, 4, 96, 0.8, 0.05, 200
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X, Z = X.ravel().astype(float), Z.ravel().astype(float)
    # centred across the periodic z extent, far (> 7 widths) from its wrap
    C0 = np.exp(-((X - 50.0) ** 2 + (Z - 47.5) ** 2) / (2 * 4.0 ** 2))
    c = O.lattice_tables(O.D3Q7)[0]
    cs2 = 0.25
    w = np.where((c ** 2).sum(1) == 0, 0.25, 0.125)
    g = np.array([w[i] * C0 * (1 + c[i, 0] * ux / cs2) for i in range(7)])
    u = np.zeros((3, X.size))
    u[0] = ux
    D = (tau - 0.5) * cs2
    _, C = O.ad_run(np.zeros((nz, ny, nx), np.uint8), g, u, D, 1.0, 0.0, T, periodic=(1, 1, 1))
    M0, M = C0.sum(), C.sum()
    assert abs(M - M0) / M0 < 1e-13
    assert abs((X * C).sum() / M - (X * C0).sum() / M0 - ux * T) < 1e-10
    assert abs((Z * C).sum() / M - (Z * C0).sum() / M0) < 1e-10
    om = 1.0 / tau
    for A, a2 in ((X, cs2 - ux ** 2), (Z, cs2)):
        V0 = (A * A * C0).sum() - (A * C0).sum() ** 2 / M0
        pred = V0 + sum(2 * (1 - om) * a2 * M0 / om * (1 - (1 - om) ** t) + a2 * M0 for t in range(T))
        V = (A * A * C).sum() - (A * C).sum() ** 2 / M
        assert abs(V - pred) / pred < 1e-11


def test_gaussian_pulse_second_order_exact_recurrences():
    """D2Q9 substrate with the Eq. 5 equilibrium, uniform u, started at
    equilibrium.  Totals over the box obey a closed linear map: the
    centroid moves exactly u per step, and with d = Q - u M1 (Q = sum x
    c_x g) the central second moment V obeys
        V(t+1) - V(t) = 2 (1-w) d_t + P_eq - M u^2,
        d_(t+1) = (1-w) d_t + P_eq - M u^2,  d_0 = 0,
    where P_eq = sum c_x^2 g_eq = M (c_s^2 + u^2) for this equilibrium
    (M c_s^2 for the linear form).  So the variance grows by exactly
    2 M D per step in the long run: no -u^2 numerical diffusion."""
    # a box large enough that the periodic images stay below round-off
    nx, ny, tau, ux, T = 300, 160, 0.8, 0.05, 300
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    X, Y = X.ravel(), Y.ravel()
    C0 = np.exp(-((X - 80.0) ** 2 + (Y - 80.0) ** 2) / (2 * 6.0 ** 2))
    c, w, opp, cs2 = O.lattice_tables(O.D2Q9)
    cu = c[:, 0] * ux
    g = np.array([w[i] * C0 * (1 + 3 * cu[i] + 4.5 * cu[i] ** 2 - 1.5 * ux ** 2) for i in range(9)])
    u = np.zeros((2, nx * ny))
    u[0] = ux
    D = (tau - 0.5) * cs2
    _, C = O.ad_run(np.zeros((ny, nx), np.uint8), g, u, D, 1.0, 0.0, T, periodic=(1, 1, 0),
                    lat=O.D2Q9)
    M0, M = C0.sum(), C.sum()
    assert abs(M - M0) / M0 < 1e-13
    X0 = (X * C0).sum() / M0
    assert abs((X * C).sum() / M - X0 - ux * T) < 1e-10
    om = 1.0 / tau
    V = (X * X * C0).sum() - (X * C0).sum() ** 2 / M0
    d = 0.0
    for _ in range(T):
        V += 2 * (1 - om) * d + M0 * cs2
        d = (1 - om) * d + M0 * cs2
    Vg = (X * X * C).sum() - (X * C).sum() ** 2 / M
    assert abs(Vg - V) / V < 1e-11
    # across the flow (u_y = 0) the same recurrence holds with u = 0
    Vy = (Y * Y * C0).sum() - (Y * C0).sum() ** 2 / M0
    d = 0.0
    for _ in range(T):
        Vy += 2 * (1 - om) * d + M0 * cs2
        d = (1 - om) * d + M0 * cs2
    Vyg = (Y * Y * C).sum() - (Y * C).sum() ** 2 / M
    assert abs(Vyg - Vy) / Vy < 1e-11


def test_gaussian_pulse_continuum():
    """Continuum limit: Gaussian with variance s0^2 + 2 D_eff t, where the
    linear equilibrium gives D_eff = (tau-1/2)(c_s^2 - u^2) along the flow."""
    nx, ny, tau, ux, T, s0 = 240, 96, 0.8, 0.05, 300, 8.0
    X, Y, C0, g, u, cs2 = _gauss_setup(nx, ny, tau, ux, s0, 80.0, 48.0)
    _, C = O.ad_run(np.zeros((ny, nx), np.uint8), g, u, (tau - 0.5) * cs2, 1.0, 0.0, T,
                    periodic=(1, 1, 0))
    sx2 = s0 ** 2 + 2 * (tau - 0.5) * (cs2 - ux ** 2) * T
    sy2 = s0 ** 2 + 2 * (tau - 0.5) * cs2 * T
    ex = C0.sum() / (2 * np.pi * math.sqrt(sx2 * sy2)) * np.exp(
        -(X - 80.0 - ux * T) ** 2 / (2 * sx2) - (Y - 48.0) ** 2 / (2 * sy2))
    assert np.linalg.norm(C - ex) / np.linalg.norm(ex) < 2e-3


def _ad_channel(N, u, k):
    ny = 3
    cls = np.zeros((ny, N), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    if k > 0:
        cls[1] = O.BIOFILM
    uu = np.zeros((2, ny * N))
    uu[0] = u
    return cls, uu


def _two_mode(N, tau, u, k, outlet, c_in, c_out, w=1.0 / 6.0, cs2=1.0 / 3.0):
    """Exact steady solution of the D2Q5 map on a y-uniform channel: in the
    bulk every population is a combination of r^x modes, r a root of
    (b + G a) r^2 - (a (A + b) + G (1 + a^2)) r + (A + G a) = 0 with
    a = 1 - 1/tau, A = w(1+3u)/tau - w k, b = w(1-3u)/tau - w k,
    G = 1/3 + (2/3) k tau, w = 1/6; the inlet and outlet link rules fix the
    two amplitudes.  The rest and transverse populations (weight 1 - 2w
    together; the transverse ones bounce back off the channel walls) hold
    (1 - 2w) C (1 - k tau) at steady state, so G = 1 - (1 - 2w)(1 - k tau)
    in general, and 3u is u / c_s^2: with w = 1/8, c_s^2 = 1/4 the same
    solution holds for D3Q7 on a y- and z-uniform duct."""
    om = 1.0 / tau
    a = 1 - om
    A = om * w * (1 + u / cs2) - w * k
    B = om * w * (1 - u / cs2) - w * k
    G = 1.0 - (1.0 - 2.0 * w) * (1.0 - k / om)
    roots = np.roots([B + G * a, -(a * (A + B) + G * (1 + a * a)), A + G * a])
    a1 = lambda r: A * r / (r - a)      # post-collision +x amplitude
    a3 = lambda r: B / (1 - a * r)      # post-collision -x amplitude
    M = np.zeros((2, 2))
    rhs = np.array([2 * w * c_in, 0.0 if outlet == 0 else 2 * w * c_out])
    for m, r in enumerate(roots):
        M[0, m] = a1(r) / r + a3(r)
        M[1, m] = (a3(r) * r ** N - a3(r) * r ** (N - 1)) if outlet == 0 else \
                  (a3(r) * r ** N + a1(r) * r ** (N - 1))
    amp = np.linalg.solve(M, rhs)
    x = np.arange(N)
    return sum(amp[m] * roots[m] ** x for m in range(2))


@pytest.mark.parametrize("N,tau,u,k,outlet,c_out", [
    (64, 0.7, 0.01, 1e-3, 0, 0.0),
    (50, 0.6, 0.02, 5e-3, 0, 0.0),
    (40, 1.0, 0.03, 1e-2, 0, 0.0),
    (64, 0.7, 0.01, 1e-3, 1, 0.3),
    (64, 0.7, 0.01, 0.0, 1, 0.3),
])
def test_ad_1d_exact_discrete_solution(N, tau, u, k, outlet, c_out):
    cls, uu = _ad_channel(N, u, k)
    D = (tau - 0.5) / 3
    g = O.ad_init(cls, uu, 1.0)
    _, C = O.ad_run(cls, g, uu, D, 1.0, k, 200000, outlet, c_out)
    C = C.reshape(3, N)[1]
    assert np.abs(C - _two_mode(N, tau, u, k, outlet, 1.0, c_out)).max() < 1e-12


@pytest.mark.parametrize("N,tau,u,k,outlet,c_out", [
    (48, 0.7, 0.01, 1e-3, 0, 0.0),
    (40, 1.0, 0.03, 1e-2, 0, 0.0),
    (48, 0.7, 0.01, 1e-3, 1, 0.3),
])
def test_ad_1d_exact_discrete_solution_d3q7(N, tau, u, k, outlet, c_out):
    """D3Q7 on a 3 x 3 duct (walls around one line of nodes, biofilm on it
    when k > 0): the two-mode solution with the D3Q7 weights."""
    cls = np.full((3, 3, N), O.WALL, np.uint8)
    cls[1, 1] = O.BIOFILM if k > 0 else O.FLUID
    uu = np.zeros((3, cls.size))
    uu[0] = u
    D = (tau - 0.5) / 4
    g = O.ad_init(cls, uu, 1.0)
    _, C = O.ad_run(cls, g, uu, D, 1.0, k, 200000, outlet, c_out)
    C = C.reshape(3, 3, N)[1, 1]
    assert np.abs(C - _two_mode(N, tau, u, k, outlet, 1.0, c_out, w=1.0 / 8.0, cs2=0.25)).max() < 1e-12


def test_ad_no_sink_zero_gradient_is_uniform():
    cls, uu = _ad_channel(64, 0.02, 0.0)
    r = O.ad_solve(cls, uu, 0.1, 1.0, 0.0, 1e-14, 5000)
    C = r["C"].reshape(3, 64)[1]
    assert np.abs(C - 1.0).max() < 1e-14


def test_ad_1d_continuum_second_order():
    """Dirichlet-Dirichlet, no sink: C = c_in + (c_out - c_in)
    (e^{u xi/D} - 1)/(e^{u L/D} - 1), xi = x + 1/2, L = N; error O(dx^2)."""
    errs = []
    for N in (32, 64, 128):
        tau = 0.8
        D = (tau - 0.5) / 3
        u = 0.1 * 32 / N
        cls, uu = _ad_channel(N, u, 0.0)
        r = O.ad_solve(cls, uu, D, 1.0, 0.0, 1e-13, 2_000_000, outlet=1, c_out=0.0)
        assert r["status"] == "OK"
        C = r["C"].reshape(3, N)[1]
        xi = np.arange(N) + 0.5
        ex = 1.0 - (np.exp(u * xi / D) - 1) / (np.exp(u * N / D) - 1)
        errs.append(np.abs(C - ex).max())
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 3.0
    assert errs[2] < 1e-2


def test_ad_steady_flux_balance_porous():
    """At steady state inflow - outflow = substrate consumed by the sink."""
    cls = O.biofilm_layer(_porous(64, 24, 5, 0.25))
    assert O.percolates(cls)
    fl = O.fluid_solve(cls, 0.8, 0.02, 1e-9, 60000)
    assert fl["status"] == "OK"
    ad = O.ad_solve(cls, fl["U"], 0.1, 1.0, 5e-3, 1e-12, 200000)
    assert ad["status"] == "OK"
    fin, fout, sink = O.ad_fluxes(cls, ad["g"], 1.0, 5e-3)
    assert sink > 0
    assert abs((fin - fout) - sink) / sink < 1e-6
    fi, fo = O.fluid_fluxes(cls, fl["f"], 0.02)
    assert abs(fi - fo) / fi < 1e-6


def test_steady_balances_3d_fibrous():
    """3-D (D3Q19 + D3Q7) on a seeded fibre electrode with its biofilm
    layer: each inlet node takes in exactly u_in per step, fluid inflow
    equals outflow at steady state, and substrate inflow - outflow equals
    what the biofilm consumes."""
    st, cls, _ = O.geom_fibres(32, 14, 14, 1, 2, 0.2, 3)
    assert st == "OK"
    cls = O.biofilm_layer(cls)
    assert O.percolates(cls)
    fl = O.fluid_solve(cls, 0.8, 0.02, 1e-9, 100000)
    assert fl["status"] == "OK"
    fi, fo = O.fluid_fluxes(cls, fl["f"], 0.02)
    assert fi == pytest.approx(0.02 * 12 * 12, rel=1e-14)
    assert abs(fi - fo) / fi < 1e-6
    ad = O.ad_solve(cls, fl["U"], 0.1, 1.0, 5e-3, 1e-12, 200000)
    assert ad["status"] == "OK"
    fin, fout, sink = O.ad_fluxes(cls, ad["g"], 1.0, 5e-3)
    assert sink > 0
    assert abs((fin - fout) - sink) / sink < 1e-6


# ---------------------------------------------------------- stop semantics
def test_blocked_medium_has_no_flow():
    """A medium that does not percolate carries no steady flow: the part
    reached from the inlet alone would take in u_in per inlet link forever,
    so it is left out of the flow domain, and the part open to the outlet
    rests at rho_out = 1 (the library rejects such masks up front)."""
    cls = O.biofilm_layer(_porous(64, 24, 4, 0.25))
    assert not O.percolates(cls)
    dom = O.flow_domain(cls).ravel()
    assert not dom[::64].any()          # no inlet node is in the domain
    r = O.fluid_solve(cls, 0.8, 0.02, 1e-6, 5000)
    assert r["status"] == "OK" and r["iters"] == 100
    U, rho = O.fluid_moments(cls, r["f"])
    # round-off only: sum w_i is 1 to an ulp, and the outlet rule meets
    # that ulp asymmetrically
    assert np.abs(U).max() < 1e-14
    assert np.abs(rho[dom] - 1.0).max() < 1e-14 and np.all(rho[~dom] == 0.0)
    fin, fout = O.fluid_fluxes(cls, r["f"], 0.02)
    assert fin == 0.0 and abs(fout) < 1e-13


def test_closed_pores_do_not_touch_the_flow():
    """Closed pores exchange nothing with the flow: the domain's populations
    equal, bit for bit, those of the same medium with its pores filled
    solid, and the pores hold no populations, u = 0 and rho = 0."""
    cls = O.biofilm_layer(_porous(64, 32, 8, 0.3))
    dom = O.flow_domain(cls)
    pores = (cls == O.FLUID) & ~dom
    assert pores.sum() > 0 and O.percolates(cls)
    filled = cls.copy()
    filled[pores] = O.SOLID
    fa, Ua, ra = O.fluid_run(cls, O.fluid_init(cls), 0.8, 0.02, 400)
    fb, Ub, rb = O.fluid_run(filled, O.fluid_init(filled), 0.8, 0.02, 400)
    assert np.array_equal(fa, fb) and np.array_equal(Ua, Ub) and np.array_equal(ra, rb)
    flat = pores.ravel()
    assert np.all(fa[:, flat] == 0.0) and np.all(Ua[:, flat] == 0.0) and np.all(ra[flat] == 0.0)


def test_solve_status_codes():
    cls = O.biofilm_layer(_porous(48, 20, 5, 0.2))
    assert O.percolates(cls)
    assert O.fluid_solve(cls, 0.8, 0.01, 1e-6, 1)["status"] == "NOT_CONVERGED"
    r = O.fluid_solve(cls, 0.8, 0.01, 1e-6, 1)
    assert r["iters"] == 1
    r = O.fluid_solve(cls, 0.8, 0.01, 1e-3, 100000)
    assert r["status"] == "OK" and r["iters"] % 100 == 0 and r["residual"] <= 1e-3
    # unstable: tau -> 1/2 with a strong inflow blows up
    assert O.fluid_solve(cls, 0.5001, 0.09, 1e-6, 20000)["status"] == "EDIVERGED"
    # a floor above tol: round-off plateau -> STALLED
    cls2, uu = _ad_channel(16, 0.02, 1e-2)
    r = O.ad_solve(cls2, uu, 0.1, 1.0, 1e-2, 1e-30, 10_000_000, check_every=10, stall_checks=20)
    assert r["status"] in ("STALLED", "OK")
    if r["status"] == "OK":
        assert r["residual"] == 0.0


# --------------------------------------------------------------- brute force
def _push_fluid(cls, f, tau, u_in, c, w, opp):
    """Independent push form of one fluid step on a tiny grid: every stored
    post-collision population is sent along its velocity; one that would
    enter a blocked node returns reversed; one leaving through x < 0 returns
    reversed with the moving-wall term; one leaving through x >= nx returns
    as twice the even part of the equilibrium at rho_out = 1 (with the
    velocity u* of the node's stored state) minus itself.  Then collide with
    Eq. 5."""
    ny, nx = cls.shape
    q = len(w)
    N = nx * ny
    arr = np.full((q, N), np.nan)
    for y in range(ny):
        for x in range(nx):
            n = x + nx * y
            if cls[y, x] != O.FLUID:
                continue
            for i in range(q):
                p = f[i, n]
                tx, ty = x + c[i, 0], y + c[i, 1]
                j = opp[i]
                if tx < 0:
                    arr[j, n] = p + 6 * w[j] * c[j, 0] * u_in
                elif tx >= nx:
                    rs = f[:, n].sum()
                    usx = sum(c[k, 0] * f[k, n] for k in range(q)) / rs
                    usy = sum(c[k, 1] * f[k, n] for k in range(q)) / rs
                    cu = c[j, 0] * usx + c[j, 1] * usy
                    arr[j, n] = -p + 2 * w[j] * 1.0 * (1 + 4.5 * cu * cu - 1.5 * (usx ** 2 + usy ** 2))
                elif ty < 0 or ty >= ny or cls[ty, tx] != O.FLUID:
                    arr[j, n] = p
                else:
                    arr[i, tx + nx * ty] = p
    out = np.zeros((q, N))
    for n in range(N):
        if cls.ravel()[n] != O.FLUID:
            continue
        fi = arr[:, n]
        assert not np.isnan(fi).any()
        rho = sum(fi)
        ux = sum(c[i, 0] * fi[i] for i in range(q)) / rho
        uy = sum(c[i, 1] * fi[i] for i in range(q)) / rho
        for i in range(q):
            cu = c[i, 0] * ux + c[i, 1] * uy
            fe = w[i] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
            out[i, n] = fi[i] - (fi[i] - fe) / tau
    return out


def _push_ad(cls, g, u, tau_d, c_in, k, c, w, opp):
    ny, nx = cls.shape
    q = len(w)
    N = nx * ny
    arr = np.full((q, N), np.nan)
    blocked = lambda t: t in (O.SOLID, O.WALL)
    for y in range(ny):
        for x in range(nx):
            n = x + nx * y
            if blocked(cls[y, x]):
                continue
            for i in range(q):
                p = g[i, n]
                tx, ty = x + c[i, 0], y + c[i, 1]
                j = opp[i]
                if tx < 0:
                    arr[j, n] = -p + 2 * w[j] * c_in
                elif tx >= nx:
                    arr[j, n] = g[j, n]          # ghost column copies the node
                elif ty < 0 or ty >= ny or blocked(cls[ty, tx]):
                    arr[j, n] = p
                else:
                    arr[i, tx + nx * ty] = p
    out = np.zeros((q, N))
    for n in range(N):
        if blocked(cls.ravel()[n]):
            continue
        gi = arr[:, n]
        assert not np.isnan(gi).any()
        C = sum(gi)
        kk = k if cls.ravel()[n] == O.BIOFILM else 0.0
        for i in range(q):
            cu = c[i, 0] * u[0, n] + c[i, 1] * u[1, n]
            ge = w[i] * C * (1 + 3 * cu)
            out[i, n] = gi[i] - (gi[i] - ge) / tau_d - w[i] * kk * C
    return out


def _push_ad9(cls, g, u, tau_d, c_in, k, K, outlet, c_out):
    """Push form of one D2Q9 substrate step with the Eq. 5 equilibrium:
    every stored population is sent along c_i; one that would enter a solid
    comes back reversed; one leaving through x < 0 is replaced, in the node
    it left, by -itself + 2 w_i c_in (1 + 9/2 (c.u)^2 - 3/2 u^2) of the
    reversed direction (u the node's velocity); one leaving through x >= nx
    by the node's own value (zero gradient) or the same Dirichlet form with
    c_out.  Then collide, with the Monod sink k C / (C + K) on biofilm."""
    ny, nx = cls.shape
    c, w, opp, cs2 = O.lattice_tables(O.D2Q9)
    N = nx * ny
    arr = np.full((9, N), np.nan)
    blocked = lambda t: t in (O.SOLID, O.WALL)
    for y in range(ny):
        for x in range(nx):
            n = x + nx * y
            if blocked(cls[y, x]):
                continue
            ux, uy = u[0, n], u[1, n]
            for i in range(9):
                p = g[i, n]
                tx, ty = x + c[i, 0], y + c[i, 1]
                j = opp[i]
                cuj = c[j, 0] * ux + c[j, 1] * uy
                even = w[j] * (1 + 4.5 * cuj * cuj - 1.5 * (ux * ux + uy * uy))
                if tx < 0:
                    arr[j, n] = -p + 2 * even * c_in
                elif tx >= nx:
                    arr[j, n] = -p + 2 * even * c_out if outlet == 1 else g[j, n]
                elif ty < 0 or ty >= ny or blocked(cls[ty, tx]):
                    arr[j, n] = p
                else:
                    arr[i, tx + nx * ty] = p
    out = np.zeros((9, N))
    for n in range(N):
        if blocked(cls.ravel()[n]):
            continue
        gi = arr[:, n]
        assert not np.isnan(gi).any()
        C = sum(gi)
        q = k * C / (C + K) if cls.ravel()[n] == O.BIOFILM else 0.0
        ux, uy = u[0, n], u[1, n]
        for i in range(9):
            cu = c[i, 0] * ux + c[i, 1] * uy
            ge = w[i] * C * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
            out[i, n] = gi[i] - (gi[i] - ge) / tau_d - w[i] * q
    return out


@pytest.mark.parametrize("outlet", [0, 1])
def test_bruteforce_push_ad_d2q9(outlet):
    cls = _tiny_mask()
    rng = np.random.default_rng(7 + outlet)
    u = 0.05 * (rng.random((2, cls.size)) - 0.5)
    act = ~np.isin(cls.ravel(), [O.SOLID, O.WALL])
    g = rng.random((9, cls.size)) * act
    D = 0.08
    tau_d = 0.5 + D * 3
    for _ in range(4):
        want = _push_ad9(cls, g, u, tau_d, 0.9, 0.01, 0.3, outlet, 0.2)
        got, _ = O.ad_step(cls, g, u, D, 0.9, 0.01, outlet=outlet, c_out=0.2, lat=O.D2Q9, k_half=0.3)
        assert np.abs(got - want).max() < 1e-15
        g = got


def _tiny_mask():
    cls = np.zeros((5, 6), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    cls[2, 3] = O.SOLID
    cls[1, 3] = O.BIOFILM
    return cls


def test_bruteforce_push_fluid():
    cls = _tiny_mask()
    c, w, opp, _ = O.lattice_tables(O.D2Q9)
    rng = np.random.default_rng(3)
    f = O.fluid_init(cls) * (1 + 0.2 * rng.random((9, cls.size))) * (cls.ravel() == 0)
    for _ in range(4):
        want = _push_fluid(cls, f, 0.73, 0.04, c, w, opp)
        got, _, _ = O.fluid_step(cls, f, 0.73, 0.04)
        assert np.abs(got - want).max() < 1e-15
        f = got


def test_bruteforce_push_ad():
    cls = _tiny_mask()
    c, w, opp, _ = O.lattice_tables(O.D2Q5)
    rng = np.random.default_rng(4)
    u = 0.05 * (rng.random((2, cls.size)) - 0.5)
    act = ~np.isin(cls.ravel(), [O.SOLID, O.WALL])
    g = rng.random((5, cls.size)) * act
    D = 0.08
    tau_d = 0.5 + D * 3
    for _ in range(4):
        want = _push_ad(cls, g, u, tau_d, 0.9, 0.01, c, w, opp)
        got, _ = O.ad_step(cls, g, u, D, 0.9, 0.01)
        assert np.abs(got - want).max() < 1e-15
        g = got


def _tiny_mask3d():
    cls = np.zeros((5, 5, 6), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    cls[:, 0] = O.WALL
    cls[:, -1] = O.WALL
    cls[2, 2, 3] = O.SOLID
    cls[1, 2, 2] = O.BIOFILM
    return cls


def _push3(cls, f, c, send):
    """Push every stored population of the active nodes along its velocity;
    send(n, i, p, target) returns (direction, node) for pushes that leave
    through x or hit a blocked node, else None for a plain move."""
    nz, ny, nx = cls.shape
    q = c.shape[0]
    arr = np.full((q, cls.size), np.nan)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                n = x + nx * (y + ny * z)
                for i in range(q):
                    t = (x + c[i, 0], y + c[i, 1], z + c[i, 2])
                    r = send(n, i, f[i, n], t)
                    if r is None:
                        continue
                    if r is True:
                        arr[i, t[0] + nx * (t[1] + ny * t[2])] = f[i, n]
                    else:
                        arr[r[0], n] = r[1]
    return arr


def test_bruteforce_push_fluid_d3q19():
    """One D3Q19 fluid step in push form on a 6 x 5 x 5 duct with a solid
    and a biofilm node, against the oracle's pull form: moving-wall inlet,
    anti-bounce-back outlet at rho_out = 1 with the node's own velocity,
    bounce-back on blocked nodes, BGK with the textbook D3Q19 equilibrium
    (weights 1/3, 1/18, 1/36)."""
    cls = _tiny_mask3d()
    nz, ny, nx = cls.shape
    c, _, opp, _ = O.lattice_tables(O.D3Q19)
    w = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int(k)] for k in (c ** 2).sum(1)])
    fl = cls.ravel() == O.FLUID
    rng = np.random.default_rng(6)
    f = np.outer(w, np.ones(cls.size)) * (1 + 0.2 * rng.random((19, cls.size))) * fl
    tau, u_in = 0.71, 0.03
    for _ in range(3):
        def send(n, i, p, t):
            if not fl[n]:
                return None
            j = opp[i]
            if t[0] < 0:
                return (j, p + 6 * w[j] * c[j, 0] * u_in)
            if t[0] >= nx:
                us = c.T @ f[:, n] / f[:, n].sum()
                cu = c[j] @ us
                return (j, -p + 2 * w[j] * (1 + 4.5 * cu * cu - 1.5 * us @ us))
            if cls[t[2], t[1], t[0]] != O.FLUID:
                return (j, p)
            return True
        arr = _push3(cls, f, c, send)
        want = np.zeros_like(f)
        for n in np.flatnonzero(fl):
            fi = arr[:, n]
            assert not np.isnan(fi).any()
            rho = fi.sum()
            u = c.T @ fi / rho
            cu = c @ u
            want[:, n] = fi - (fi - w * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * u @ u)) / tau
        got, _, _ = O.fluid_step(cls, f, tau, u_in)
        assert np.abs(got - want).max() < 1e-15
        f = got


def test_bruteforce_push_ad_d3q7():
    """One D3Q7 substrate step in push form on the same duct: anti-bounce-
    back Dirichlet inlet, zero-gradient outlet, zero-flux solids and walls,
    biofilm active with the first-order sink, linear equilibrium with the
    textbook weights 1/4 and 1/8 (c_s^2 = 1/4)."""
    cls = _tiny_mask3d()
    nz, ny, nx = cls.shape
    c, _, opp, _ = O.lattice_tables(O.D3Q7)
    w = np.where((c ** 2).sum(1) == 0, 0.25, 0.125)
    act = ~np.isin(cls.ravel(), [O.SOLID, O.WALL])
    rng = np.random.default_rng(7)
    u = 0.05 * (rng.random((3, cls.size)) - 0.5)
    g = rng.random((7, cls.size)) * act
    D, c_in, k = 0.06, 0.9, 0.01
    tau_d = 0.5 + D / 0.25
    for _ in range(3):
        def send(n, i, p, t):
            if not act[n]:
                return None
            j = opp[i]
            if t[0] < 0:
                return (j, -p + 2 * w[j] * c_in)
            if t[0] >= nx:
                return (j, g[j, n])
            if cls[t[2], t[1], t[0]] in (O.SOLID, O.WALL):
                return (j, p)
            return True
        arr = _push3(cls, g, c, send)
        want = np.zeros_like(g)
        for n in np.flatnonzero(act):
            gi = arr[:, n]
            assert not np.isnan(gi).any()
            C = gi.sum()
            kk = k if cls.ravel()[n] == O.BIOFILM else 0.0
            want[:, n] = gi - (gi - w * C * (1 + 4 * (c @ u[:, n]))) / tau_d - w * kk * C
        got, _ = O.ad_step(cls, g, u, D, c_in, k)
        assert np.abs(got - want).max() < 1e-15
        g = got


def test_inlet_injects_exactly_u_in_per_node():
    cls = _tiny_mask()
    rng = np.random.default_rng(5)
    f = O.fluid_init(cls) * (1 + 0.1 * rng.random((9, cls.size))) * (cls.ravel() == 0)
    fin, _ = O.fluid_fluxes(cls, f, 0.03)
    assert fin == pytest.approx(0.03 * 3, rel=1e-14)

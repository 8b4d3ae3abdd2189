"""Pins of the bio-electrochemical oracle (Sec. 2.2, Eqs. 14-21, Table 1).

Each check rests on something other than the oracle's own formulas: the
Kirchhoff balance the current must satisfy (Eq. 17), the charge passed
against the mediator oxidised, independent root solves by scipy on a
different formulation of the same equations, the fixed point of the
interval update, and the currents and voltage the paper reports.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle.bioelec as B

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _state(n_nodes=40, n_bio=12, seed=0, c_lat=1.0):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.2, n_nodes) * c_lat
    cbio = np.zeros(n_nodes)
    idx = rng.choice(n_nodes, n_bio, replace=False)
    cbio[idx] = rng.uniform(100.0, 600.0, n_bio)
    mox = np.zeros(n_nodes)
    mox[idx] = rng.uniform(0.0, 0.05, n_bio)
    return C, cbio, mox


def test_eq16_rate_at_half_saturation_and_limits():
    p = B.table1_params(1.0)
    assert B.consumption_rate(p["K_s"], p["K_Mox"], p) == p["q_max"] / 4
    assert B.consumption_rate(0.0, 0.03, p) == 0.0
    assert B.consumption_rate(20.0, 0.0, p) == 0.0
    big = B.consumption_rate(1e12 * p["K_s"], 1e12 * p["K_Mox"], p)
    assert abs(big - p["q_max"]) < 1e-10 * p["q_max"]


def test_kirchhoff_eq17_holds_with_eps_zero():
    """With eps = 0, Eq. 20 is Eq. 17 solved for I: the returned current and
    overpotentials close the voltage loop I R_ext = E0 - I R_int - n_conc - n_act."""
    p = B.table1_params(1.0)
    p["eps"] = 0.0
    for seed in range(4):
        C, cbio, mox = _state(seed=seed)
        _, o = B.bio_step(C, cbio, mox, p, C.size)
        assert o["I_cell"] > 0.0
        lhs = o["I_cell"] * p["R_ext"]
        rhs = p["E0"] - o["I_cell"] * p["R_int"] - o["n_conc"] - o["n_act"]
        assert abs(lhs - rhs) < 1e-13, (lhs, rhs)


def test_eq20_holds_with_eps():
    p = B.table1_params(1.0)
    C, cbio, mox = _state(seed=7)
    _, o = B.bio_step(C, cbio, mox, p, C.size)
    Mred = o["M_red"]
    rhs = (p["E0"] - o["n_conc"] - o["n_act"]) / (p["R_int"] + p["R_ext"]) * Mred / (p["eps"] + Mred)
    # the root is exact to a few ulps of I; the right-hand side falls
    # steeply with I (a larger current oxidises more mediator), which
    # scales that into the residual
    assert abs(o["I_cell"] - rhs) <= 1e-11 * rhs
    # the load voltage is the reported output, Eq. 21 the loop total
    assert o["V_cell"] == o["I_cell"] * p["R_ext"]
    assert o["V_total"] == o["I_cell"] * (p["R_int"] + p["R_ext"])


def test_charge_passed_equals_mediator_oxidised():
    """Summed over the biomass, Eq. 15 moves gamma I dt/(m F) of mediator to
    the oxidised form and Y q_a dt (q_a at the new state) back: the interval
    change of the biomass-weighted mediator is exactly their difference."""
    p = B.table1_params(1.0)
    C, cbio, mox = _state(seed=3)
    C = 0.4 + 0.6 * C          # substrate everywhere: no cell reaches the cap
    mox = 0.5 * mox
    n_nodes = C.size
    new, o = B.bio_step(C, cbio, mox, p, n_nodes)
    cells = cbio > 0
    assert np.all(new[cells] < p["M_total"])          # cap not active here
    v = p["V_a"] / n_nodes
    dM = float(np.sum(cbio[cells] * v * (new[cells] - mox[cells])))
    S = p["c_scale"] * C[cells]
    q = B.consumption_rate(S, new[cells], p)
    reduced = float(np.sum(cbio[cells] * v * p["Y"] * q)) * p["dt_hours"] / 24.0
    oxidised = p["gamma"] * o["I_cell"] * p["dt_hours"] * 3600.0 / (p["m"] * B.FARADAY)
    assert abs(dM - (oxidised - reduced)) < 1e-12 * max(oxidised, reduced)
    assert abs(o["biomass"] - float(np.sum(cbio[cells])) * v) < 1e-12 * o["biomass"]


def _nested_brentq(C, cbio, mox, p, n_nodes):
    """The same interval solved another way: each cell's Eq. 15 by scipy's
    brentq on M (not the quadratic formula), the current by brentq on
    I - I_20(I)."""
    cells = np.flatnonzero(cbio > 0)
    cb, M0 = cbio[cells], mox[cells]
    S = p["c_scale"] * np.maximum(C[cells], 0.0)
    dt_s, dt_d = p["dt_hours"] * 3600.0, p["dt_hours"] / 24.0
    biomass = float(np.sum(cb)) * p["V_a"] / n_nodes

    def cell_M(I):
        beta = p["gamma"] * I * dt_s / (p["m"] * B.FARADAY * biomass)
        out = []
        for s, m0 in zip(S, M0):
            g = lambda M: M - m0 + p["Y"] * dt_d * B.consumption_rate(s, M, p) - beta
            hi = m0 + beta + 1.0
            out.append(min(brentq(g, 0.0, hi, xtol=1e-300, rtol=8.9e-16, maxiter=500), p["M_total"]))
        return np.array(out)

    def F(I):
        M = cell_M(I)
        mbar = float(np.sum(cb * M) / np.sum(cb))
        Mred = p["M_total"] - mbar
        if Mred <= 0:
            return I
        phi = B.R_GAS * p["T"] / B.FARADAY
        n_conc = phi * math.log(p["M_total"] / Mred)
        n_act = I * phi * mbar / (p["m"] * p["A_a"] * p["I0"] * Mred)
        I20 = max(0.0, (p["E0"] - n_conc - n_act) * Mred / ((p["R_int"] + p["R_ext"]) * (p["eps"] + Mred)))
        return I - I20

    I = brentq(F, 0.0, p["E0"] / (p["R_int"] + p["R_ext"]), xtol=1e-22, rtol=8.9e-16, maxiter=500)
    return I, cells, cell_M(I)


@pytest.mark.parametrize("seed", [1, 2])
def test_matches_nested_scalar_root_solves(seed):
    p = B.table1_params(0.8)
    C, cbio, mox = _state(n_nodes=30, n_bio=5, seed=seed, c_lat=0.8)
    new, o = B.bio_step(C, cbio, mox, p, C.size)
    I, cells, M = _nested_brentq(C, cbio, mox, p, C.size)
    assert abs(o["I_cell"] - I) < 1e-12 * I
    assert np.allclose(new[cells], M, rtol=1e-11, atol=1e-17)


def test_uniform_cells_reduce_to_one_scalar_equation():
    """Identical cells: the interval is one equation in M, with the current
    of Eq. 20 at M in closed form (n_act is linear in I):
        I(M) = h (E0 - n_conc) / (R_tot + h r),  h = M_red/(eps + M_red),
        r = R T/(F m A_a I0) * M/M_red,
    and M - M0 + Y q_a(M) dt - beta(I(M)) = 0."""
    p = B.table1_params(1.0)
    n_nodes, nb = 400, 25
    C = np.full(n_nodes, 0.6)
    cbio = np.zeros(n_nodes)
    cbio[:nb] = 450.0
    mox = np.where(cbio > 0, 0.04, 0.0)
    new, o = B.bio_step(C, cbio, mox, p, n_nodes)
    S = p["c_scale"] * 0.6
    biomass = nb * 450.0 * p["V_a"] / n_nodes
    phi = B.R_GAS * p["T"] / B.FARADAY
    R_tot = p["R_int"] + p["R_ext"]

    def I_of(M):
        Mred = p["M_total"] - M
        h = Mred / (p["eps"] + Mred)
        r = phi / (p["m"] * p["A_a"] * p["I0"]) * M / Mred
        return max(0.0, h * (p["E0"] - phi * math.log(p["M_total"] / Mred)) / (R_tot + h * r))

    def G(M):
        beta = p["gamma"] * I_of(M) * 3600.0 / (p["m"] * B.FARADAY * biomass)
        return M - 0.04 + p["Y"] / 24.0 * B.consumption_rate(S, M, p) - beta

    M = brentq(G, 0.0, p["M_total"] * (1 - 1e-12), xtol=1e-300, rtol=8.9e-16, maxiter=500)
    assert np.allclose(new[:nb], M, rtol=1e-11)
    assert abs(o["I_cell"] - I_of(M)) < 1e-11 * o["I_cell"]


def test_repeated_intervals_reach_the_mediator_balance():
    """Fixed substrate field: the interval map converges to the steady state
    of Eq. 15, where reduction and oxidation per interval balance."""
    p = B.table1_params(1.0)
    n_nodes, nb = 400, 25
    C = np.full(n_nodes, 0.5)
    cbio = np.zeros(n_nodes)
    cbio[:nb] = 450.0
    mox = np.where(cbio > 0, p["M_total"], 0.0)
    for _ in range(400):
        mox, o = B.bio_step(C, cbio, mox, p, n_nodes)
    S = p["c_scale"] * 0.5
    red = p["Y"] * B.consumption_rate(S, mox[0], p) / 24.0
    ox = p["gamma"] * o["I_cell"] * 3600.0 / (p["m"] * B.FARADAY * o["biomass"])
    assert abs(red - ox) < 1e-10 * red
    assert 0.0 < o["M_ox"] < p["M_total"]


def test_no_biomass_no_current():
    p = B.table1_params(1.0)
    new, o = B.bio_step(np.ones(10), np.zeros(10), np.zeros(10), p, 10)
    assert o["I_cell"] == 0.0 and o["V_cell"] == 0.0 and o["n_cells"] == 0


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def test_reported_steady_output_is_the_load_voltage():
    """The paper's steady current and voltage (results of Sec. 4) with
    Table 1's resistances: V = I R_ext, not I (R_int + R_ext) of Eq. 21."""
    g = _golden("mfc_reported_outputs.txt")
    v_load = g["I_steady_A"] * g["R_ext_ohm"]
    v_eq21 = g["I_steady_A"] * (g["R_ext_ohm"] + g["R_int_ohm"])
    assert abs(v_load - g["V_steady_V"]) < 0.02 * g["V_steady_V"]
    assert abs(v_eq21 - g["V_steady_V"]) > 0.5 * g["V_steady_V"]
    # the same current bounds the losses: E0 - I R_tot is what the
    # overpotentials take
    losses = g["E0_V"] - g["I_steady_A"] * (g["R_ext_ohm"] + g["R_int_ohm"])
    assert 0.0 < losses < 0.1


def test_negative_concentration_tail_is_not_consumed():
    """A biomass cell where the lattice field dips below zero reduces no
    mediator: its M_ox only gains the current's share beta = gamma I dt /
    (m F biomass)."""
    p = B.table1_params(1.0)
    C, cbio, mox = _state(seed=5)
    j = int(np.flatnonzero(cbio > 0)[0])
    C[j] = -0.05
    mox[j] = 0.01
    new, o = B.bio_step(C, cbio, mox, p, C.size)
    beta = p["gamma"] * o["I_cell"] * 3600.0 / (p["m"] * B.FARADAY * o["biomass"])
    assert o["I_cell"] > 0.0
    assert abs(new[j] - min(0.01 + beta, p["M_total"])) < 1e-15

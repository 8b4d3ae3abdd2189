"""Pins of the oracle's stop rule and of its coupled loop (CPU only).

The paper runs each lattice Boltzmann solver to equilibrium (Sec. 3)
and re-converges both after every biofilm update (the model loop of Sec. 2).
The reading made precise: at checks t = K, 2K, ... the residual is the
largest change per step over the check interval; the solve stops at the
first check with r <= tol (OK), on NaN/Inf or |u| > 0.3 (EDIVERGED), or
after `window` consecutive checks that set neither a new maximum of r nor a
new minimum since the last maximum (STALLED).

* The rule itself is pinned on hand-written residual sequences whose
  deciding check is worked out by hand from that statement: a plateau, a
  rise before a decay, a new minimum that restarts the count, a new maximum
  that restarts it, and the OK / EDIVERGED branches.  An off-by-one in the
  count or a wrong reset at a new peak moves the deciding check.
* The solves are pinned to the rule and to the residual's definition: the
  residual sequence is rebuilt from fixed-step runs (no residual logic) and
  the solve must stop at the check the rule picks on it, with that status.
* The coupled loop is pinned by decomposition: with no update it is the two
  plain solves; one update is the growth pick, the cell change and two warm
  solves; the accumulated consumption is the sum of the per-update values.
"""
import numpy as np
import pytest

import oracle as O


# ------------------------------------------------------ hand-made sequences
# (sequence, tol, window) -> (status, index of the deciding check), each
# worked out by hand from the rule's statement.
HAND = [
    # a plateau right after the first check: the first check is the peak,
    # the next three set nothing new -> stop at the third of them
    (([5.0, 5.0, 5.0, 5.0, 5.0], 1e-6, 3), ("STALLED", 3)),
    # decay then plateau: 4 and 3 are new minima; the flat 3s count 1, 2, 3
    (([5.0, 4.0, 3.0, 3.0, 3.0, 3.0, 3.0], 1e-6, 3), ("STALLED", 5)),
    # a filling transient: the rise sets new maxima (no count), then the decay
    # sets new minima; only the final plateau counts
    (([1.0, 2.0, 3.0, 3.0, 2.5, 2.5, 2.5, 2.5], 1e-6, 3), ("STALLED", 7)),
    # a new minimum restarts the count: 3 (count 0), 3, 3 (count 2), 2 (new
    # minimum, count 0), 2, 2, 2 (count 3)
    (([5.0, 3.0, 3.0, 3.0, 2.0, 2.0, 2.0, 2.0], 1e-6, 3), ("STALLED", 7)),
    # a new maximum restarts the count and resets the minimum: after 6 the
    # value 4 is a new minimum (below 6) although it is above the old one
    (([5.0, 3.0, 3.0, 6.0, 4.0, 4.0, 4.0, 4.0], 1e-6, 3), ("STALLED", 7)),
    # a new maximum restarts a count already under way: 3, 3 (count 2), 6
    # (new peak, count 0), 6, 6 (count 2): not yet stalled
    (([5.0, 3.0, 3.0, 3.0, 6.0, 6.0, 6.0], 1e-6, 3), ("NOT_CONVERGED", 7)),
    # a rise that stays below the peak is neither: it counts
    (([5.0, 3.0, 3.0, 4.0, 4.0], 1e-6, 3), ("STALLED", 4)),
    # equal to the minimum is not a new minimum; equal to the peak is not a
    # new maximum
    (([5.0, 2.0, 5.0, 2.0], 1e-6, 2), ("STALLED", 3)),
    # strictly decreasing: never stalls, never reaches tol
    (([1.0, 0.5, 0.25, 0.125, 0.0625], 1e-6, 1), ("NOT_CONVERGED", 5)),
    # tol reached at the first check at or below it, also while counting
    (([5.0, 3.0, 3.0, 1e-6, 0.0], 1e-6, 3), ("OK", 3)),
    (([5.0, 3.0, 3.0, 3.0, 1e-7], 1e-6, 4), ("OK", 4)),
    # window 0 disables the stall test
    (([5.0] * 50, 1e-6, 0), ("NOT_CONVERGED", 50)),
    # window 1: the first check that sets nothing stops the solve
    (([5.0, 4.0, 4.0], 1e-6, 1), ("STALLED", 2)),
    # NaN and infinity diverge at once
    (([5.0, 4.0, float("nan"), 1e-9], 1e-6, 3), ("EDIVERGED", 2)),
    (([5.0, float("inf")], 1e-6, 3), ("EDIVERGED", 1)),
]


@pytest.mark.parametrize("case,expect", HAND)
def test_stop_rule_hand_sequences(case, expect):
    r, tol, window = case
    assert O.stall_rule(r, tol, window) == expect


def test_stop_rule_low_mach_guard():
    r = [5.0, 4.0, 3.0, 2.0]
    # |u| above 0.3 at the third check diverges there; 0.3 itself does not
    assert O.stall_rule(r, 1e-6, 3, umax=[0.1, 0.2, 0.31, 0.1]) == ("EDIVERGED", 2)
    assert O.stall_rule(r, 1e-6, 3, umax=[0.1, 0.3, 0.3, 0.3]) == ("NOT_CONVERGED", 4)
    # divergence outranks convergence at the same check
    assert O.stall_rule([5.0, 1e-9], 1e-6, 3, umax=[0.1, 0.5]) == ("EDIVERGED", 1)
    assert O.stall_rule([5.0, 1e-9], 1e-6, 3, umax=[0.1, float("nan")]) == ("EDIVERGED", 1)


# ------------------------------------------- solves stop where the rule says
def _channel(nx=16, u=0.02):
    """y-uniform substrate channel between WALL rows, a BIOFILM row in the
    middle (sink), constant velocity along x."""
    cls = np.zeros((3, nx), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    cls[1] = O.BIOFILM
    uu = np.zeros((2, 3 * nx))
    uu[0] = u
    return cls, uu


def _porous_substrate():
    """A small porous electrode with its biofilm layer and a seeded frozen
    velocity (x component 0.01-0.015, y component within +-0.002, zero off
    FLUID nodes): its FP64 substrate solve ends on a round-off floor that
    wobbles near 1e-15 instead of reaching an exact fixed point."""
    st, cls, _ = O.geom_discs(32, 16, 2, 3, 0.2, 0, 3)
    assert st == "OK"
    cls = O.biofilm_layer(cls)
    rng = np.random.default_rng(1)
    uu = np.zeros((2, cls.size))
    uu[0] = 0.01 + 0.005 * rng.random(cls.size)
    uu[1] = 0.004 * (rng.random(cls.size) - 0.5)
    uu[:, cls.ravel() != O.FLUID] = 0.0
    return cls, uu


def test_ad_solve_stalls_at_the_check_the_rule_picks():
    cls, uu = _porous_substrate()
    D, c_in, k, K, window = 0.1, 1.0, 1e-2, 7, 3
    g0 = O.ad_init(cls, uu, c_in)
    # residual sequence from fixed-step runs: C at t = 0, K, 2K, ...
    active = ~np.isin(cls.ravel(), [O.SOLID, O.WALL])
    Cprev = O.ad_moment(cls, g0, k)
    g, rs = g0, []
    for _ in range(2600):
        g, C = O.ad_run(cls, g, uu, D, c_in, k, K)
        rs.append(float(np.abs(C - Cprev)[active].max()) / (K * c_in))
        Cprev = C
    # tol below the FP64 round-off floor: the rule must stall on it
    tol = 1e-30
    status, at = O.stall_rule(rs, tol, window)
    assert status == "STALLED", (status, at)
    # it stops on the floor, not in the decay
    assert 0.0 < rs[at] < 1e-13
    r = O.ad_solve(cls, uu, D, c_in, k, tol, 10_000_000, check_every=K, stall_checks=window)
    assert r["status"] == "STALLED"
    assert r["iters"] == K * (at + 1)
    assert r["residual"] == rs[at]
    # a longer window stops later (the count can reach it one check later
    # at the earliest)
    r2 = O.ad_solve(cls, uu, D, c_in, k, tol, 10_000_000, check_every=K, stall_checks=window + 2)
    st2, at2 = O.stall_rule(rs, tol, window + 2)
    assert r2["status"] == st2 == "STALLED" and r2["iters"] == K * (at2 + 1) and at2 > at
    # a tol above the floor ends OK at the first check at or below it
    tol_ok = 1e-12
    st3, at3 = O.stall_rule(rs, tol_ok, window)
    r3 = O.ad_solve(cls, uu, D, c_in, k, tol_ok, 10_000_000, check_every=K, stall_checks=window)
    assert st3 == r3["status"] == "OK" and r3["iters"] == K * (at3 + 1)
    assert rs[at3] <= tol_ok < min(rs[:at3])


def test_fluid_solve_stops_at_the_check_the_rule_picks():
    st, cls, _ = O.geom_discs(48, 20, 2, 4, 0.25, 0, 7)
    assert st == "OK"
    cls = O.biofilm_layer(cls)
    assert O.percolates(cls)
    tau, u_in, K, window = 0.8, 0.01, 20, 15
    f = O.fluid_init(cls)
    Uprev, _ = O.fluid_moments(cls, f)
    rs, um = [], []
    for _ in range(1500):
        f, U, _ = O.fluid_run(cls, f, tau, u_in, K)
        rs.append(float(np.abs(U - Uprev).max()) / (K * u_in))
        um.append(float(np.abs(U).max()))
        Uprev = U
    # the filling transient: the residual rises before it decays
    assert max(rs[:10]) > rs[0]
    # a short window stalls inside the transient's wobble; a long one runs
    # on to the tolerance
    for tol, win, want in ((2e-4, window, "OK"), (1e-30, 3, "STALLED")):
        status, at = O.stall_rule(rs, tol, win, umax=um)
        assert status == want, (tol, status, at)
        r = O.fluid_solve(cls, tau, u_in, tol, 10_000_000, check_every=K, stall_checks=win)
        assert r["status"] == status
        assert r["iters"] == K * (at + 1)
        assert r["residual"] == rs[at]


def test_solve_max_iter_between_checks():
    # max_iter that is not a multiple of K stops at max_iter itself
    cls, uu = _channel()
    r = O.ad_solve(cls, uu, 0.1, 1.0, 1e-2, 1e-30, 37, check_every=10, stall_checks=20)
    assert r["status"] == "NOT_CONVERGED" and r["iters"] == 37


# --------------------------------------------------------- the coupled loop
PH = dict(tau=0.8, u_in=0.01, D=0.2 / 3.0, c_in=1.0, k_sink=1e-3, tol=1e-5, max_iter=200_000)


def _electrode():
    st, cls, _ = O.geom_discs(64, 32, 3, 5, 0.3, 0, 5)
    assert st == "OK"
    cls = O.biofilm_layer(cls)
    assert O.percolates(cls)
    return cls


def _plain(cls, f=None, g=None):
    """Fluid then substrate steady solves (warm where states are given)."""
    rf = O.fluid_solve(cls, PH["tau"], PH["u_in"], PH["tol"], PH["max_iter"], f=f)
    if g is None:
        g = O.ad_init(cls, rf["U"], PH["c_in"])
    ra = O.ad_solve(cls, rf["U"], PH["D"], PH["c_in"], PH["k_sink"], PH["tol"], PH["max_iter"], g=g)
    J = O.ad_fluxes(cls, ra["g"], PH["c_in"], PH["k_sink"])[2]
    return rf, ra, J


def _coupled(cls, xi):
    return O.coupled_run(cls, PH["tau"], PH["u_in"], PH["D"], PH["c_in"], PH["k_sink"],
                         PH["tol"], PH["max_iter"], xi)


def _biofilm_neighbour(cls, p):
    ny, nx = cls.shape
    y, x = divmod(p, nx)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if (dx or dy) and 0 <= y + dy < ny and 0 <= x + dx < nx:
                if cls[y + dy, x + dx] == O.BIOFILM:
                    return True
    return False


def test_coupled_loop_without_updates_is_the_two_plain_solves():
    cls = _electrode()
    c = _coupled(cls, np.zeros(0))
    rf, ra, J = _plain(cls)
    assert c["status"] == "OK" and rf["status"] == "OK" and ra["status"] == "OK"
    assert c["iters_fluid"][0] == rf["iters"] and c["iters_ad"][0] == ra["iters"]
    assert np.array_equal(c["U"], rf["U"]) and np.array_equal(c["C"], ra["C"])
    assert c["J"][0] == J
    assert c["J_accum"] == 0.0
    assert np.array_equal(c["cls"], cls)


def test_coupled_loop_one_update_is_pick_change_and_warm_solves():
    cls = _electrode()
    xi = 0.37
    rf, ra, _ = _plain(cls)
    p = O.growth_pick(cls, ra["C"], xi)
    ny, nx = cls.shape
    assert cls.ravel()[p] == O.FLUID and 1 <= p % nx <= nx - 2 and _biofilm_neighbour(cls, p)
    cls1 = cls.copy()
    cls1.ravel()[p] = O.BIOFILM
    f = rf["f"].copy()
    f[:, p] = 0.0                       # its fluid populations are dropped
    rf1, ra1, J1 = _plain(cls1, f=f, g=ra["g"])   # its substrate populations kept
    c = _coupled(cls, np.array([xi]))
    assert c["status"] == "OK"
    assert c["picked"][0] == p
    assert np.array_equal(c["cls"], cls1)
    assert c["iters_fluid"][1] == rf1["iters"] and c["iters_ad"][1] == ra1["iters"]
    assert np.array_equal(c["U"], rf1["U"]) and np.array_equal(c["C"], ra1["C"])
    assert c["J"][1] == J1 and c["J_accum"] == J1
    # warm re-solves after a one-cell change take fewer steps than cold ones
    assert rf1["iters"] < rf["iters"]


def test_coupled_loop_accumulates_and_grows_biofilm():
    cls = _electrode()
    xi = np.array([0.9, 0.05, 0.5, 0.71])
    c = _coupled(cls, xi)
    assert c["status"] == "OK"
    acc = 0.0
    for m in range(1, len(xi) + 1):
        acc += c["J"][m]
    assert c["J_accum"] == acc
    picked = c["picked"]
    assert len(set(picked.tolist())) == len(xi)
    changed = np.flatnonzero(c["cls"].ravel() != cls.ravel())
    assert np.array_equal(np.sort(changed), np.sort(picked))
    assert np.all(c["cls"].ravel()[picked] == O.BIOFILM)
    assert np.all(cls.ravel()[picked] == O.FLUID)
    # each pick had a biofilm neighbour in the mask at its own update
    cur = cls.copy()
    for p in picked:
        assert _biofilm_neighbour(cur, int(p))
        cur.ravel()[p] = O.BIOFILM
    # consumption grows with the biofilm it is taken over (more sink nodes)
    assert c["J"][-1] > c["J"][0]

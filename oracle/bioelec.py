"""FP64 numpy reference of the bio-electrochemical model (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke
check and the CPU-baseline leg of the benchmark, never by the library.  It
shares no code or constant with the HIP library.

Tsompanas et al., arXiv 1802.07525, Sec. 2.2 (Eqs. 14-21), Table 1.  Once
per model interval (one hour, Sec. 3), after the two lattice Boltzmann
solves, the model updates the intracellular mediator of every cell holding
biomass and the cell's electrical outputs:

  Eq. 14  M_total = M_red + M_ox                       (per unit biomass)
  Eq. 15  M_ox(t+1) = M_ox(t) - Y q_a + gamma I/(m F) / (V_a C_bio)
  Eq. 16  q_a = q_max C_s/(C_s + K_s) * M_ox/(M_ox + K_Mox)
  Eq. 17  I R_ext = E0 - I R_int - n_conc - n_act      (Kirchhoff)
  Eq. 18  n_conc = (R T / F) ln(M_total / M_red)       (Nernst)
  Eq. 19  n_act = I/(A_a I0) * R T/(m F) * M_ox/M_red  (Butler-Volmer, linearised)
  Eq. 20  I = (E0 - n_conc - n_act)/(R_int + R_ext) * M_red/(eps + M_red)
  Eq. 21  V = I (R_int + R_ext)

Readings (the paper is silent or ambiguous):
  - Eq. 15 advances one interval.  Its rates are taken at the new state
    (backward Euler): with Table 1's values one hour of reduction,
    Y q_max/24 ~ 0.2, and of oxidation at ~1 mA both exceed M_total = 0.05,
    so the update evaluated at the old state flips the mediator between 0
    and M_total every hour.  At the new state the update is unconditionally
    stable and its fixed point is the steady mediator balance.
  - Units: q_max per day, the interval in hours; C_s in mg/L is the lattice
    concentration times c_scale (c_in maps to Table 1's C_s^in).
  - V_a C_bio in Eq. 15 is the total biomass in the compartment: the sum
    over biomass cells of C_bio times the cell volume V_a/N (N lattice
    cells).  The current then oxidises every unit of biomass alike and the
    mediator oxidised in total is gamma I dt/(m F), the charge passed.
  - Eqs. 18-20 take the biomass-weighted means of M_ox and M_red (one cell
    current for the whole anode).
  - The negative-concentration tail of the lattice field is not consumed:
    q_a uses max(C_s, 0).  M_ox is kept within [0, M_total] (Eq. 14).
  - Eq. 20 holds at the new state; with n_act linear in I the current is
    the unique root of F(I) = I - max(0, I_20(I)), found by bisection on
    [0, E0/(R_int + R_ext)] (F rises with I: a larger current oxidises more
    mediator, which lowers M_red and the right-hand side of Eq. 20).
  - The reported output voltage is the load voltage I R_ext, the left side
    of Eq. 17: the paper's steady 0.91 mA and ~330 mV satisfy it, whereas
    Eq. 21 would give twice that.  V_total = I (R_int + R_ext) (Eq. 21) is
    reported beside it.
  - Not in Table 1: T = 298.15 K; eps = 0.01 M_total; A_a the electrode's
    projected face, 48 mm x 65 mm; V_a = 17 x 60 x 65 mm^3.
"""
import math

import numpy as np

R_GAS = 8.314462618     # J / (mol K)
FARADAY = 96485.33212   # C / mol

# root-solve iteration cap (bisection halvings); the loop stops earlier once
# the midpoint no longer lies strictly inside the bracket
ROOT_ITERS = 80


def table1_params(c_in_lattice):
    """Table 1's values (mg, L, day, A, V, ohm, m^2) plus the readings above."""
    M_total = 0.05
    return dict(q_max=8.48, K_s=20.0, M_total=M_total, K_Mox=0.02 * M_total,
                Y=0.5687, gamma=663400.0, m=2.0, I0=1e-3, E0=0.7,
                R_ext=360.0, R_int=360.0, A_a=48e-3 * 65e-3, V_a=17 * 60 * 65 * 1e-6,
                T=298.15, eps=0.01 * M_total, C0_bio=450.0,
                c_scale=410.0 / c_in_lattice, dt_hours=1.0)


def consumption_rate(Cs, Mox, p):
    """Eq. 16: double-Monod substrate consumption, mg substrate/(mg biomass day)."""
    return p["q_max"] * Cs / (Cs + p["K_s"]) * Mox / (Mox + p["K_Mox"])


def cell_mediator(M0, a, beta, p):
    """Eq. 15 over one interval with the reduction at the new state:
    M = M0 - a M/(M + K) + beta, K = K_Mox, a = Y q_max dt S/(S + K_s) and
    beta the oxidation by the current.  Multiplying out gives
    M^2 + (K + a - M0 - beta) M - (M0 + beta) K = 0, whose root M >= 0 is
    the textbook quadratic formula; then Eq. 14 caps M at M_total."""
    K = p["K_Mox"]
    b = K + a - (M0 + beta)
    c = -(M0 + beta) * K
    M = (-b + np.sqrt(b * b - 4.0 * c)) / 2.0
    return np.minimum(M, p["M_total"])


def overpotentials(I, Mox_mean, p):
    """Eqs. 18-19 at mean M_ox (M_red from Eq. 14); n_conc is +inf when no
    mediator is reduced."""
    phi = R_GAS * p["T"] / FARADAY
    Mred = p["M_total"] - Mox_mean
    if Mred <= 0.0:
        return math.inf, math.inf
    n_conc = phi * math.log(p["M_total"] / Mred)
    n_act = I / (p["A_a"] * p["I0"]) * phi / p["m"] * (Mox_mean / Mred)
    return n_conc, n_act


def current_eq20(I, Mox_mean, p):
    """Right-hand side of Eq. 20 at trial current I, floored at 0."""
    Mred = p["M_total"] - Mox_mean
    if Mred <= 0.0:
        return 0.0
    n_conc, n_act = overpotentials(I, Mox_mean, p)
    val = (p["E0"] - n_conc - n_act) / (p["R_int"] + p["R_ext"]) * Mred / (p["eps"] + Mred)
    return max(val, 0.0)


def bio_step(C, cbio, mox, p, n_cells):
    """One interval of the bio-electrochemical model.

    C: lattice concentration at every node; cbio: biomass (mg/L) at every
    node (0 where none); mox: M_ox at every node (ignored where cbio = 0);
    n_cells: lattice cells N of the compartment.  Returns (new M_ox at every
    node, outputs)."""
    C = np.asarray(C, np.float64).reshape(-1)
    cbio = np.asarray(cbio, np.float64).reshape(-1)
    mox = np.asarray(mox, np.float64).reshape(-1)
    cells = np.flatnonzero(cbio > 0.0)
    out_mox = mox.copy()
    dt_day = p["dt_hours"] / 24.0
    dt_s = p["dt_hours"] * 3600.0
    R_tot = p["R_int"] + p["R_ext"]
    if cells.size == 0:
        out = dict(I_cell=0.0, V_cell=0.0, V_total=0.0, n_conc=0.0, n_act=0.0,
                   M_ox=0.0, M_red=0.0, biomass=0.0, q_total=0.0, n_cells=0, root_iters=0)
        return out_mox, out
    cb = cbio[cells]
    M0 = mox[cells]
    S = p["c_scale"] * np.maximum(C[cells], 0.0)
    a = p["Y"] * p["q_max"] * dt_day * S / (S + p["K_s"])
    v = p["V_a"] / n_cells
    sum_cb = 0.0
    for x in cb:                      # ascending node order
        sum_cb += x
    biomass = sum_cb * v

    def mean_mox(I):
        beta = p["gamma"] * I * dt_s / (p["m"] * FARADAY * biomass)
        M = cell_mediator(M0, a, beta, p)
        s = 0.0
        for w, m in zip(cb, M):
            s += w * m
        return M, s / sum_cb

    lo, hi = 0.0, p["E0"] / R_tot
    iters = 0
    for _ in range(ROOT_ITERS):
        mid = lo + (hi - lo) / 2.0
        if not (lo < mid < hi):
            break
        iters += 1
        _, mbar = mean_mox(mid)
        if mid - current_eq20(mid, mbar, p) > 0.0:
            hi = mid
        else:
            lo = mid
    I = lo
    M, mbar = mean_mox(I)
    out_mox[cells] = M
    n_conc, n_act = overpotentials(I, mbar, p)
    q = consumption_rate(S, M, p)
    q_total = 0.0
    for w, x in zip(cb, q):
        q_total += w * x
    q_total *= v / 24.0               # mg substrate per hour
    out = dict(I_cell=I, V_cell=I * p["R_ext"], V_total=I * R_tot, n_conc=n_conc,
               n_act=n_act, M_ox=mbar, M_red=p["M_total"] - mbar, biomass=biomass,
               q_total=q_total, n_cells=int(cells.size), root_iters=iters)
    return out_mox, out

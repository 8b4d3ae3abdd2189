"""Seeded synthetic workloads: sizes, parameters, seeds and random draws.

This module holds no lattice arithmetic.  It names the workloads (grid,
electrode generator settings, relaxation times, inflow, sink, tolerance and
seed) and draws the random inputs both the HIP path and the oracle receive:
random population states for fixed-step comparisons, the uniform numbers of
the biofilm growth draws, the parameters and arrival times of a served
request stream, and the biomass and mediator fields and Table 1 values of
the bio-electrochemical model.  Each side builds its electrode mask itself from the
generator settings and seed here.

Substrate diffusivities are given directly as D = c_s^2 (tau_D - 1/2)
(c_s^2 = 1/3 for D2Q5, 1/4 for D3Q7) for the tau_D values the workloads
name.  `layer` says whether the one-cell biofilm layer (the nodes the
substrate sink acts on) is grown around the electrode.
"""
import numpy as np

WORKLOADS = {
    # 2-D plain method, 128 x 64 channel; discs (radius 3-6, solid fraction
    # 0.3) in the middle 64 columns, 1-cell biofilm layer; tau_D = 0.7.
    "c1": dict(name="d2q9+d2q5 128x64 discs r3-6 solid0.3", nx=128, ny=64, nz=1,
               geom="discs", r_min=3, r_max=6, solid=0.3, overlap=0, seed=1, layer=True,
               tau=0.8, u_in=0.01, D=0.2 / 3.0, c_in=1.0, k=1e-3, tol=1e-8, max_iter=10000),
    # 2-D single solve, 1024 x 512; discs radius 4-10, porosity 0.6 over the
    # central half; tau = tau_D = 0.6, u_in = 0.02.  No biofilm layer: none
    # is named for this workload, and on these near-jammed discs the layer
    # closes the 1-2 cell throats and drives the pore velocity past 0.3.
    "c2": dict(name="d2q9+d2q5 1024x512 discs r4-10 porosity0.6", nx=1024, ny=512, nz=1,
               geom="discs", r_min=4, r_max=10, solid=0.4, overlap=0, seed=2, layer=False,
               tau=0.6, u_in=0.02, D=0.1 / 3.0, c_in=1.0, k=1e-3, tol=1e-6, max_iter=3_000_000),
    # 3-D, 256 x 128 x 128; random cylinders radius 2-4, porosity 0.8;
    # tau = 0.7, tau_D = 0.65 (D3Q7, c_s^2 = 1/4).
    "c3": dict(name="d3q19+d3q7 256x128x128 fibres r2-4 porosity0.8", nx=256, ny=128, nz=128,
               geom="fibres", r_min=2, r_max=4, solid=0.2, overlap=1, seed=3, layer=True,
               tau=0.7, u_in=0.01, D=0.15 / 4.0, c_in=1.0, k=1e-3, tol=1e-6, max_iter=3_000_000),
    # coupled biofilm loop, 512 x 256, porosity 0.7, 200 growth updates; the
    # physics is not named for this workload: the 128 x 64 workload's
    # (tau = 0.8, u_in = 0.01, tau_D = 0.7) is used.
    "c5": dict(name="d2q9+d2q5 512x256 discs r3-6 porosity0.7 coupled", nx=512, ny=256, nz=1,
               geom="discs", r_min=3, r_max=6, solid=0.3, overlap=0, seed=5, layer=True,
               tau=0.8, u_in=0.01, D=0.2 / 3.0, c_in=1.0, k=1e-3, tol=1e-6, max_iter=1_000_000,
               updates=200),
    # the model loop of Sec. 2 (fluid, substrate, bio-electrochemistry,
    # biofilm), one hour per interval, over the 72 hours the paper simulates:
    # the coupled workload's 512 x 256 electrode, bare (the biofilm attaches
    # and grows), Table 1's bio parameters
    "mfc": dict(name="d2q9+d2q5 512x256 discs r3-6 porosity0.7 model loop 72h", nx=512, ny=256,
                nz=1, geom="discs", r_min=3, r_max=6, solid=0.3, overlap=0, seed=5, layer=False,
                tau=0.8, u_in=0.01, D=0.2 / 3.0, c_in=1.0, k=1e-3, tol=1e-6,
                max_iter=1_000_000, hours=72),
    # large 2-D bandwidth point (well beyond the 256 MB last-level cache)
    "c2_hbm": dict(name="d2q9+d2q5 8192x4096 discs r4-10 porosity0.6", nx=8192, ny=4096, nz=1,
                   geom="discs", r_min=4, r_max=10, solid=0.4, overlap=0, seed=2, layer=False,
                   tau=0.6, u_in=0.02, D=0.1 / 3.0, c_in=1.0, k=1e-3, tol=1e-6, max_iter=2000),
}

# served stream: request i draws its parameters from seed SERVE_SEED and its
# electrode from seed SERVE_GEOM_BASE + i
SERVE_SEED = 4
SERVE_GEOM_BASE = 4_000_000
SERVE_RATES = (1, 5, 20, 50, 100, 200, 400, 800)


def scaled(w, nx, ny, nz=None, **over):
    """A copy of workload w with another grid (same physics and seed)."""
    d = dict(w)
    d.update(nx=nx, ny=ny)
    if nz is not None:
        d["nz"] = nz
    d.update(over)
    return d


def random_populations(q, n, seed, scale=0.05, base=None):
    """q x n state: base (if given) times (1 + scale * U[-1, 1))."""
    rng = np.random.default_rng(seed)
    r = 1.0 + scale * (2.0 * rng.random((q, n)) - 1.0)
    return r if base is None else base * r


def random_velocity(dim, n, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    return amp * (2.0 * rng.random((dim, n)) - 1.0)


def growth_draws(count, seed):
    """Uniform numbers in [0, 1) for the biofilm growth picks."""
    return np.random.default_rng(seed).random(count)


# Bio-electrochemical model (Sec. 2.2): Table 1's values (mg, L, day, A, V,
# ohm) and the values Table 1 does not give -- temperature 298.15 K,
# eps = 0.01 M_total, the electrode's projected face 48 x 65 mm as A_a and
# the compartment 17 x 60 x 65 mm as V_a.  The lattice concentration c_in
# stands for Table 1's inflow of 410 mg/L.
BIO_TABLE1 = dict(q_max=8.48, K_s=20.0, M_total=0.05, K_Mox=0.02 * 0.05, Y=0.5687,
                  gamma=663400.0, m=2.0, I0=1e-3, E0=0.7, R_ext=360.0, R_int=360.0,
                  A_a=48e-3 * 65e-3, V_a=17 * 60 * 65 * 1e-6, T=298.15, eps=0.01 * 0.05,
                  C0_bio=450.0, dt_hours=1.0)
BIO_CIN_MG_L = 410.0


def bio_params(c_in, **over):
    """BIO_TABLE1 with c_scale = 410 mg/L / c_in, plus overrides."""
    d = dict(BIO_TABLE1)
    d["c_scale"] = BIO_CIN_MG_L / c_in
    d.update(over)
    return d


def biomass_field(cls, seed, c0=450.0, spread=0.5, biofilm=3):
    """C_bio per node: c0 * U[1 - spread, 1 + spread) on BIOFILM nodes, 0
    elsewhere."""
    flat = np.asarray(cls).reshape(-1)
    rng = np.random.default_rng(seed)
    r = c0 * (1.0 - spread + 2.0 * spread * rng.random(flat.size))
    return np.where(flat == biofilm, r, 0.0)


def mediator_field(cls, seed, m_total=0.05, biofilm=3):
    """M_ox per node: U[0, m_total) on BIOFILM nodes, 0 elsewhere."""
    flat = np.asarray(cls).reshape(-1)
    r = m_total * np.random.default_rng(seed).random(flat.size)
    return np.where(flat == biofilm, r, 0.0)


def serve_requests(n, rate, seed=SERVE_SEED):
    """n requests with Poisson arrivals at `rate` per second.  Each is a dict
    with arrival time, grid (nx log-uniform between 64 and 2048, ny = nx/2),
    porosity U[0.4, 0.9], tau U[0.55, 1.2], u_in U[0.005, 0.03], D for
    tau_D = 0.6, k = 1e-3, tol = 1e-6 and its electrode seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n) if rate > 0 else np.zeros(n)
    t = np.cumsum(gaps) - gaps[0]
    xi = rng.random(n)
    out = []
    for i in range(n):
        nx = int(round(64 * 32 ** xi[i]))
        nx = max(64, min(2048, nx))
        out.append(dict(
            i=i, arrival=float(t[i]), nx=nx, ny=nx // 2, nz=1,
            porosity=float(rng.uniform(0.4, 0.9)), tau=float(rng.uniform(0.55, 1.2)),
            u_in=float(rng.uniform(0.005, 0.03)), D=0.1 / 3.0, c_in=1.0, k=1e-3, tol=1e-6,
            r_min=3, r_max=6, overlap=1, seed=SERVE_GEOM_BASE + i))
    return out

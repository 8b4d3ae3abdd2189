"""Agent-based biofilm formation and the model loop -- FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
CPU-baseline leg, never by the library; it shares no code with it.

Tsompanas et al., arXiv 1802.07525, Sec. 2.3 (biofilm formation), Sec. 2
(model loop) and Table 1 (k_ata, C0_bio, C_max, fr_spr).  Once per model
interval, after the bio-electrochemical update, the biomass field changes in
three stages, in the paper's order:

  attachment  k_ata cells, drawn at random among the front between the fluid
              and the electrode, receive C0_bio;
  growth      every cell's biomass grows at the double-Monod consumption
              rate of Eq. 16 (the mediator per unit biomass is unchanged, so
              the mediator grows with it);
  spreading   a cell above C_max passes fr_spr of its biomass to a free
              neighbour; with none free, a random walk through the biomass
              finds a free cell and the biomass along the walk moves one
              cell outward to free the initial cell's neighbour first.
Cells that gain biomass become BIOFILM (blocked for the fluid, sink for the
substrate), so the two lattice Boltzmann solves run again next interval.

Readings (the paper is silent or ambiguous):
  - The front is the FLUID cells with a SOLID (electrode) neighbour among
    the fluid lattice's directions; cells of the inlet and outlet columns are
    never given biomass (they hold the boundary conditions).  A free cell is
    a FLUID cell outside those columns.  BIOFILM cells can be walked
    through; SOLID, WALL and the grid's edge cannot.
  - Attachment draws min(k_ata, front size) cells without replacement (a
    partial Fisher-Yates shuffle of the front in ascending node order).  An
    attached cell starts with C0_bio and fully oxidised mediator (M_total).
  - Growth: C_bio += C_bio Y_bio q_a dt, q_a of Eq. 16 (per day) from the
    current substrate field and mediator.  The paper gives no biomass yield;
    Y_bio = 1 (growth rate per unit biomass = q_a) reads the text literally,
    and with Table 1's q_max it grows a cell by up to ~35% an hour.  Attached
    cells grow in the same interval.
  - Spreading visits nodes once in ascending order and acts on a node whose
    biomass exceeds C_max when it is visited.  A free neighbour is drawn
    uniformly among the free neighbours.  The walk steps in a uniformly drawn
    direction; a step into a blocked cell is spent in place; revisiting a
    cell erases the loop (loop-erased walk), so the path is simple; the walk
    ends at its first free cell or, after max_walk steps, gives up (no
    spreading).  Along the path p0 (the full cell), p1, ..., pk (free) each
    cell's biomass and mediator move to the next cell, from pk-1 down to p1;
    then p1 receives fr_spr C_bio(p0) with p0's mediator and p0 keeps the
    rest.
  - Random numbers: the SplitMix64 stream of the interval's seed, in the
    order the stages consume them; u = (x >> 11) 2^-53 and an index in
    [0, m) is floor(u m).  The model loop's interval h uses output h of the
    stream of its base seed as that interval's seed.
"""
import numpy as np

import oracle as O
import oracle.bioelec as OB

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


class Draws:
    """SplitMix64 outputs of one seed, in order (the generator's state after
    k outputs is seed + k * gamma, so blocks can be produced on demand)."""

    def __init__(self, seed):
        self.seed = int(seed) & MASK64
        self.k = 0
        self.buf = []

    def _next(self):
        if not self.buf:
            state = (self.seed + self.k * GOLDEN_GAMMA) & MASK64
            self.buf = [int(x) for x in O.splitmix64(state, 1024)][::-1]
        self.k += 1
        return self.buf.pop()

    def uniform(self):
        return (self._next() >> 11) * 2.0 ** -53

    def index(self, m):
        return int(self.uniform() * m)


def _lattice(nz):
    c, _, _, _ = O.lattice_tables(O.D3Q19 if nz > 1 else O.D2Q9)
    return [tuple(int(v) for v in c[i]) for i in range(1, len(c))]


def biofilm_step(cls, C, cbio, mox, bp, fp, seed):
    """One interval of attachment, growth and spreading.

    cls: class mask (shape (ny, nx) or (nz, ny, nx)); C: substrate field
    (lattice units, every node, before this step's changes); cbio, mox:
    biomass and M_ox per node; bp: bio-electrochemical parameters (Table 1);
    fp: dict(k_ata, C_max, fr_spr, max_walk, Y_bio); seed: the interval's seed.
    Returns (cls, cbio, mox, stats) as new arrays."""
    shape = cls.shape
    nz, ny, nx = (1,) + shape if len(shape) == 2 else shape
    cls = np.array(cls, np.uint8).reshape(-1)
    C = np.asarray(C, np.float64).reshape(-1)
    cb = np.array(cbio, np.float64).reshape(-1)
    mo = np.array(mox, np.float64).reshape(-1)
    N = cls.size
    dirs = _lattice(nz)
    draws = Draws(seed)

    def coords(n):
        return n % nx, (n // nx) % ny, n // (nx * ny)

    def neighbour(n, d):
        x, y, z = coords(n)
        x2, y2, z2 = x + d[0], y + d[1], z + d[2]
        if 0 <= x2 < nx and 0 <= y2 < ny and 0 <= z2 < nz:
            return x2 + nx * (y2 + ny * z2)
        return -1

    def free(n):
        return n >= 0 and cls[n] == O.FLUID and 1 <= n % nx <= nx - 2

    new_bio = []
    # attachment
    front = [n for n in range(N)
             if free(n) and any(neighbour(n, d) >= 0 and cls[neighbour(n, d)] == O.SOLID
                                for d in dirs)]
    k = min(int(fp["k_ata"]), len(front))
    for i in range(k):
        j = i + draws.index(len(front) - i)
        front[i], front[j] = front[j], front[i]
    for n in front[:k]:
        cls[n] = O.BIOFILM
        cb[n] = bp["C0_bio"]
        mo[n] = bp["M_total"]
        new_bio.append(n)
    # growth at the consumption rate of Eq. 16
    dt_day = bp["dt_hours"] / 24.0
    has = cb > 0.0
    S = bp["c_scale"] * np.maximum(C[has], 0.0)
    q = OB.consumption_rate(S, mo[has], bp)
    cb[has] = cb[has] + dt_day * (fp["Y_bio"] * q) * cb[has]
    # spreading
    spread = walks = abandoned = 0
    for n in range(N):
        if not cb[n] > fp["C_max"]:
            continue
        nbs = [neighbour(n, d) for d in dirs]
        fr = [m for m in nbs if free(m)]
        if fr:
            path = [n, fr[draws.index(len(fr))]]
        else:
            walks += 1
            path, cur, done = [n], n, False
            for _ in range(int(fp["max_walk"])):
                m = neighbour(cur, dirs[draws.index(len(dirs))])
                if free(m):
                    path.append(m)
                    done = True
                    break
                if m >= 0 and cls[m] == O.BIOFILM:
                    if m in path:
                        path = path[: path.index(m) + 1]
                    else:
                        path.append(m)
                    cur = m
            if not done:
                abandoned += 1
                continue
        last = path[-1]
        for i in range(len(path) - 1, 1, -1):
            cb[path[i]] = cb[path[i - 1]]
            mo[path[i]] = mo[path[i - 1]]
        share = fp["fr_spr"] * cb[n]
        cb[path[1]] = share
        mo[path[1]] = mo[n]
        cb[n] = cb[n] - share
        cls[last] = O.BIOFILM
        new_bio.append(last)
        spread += 1
    cells = int(np.count_nonzero(cb > 0.0))
    biomass = 0.0
    for x in cb[cb > 0.0]:
        biomass += x
    stats = dict(attached=k, spread=spread, walks=walks, abandoned=abandoned, cells=cells,
                 new_biofilm=sorted(new_bio), biomass=biomass * bp["V_a"] / N)
    return cls.reshape(shape), cb, mo, stats


def interval_seeds(seed, n):
    return [int(x) for x in O.splitmix64(int(seed), n)]


def mfc_run(cls, w, bp, fp, n_hours, seed, tol, max_iter, cbio=None, mox=None):
    """The model loop of Sec. 2 for n_hours intervals: fluid and substrate
    solves to tol (cold, then warm from the previous interval's states), the
    bio-electrochemical update (Eqs. 14-21), then biofilm formation.  w:
    dict(tau, u_in, D, c_in, k).  Returns a list of per-interval dicts and
    the final (cls, cbio, mox); stops early with status 'EINVAL' when growth
    would close the flow path (the mask no longer percolates)."""
    cls = np.array(cls, np.uint8)
    N = cls.size
    flat = cls.reshape(-1)
    cb = np.where(flat == O.BIOFILM, bp["C0_bio"], 0.0) if cbio is None else np.array(cbio, float)
    mo = np.where(cb > 0, bp["M_total"], 0.0) if mox is None else np.array(mox, float)
    f = g = None
    seeds = interval_seeds(seed, n_hours)
    out = []
    for h in range(n_hours):
        fo = O.fluid_solve(cls, w["tau"], w["u_in"], tol, max_iter, f=f)
        f = fo["f"]
        ao = O.ad_solve(cls, fo["U"], w["D"], w["c_in"], w["k"], tol, max_iter, g=g)
        g = ao["g"]
        mo, bo = OB.bio_step(ao["C"], cb, mo, bp, N)
        cls2, cb, mo, st = biofilm_step(cls, ao["C"], cb, mo, bp, fp, seeds[h])
        rec = dict(status="OK", fluid=fo["status"], iters_fluid=fo["iters"], ad=ao["status"],
                   iters_ad=ao["iters"], bio=bo, film=st)
        if not O.percolates(cls2):
            rec["status"] = "EINVAL"
            out.append(rec)
            break
        fl = f.reshape(f.shape[0], -1)
        for n in st["new_biofilm"]:
            fl[:, n] = 0.0
        cls = cls2
        out.append(rec)
    return out, cls, cb, mo

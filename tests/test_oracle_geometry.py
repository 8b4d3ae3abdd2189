"""Pins of the oracle's integer side: the SplitMix64 stream against its
published vectors, the seeded electrode generators against a naive pure-
Python generator written from the same specification, and the biofilm
layer, link masks, percolation, the flow domain and growth pick against
brute force or an independent library (scipy's connected-component labels).
"""
import math
import os

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
MASK = (1 << 64) - 1


class _SplitMix:
    """Textbook SplitMix64 on Python integers."""

    def __init__(self, seed):
        self.s = seed & MASK

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def integer(self, lo, hi):
        return lo + self.next() % (hi - lo + 1)


def test_splitmix64_published_vectors():
    rows = []
    with open(os.path.join(HERE, "golden", "splitmix64.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    for seed, idx, val in rows:
        assert int(O.splitmix64(seed, idx + 1)[idx]) == val


def _naive_discs(nx, ny, rmin, rmax, fs, overlap, seed):
    rng = _SplitMix(seed)
    cls = np.zeros((ny, nx), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    x0, x1 = nx // 4, 3 * nx // 4
    need = math.ceil(fs * ((x1 - x0) * (ny - 2)))
    discs, count = [], 0
    for _ in range(10 ** 6):
        if count >= need:
            break
        cx = rng.integer(x0, x1 - 1)
        cy = rng.integer(1, ny - 2)
        r = rng.integer(rmin, rmax)
        if not overlap and any((cx - a) ** 2 + (cy - b) ** 2 <= (r + c) ** 2 for a, b, c in discs):
            continue
        discs.append((cx, cy, r))
        for y in range(1, ny - 1):
            for x in range(x0, x1):
                if (x - cx) ** 2 + (y - cy) ** 2 <= r * r and cls[y, x] != O.SOLID:
                    cls[y, x] = O.SOLID
                    count += 1
    return cls, discs


@pytest.mark.parametrize("seed,overlap,fs", [(1, 0, 0.3), (2, 0, 0.4), (3, 1, 0.6), (4, 1, 0.2)])
def test_discs_match_naive_generator(seed, overlap, fs):
    st, cls, ach = O.geom_discs(96, 48, 3, 6, fs, overlap, seed)
    assert st == "OK"
    naive, discs = _naive_discs(96, 48, 3, 6, fs, overlap, seed)
    assert np.array_equal(cls, naive)
    area = 48 * 46
    assert (cls == O.SOLID).sum() >= math.ceil(fs * area)
    assert ach == (cls == O.SOLID).sum() / area
    assert (cls[:, :24] != O.SOLID).all() and (cls[:, 72:] != O.SOLID).all()
    if not overlap:   # strict separation: pairwise disjoint
        for i, (a, b, r) in enumerate(discs):
            for (c, d, s) in discs[i + 1:]:
                assert (a - c) ** 2 + (b - d) ** 2 > (r + s) ** 2


def _naive_fibres(nx, ny, nz, rmin, rmax, fs, seed):
    rng = _SplitMix(seed)
    cls = np.zeros((nz, ny, nx), np.uint8)
    cls[:, 0, :] = O.WALL
    cls[:, -1, :] = O.WALL
    cls[0] = O.WALL
    cls[-1] = O.WALL
    x0, x1 = nx // 4, 3 * nx // 4
    need = math.ceil(fs * ((x1 - x0) * (ny - 2) * (nz - 2)))
    count = 0
    z, y, x = np.meshgrid(np.arange(1, nz - 1), np.arange(1, ny - 1), np.arange(x0, x1),
                          indexing="ij")
    while count < need:
        q = (rng.integer(x0, x1 - 1), rng.integer(1, ny - 2), rng.integer(1, nz - 2))
        while True:
            d = (rng.integer(-4, 4), rng.integer(-4, 4), rng.integer(-4, 4))
            if d != (0, 0, 0):
                break
        r = rng.integer(rmin, rmax)
        px, py, pz = x - q[0], y - q[1], z - q[2]
        cx = py * d[2] - pz * d[1]
        cy = pz * d[0] - px * d[2]
        cz = px * d[1] - py * d[0]
        inside = cx * cx + cy * cy + cz * cz <= r * r * (d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        sub = cls[1:nz - 1, 1:ny - 1, x0:x1]
        count += int((inside & (sub != O.SOLID)).sum())
        sub[inside] = O.SOLID
    return cls


@pytest.mark.parametrize("seed", [3, 8])
def test_fibres_match_naive_generator(seed):
    st, cls, _ = O.geom_fibres(32, 16, 14, 2, 4, 0.2, seed)
    assert st == "OK"
    assert np.array_equal(cls, _naive_fibres(32, 16, 14, 2, 4, 0.2, seed))


def _nbrs(nz):
    if nz > 1:
        c, *_ = O.lattice_tables(O.D3Q19)
    else:
        c, *_ = O.lattice_tables(O.D2Q9)
    return c


def test_biofilm_layer_bruteforce():
    st, cls, _ = O.geom_discs(64, 32, 2, 5, 0.3, 0, 21)
    lay = O.biofilm_layer(cls)
    ny, nx = cls.shape
    c = _nbrs(1)
    for y in range(ny):
        for x in range(nx):
            solid_nb = any(0 <= x + dx < nx and 0 <= y + dy < ny and cls[y + dy, x + dx] == O.SOLID
                           for dx, dy, _ in c[1:])
            if cls[y, x] == O.FLUID:
                assert lay[y, x] == (O.BIOFILM if solid_nb else O.FLUID)
            else:
                assert lay[y, x] == cls[y, x]


@pytest.mark.parametrize("nz", [1, 6])
def test_links_bruteforce(nz):
    rng = np.random.default_rng(nz)
    shape = (nz, 7, 9) if nz > 1 else (7, 9)
    cls = rng.integers(0, 4, size=shape).astype(np.uint8)
    for which, lat in ((0, O.D3Q19 if nz > 1 else O.D2Q9), (1, O.D3Q7 if nz > 1 else O.D2Q5)):
        got = O.links(cls, which)
        c, *_ = O.lattice_tables(lat)
        blocked = (1, 2, 3) if which == 0 else (1, 2)
        c3 = cls.reshape((nz, 7, 9))
        g3 = got.reshape((nz, 7, 9))
        for z in range(nz):
            for y in range(7):
                for x in range(9):
                    want = 0
                    for i in range(1, len(c)):
                        sx, sy, sz = x - c[i, 0], y - c[i, 1], z - c[i, 2]
                        if 0 <= sx < 9 and 0 <= sy < 7 and 0 <= sz < nz and c3[sz, sy, sx] in blocked:
                            want |= 1 << i
                    assert int(g3[z, y, x]) == want


def test_percolation_handmade():
    cls = np.zeros((6, 10), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    assert O.percolates(cls)
    blk = cls.copy()
    blk[1:5, 5] = O.SOLID
    assert not O.percolates(blk)
    diag = cls.copy()            # a staircase leaves only diagonal links open
    for y in range(1, 5):
        diag[y, 3 + y] = O.SOLID
        diag[y, 2 + y] = O.BIOFILM if y > 1 else O.SOLID
    diag[4, 7] = O.FLUID
    diag[4, 6] = O.FLUID
    assert O.percolates(diag) == _bfs(diag)
    bio = cls.copy()
    bio[1:5, 4] = O.BIOFILM      # biofilm is impermeable to the fluid
    assert not O.percolates(bio)


def _bfs(cls):
    ny, nx = cls.shape
    c = _nbrs(1)
    seen = set((0, y) for y in range(ny) if cls[y, 0] == O.FLUID)
    todo = list(seen)
    while todo:
        x, y = todo.pop()
        if x == nx - 1:
            return True
        for dx, dy, _ in c[1:]:
            t = (x + dx, y + dy)
            if 0 <= t[0] < nx and 0 <= t[1] < ny and t not in seen and cls[t[1], t[0]] == O.FLUID:
                seen.add(t)
                todo.append(t)
    return False


def test_percolation_random_vs_bfs():
    rng = np.random.default_rng(2)
    for _ in range(40):
        cls = (rng.random((8, 12)) < 0.45).astype(np.uint8)
        cls[0] = O.WALL
        cls[-1] = O.WALL
        assert O.percolates(cls) == _bfs(cls)


def _domain_scipy(cls):
    """Flow domain from scipy's connected components: FLUID nodes in a
    component (8-connected in 2-D, 18-connected in 3-D -- the fluid
    lattice's neighbours) that holds a FLUID node of the last column."""
    from scipy import ndimage
    fl = cls == O.FLUID
    st = ndimage.generate_binary_structure(cls.ndim, cls.ndim if cls.ndim == 2 else 2)
    lab, _ = ndimage.label(fl, structure=st)
    keep = np.unique(lab[..., -1][fl[..., -1]])
    return np.isin(lab, keep) & fl


def test_flow_domain_handmade():
    cls = np.zeros((8, 12), np.uint8)
    cls[0] = O.WALL
    cls[-1] = O.WALL
    # a closed pore: a solid ring around two fluid nodes
    cls[2:6, 3:7] = O.SOLID
    cls[3:5, 4:6] = O.FLUID
    # an inlet-only pocket: a biofilm fence from the inlet column
    cls[1:4, 0] = O.FLUID
    cls[4, 0:3] = O.BIOFILM
    cls[1:4, 2] = O.BIOFILM
    # a dead end open to the main channel (stays in the domain)
    cls[6, 9] = O.FLUID
    cls[5, 8:11] = O.SOLID
    cls[5, 9] = O.FLUID
    dom = O.flow_domain(cls)
    assert not dom[3:5, 4:6].any()
    assert not dom[1:4, 0:2].any()
    assert dom[5, 9] and dom[6, 9]
    assert dom[6, 0] and dom[3, 11]
    assert np.array_equal(dom, _domain_scipy(cls))
    # a diagonal gap is a lattice link: the ring with one corner swapped
    # for a diagonal opening joins the pore to the channel
    cls2 = cls.copy()
    cls2[2, 3] = O.FLUID
    cls2[1, 2] = O.FLUID
    assert O.flow_domain(cls2)[3, 4]
    assert np.array_equal(O.flow_domain(cls2), _domain_scipy(cls2))


@pytest.mark.parametrize("nz", [1, 5])
def test_flow_domain_random_vs_scipy(nz):
    rng = np.random.default_rng(10 + nz)
    for _ in range(30):
        shape = (nz, 9, 14) if nz > 1 else (11, 16)
        cls = (rng.random(shape) < 0.45).astype(np.uint8) * rng.integers(1, 4, size=shape).astype(np.uint8)
        got = O.flow_domain(cls)
        assert np.array_equal(got, _domain_scipy(cls))
    for seed in range(1, 6):
        st, cls, _ = O.geom_discs(96, 48, 2, 5, 0.3, 0, seed)
        cls = O.biofilm_layer(cls)
        assert np.array_equal(O.flow_domain(cls), _domain_scipy(cls))


def test_percolation_is_domain_reaching_inlet():
    """Links are symmetric, so the inlet reaches the outlet iff an inlet
    node is in the flow domain (the library decides percolation that way)."""
    rng = np.random.default_rng(12)
    for _ in range(60):
        cls = (rng.random((9, 13)) < 0.45).astype(np.uint8)
        cls[0] = O.WALL
        cls[-1] = O.WALL
        assert O.percolates(cls) == bool(O.flow_domain(cls)[:, 0].any())


def _naive_pick(cls, C, xi):
    ny, nx = cls.shape
    c = _nbrs(1)
    cand = []
    for n in range(cls.size):
        x, y = n % nx, n // nx
        if cls[y, x] != O.FLUID or not (1 <= x <= nx - 2):
            continue
        if any(0 <= x + dx < nx and 0 <= y + dy < ny and cls[y + dy, x + dx] == O.BIOFILM
               for dx, dy, _ in c[1:]):
            cand.append(n)
    if not cand:
        return -1
    wts = [max(C[n], 0.0) for n in cand]
    W = 0.0
    for v in wts:
        W += v
    if W == 0.0:
        return cand[min(int(math.floor(xi * len(cand))), len(cand) - 1)]
    cum, last = 0.0, -1
    for n, v in zip(cand, wts):
        cum += v
        if v > 0:
            last = n
        if cum > xi * W:
            return n
    return last


def test_growth_pick_bruteforce():
    st, cls, _ = O.geom_discs(40, 20, 2, 4, 0.3, 0, 6)
    cls = O.biofilm_layer(cls)
    rng = np.random.default_rng(9)
    C = rng.random(cls.size) - 0.1
    for xi in list(rng.random(30)) + [0.0, 0.999999999]:
        assert O.growth_pick(cls, C, xi) == _naive_pick(cls, C, xi)
    Z = np.zeros(cls.size)
    assert O.growth_pick(cls, Z, 0.5) == _naive_pick(cls, Z, 0.5)

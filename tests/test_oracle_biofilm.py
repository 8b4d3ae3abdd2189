"""Pins of the agent-based biofilm oracle (Sec. 2.3, Table 1).

The checks rest on facts outside the oracle's own code: SplitMix64's
published outputs (through the oracle's C generator, itself pinned to test
vectors), the front as a morphological dilation computed by scipy,
conservation of biomass and mediator under spreading, and hand-made masks
whose outcome follows from the rules alone.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
import oracle.bioelec as OB
import oracle.biofilm as BF

FP = dict(k_ata=200, C_max=512.5, fr_spr=0.4, max_walk=10000, Y_bio=1.0)


def _bp(**over):
    p = OB.table1_params(1.0)
    p.update(over)
    return p


def _channel(nx, ny):
    cls = np.full((ny, nx), O.FLUID, np.uint8)
    cls[0, :] = cls[-1, :] = O.WALL
    return cls


def test_draws_follow_the_generator_across_blocks():
    d = BF.Draws(12345)
    got = [d._next() for _ in range(3000)]
    want = [int(x) for x in O.splitmix64(12345, 3000)]
    assert got == want


def test_front_is_the_dilated_electrode_and_attachment_picks_from_it():
    st, cls, _ = O.geom_discs(64, 32, 3, 5, 0.25, 0, 9)
    assert st == "OK"
    solid = cls == O.SOLID
    near = ndimage.binary_dilation(solid, structure=np.ones((3, 3), bool))
    front = near & (cls == O.FLUID)
    front[:, 0] = front[:, -1] = False
    nfront = int(front.sum())
    C = np.ones(cls.size)
    z = np.zeros(cls.size)
    for k_ata, seed in [(7, 1), (7, 2), (nfront + 5, 3)]:
        fp = dict(FP, k_ata=k_ata)
        c2, cb, mo, s = BF.biofilm_step(cls, C, z, z, _bp(q_max=0.0), fp, seed)
        got = (c2 == O.BIOFILM) & (cls != O.BIOFILM)
        assert s["attached"] == min(k_ata, nfront) == int(got.sum())
        assert np.all(front[got])
        assert np.all(cb.reshape(cls.shape)[got] == 450.0)
        assert np.all(mo.reshape(cls.shape)[got] == 0.05)
    # different seeds draw different cells
    a = BF.biofilm_step(cls, C, z, z, _bp(q_max=0.0), dict(FP, k_ata=7), 1)[0]
    b = BF.biofilm_step(cls, C, z, z, _bp(q_max=0.0), dict(FP, k_ata=7), 2)[0]
    assert not np.array_equal(a, b)


def test_growth_multiplies_by_one_plus_rate_times_interval():
    """No attachment, nothing above C_max: each cell's biomass is multiplied
    by 1 + Y_bio q dt, q at half saturation of both factors = q_max / 4."""
    cls = _channel(12, 8)
    cls[3:5, 4:7] = O.BIOFILM
    bp = _bp()
    C = np.full(cls.size, bp["K_s"] / bp["c_scale"])
    cb = np.where(cls.reshape(-1) == O.BIOFILM, 300.0, 0.0)
    mo = np.where(cb > 0, bp["K_Mox"], 0.0)
    for Y in (1.0, 0.3):
        _, cb2, mo2, s = BF.biofilm_step(cls, C, cb, mo, bp, dict(FP, k_ata=0, Y_bio=Y), 5)
        grow = 1.0 + Y * (bp["q_max"] / 4.0) / 24.0
        assert np.allclose(cb2[cb > 0], 300.0 * grow, rtol=1e-15)
        assert np.array_equal(mo2, mo) and s["spread"] == 0


def _totals(cb, mo):
    return float(np.sum(cb)), float(np.sum(cb * mo))


def test_direct_spreading_moves_a_fraction_to_one_free_neighbour():
    cls = _channel(12, 9)
    n = 6 + 12 * 4
    cls.reshape(-1)[n] = O.BIOFILM
    cb = np.zeros(cls.size)
    mo = np.zeros(cls.size)
    cb[n], mo[n] = 600.0, 0.03
    c2, cb2, mo2, s = BF.biofilm_step(cls, np.ones(cls.size), cb, mo, _bp(q_max=0.0),
                                      dict(FP, k_ata=0), 7)
    new = np.flatnonzero((c2.reshape(-1) == O.BIOFILM) & (cls.reshape(-1) != O.BIOFILM))
    assert s["spread"] == 1 and s["walks"] == 0 and len(new) == 1
    m = int(new[0])
    assert max(abs(m % 12 - n % 12), abs(m // 12 - n // 12)) == 1
    assert cb2[m] == 0.4 * 600.0 and cb2[n] == 600.0 - 0.4 * 600.0 and mo2[m] == 0.03
    assert _totals(cb2, mo2) == pytest.approx(_totals(cb, mo), rel=1e-15)


def test_enclosed_cell_spreads_by_a_random_walk():
    """A full cell inside a 5 x 5 biofilm block has no free neighbour: the
    walk reaches the block's edge, biomass shifts outward along a simple
    path, and exactly one free cell next to the block becomes BIOFILM."""
    cls = _channel(20, 13)
    cls[4:9, 8:13] = O.BIOFILM
    flat = cls.reshape(-1)
    rng = np.random.default_rng(3)
    cb = np.where(flat == O.BIOFILM, rng.uniform(100, 400, flat.size), 0.0)
    mo = np.where(cb > 0, rng.uniform(0, 0.05, flat.size), 0.0)
    centre = 10 + 20 * 6
    cb[centre] = 700.0
    for seed in range(6):
        c2, cb2, mo2, s = BF.biofilm_step(cls, np.ones(flat.size), cb, mo, _bp(q_max=0.0),
                                          dict(FP, k_ata=0), seed)
        new = np.flatnonzero((c2.reshape(-1) == O.BIOFILM) & (flat != O.BIOFILM))
        assert s["spread"] == 1 and s["walks"] == 1 and s["abandoned"] == 0
        assert len(new) == 1
        ring = ndimage.binary_dilation(cls == O.BIOFILM, structure=np.ones((3, 3), bool))
        assert ring.reshape(-1)[new[0]]
        assert cb2[centre] == 700.0 - 0.4 * 700.0
        assert _totals(cb2, mo2) == pytest.approx(_totals(cb, mo), rel=1e-14)
        # values are only moved: the multiset of (biomass, mediator) pairs
        # is the old one with 700 split into 420 and 280
        old = sorted(zip(cb[cb > 0], mo[cb > 0]))
        old.remove((700.0, mo[centre]))
        old += [(420.0, mo[centre]), (280.0, mo[centre])]
        assert sorted(zip(cb2[cb2 > 0], mo2[cb2 > 0])) == sorted(old)


def test_walk_without_a_free_cell_gives_up():
    cls = np.full((9, 9), O.SOLID, np.uint8)
    cls[0, :] = cls[-1, :] = O.WALL
    cls[3:6, 3:6] = O.BIOFILM
    flat = cls.reshape(-1)
    cb = np.where(flat == O.BIOFILM, 300.0, 0.0)
    cb[4 + 9 * 4] = 900.0
    mo = np.where(cb > 0, 0.01, 0.0)
    c2, cb2, mo2, s = BF.biofilm_step(cls, np.ones(flat.size), cb, mo, _bp(q_max=0.0),
                                      dict(FP, k_ata=0, max_walk=500), 1)
    assert s["abandoned"] == 1 and s["spread"] == 0
    assert np.array_equal(c2, cls) and np.array_equal(cb2, cb)


def test_spreading_conserves_biomass_and_mediator_on_a_grown_electrode():
    st, cls, _ = O.geom_discs(64, 32, 3, 5, 0.25, 0, 4)
    cls = O.biofilm_layer(cls)
    flat = cls.reshape(-1)
    rng = np.random.default_rng(8)
    cb = np.where(flat == O.BIOFILM, rng.uniform(300, 900, flat.size), 0.0)
    mo = np.where(cb > 0, rng.uniform(0, 0.05, flat.size), 0.0)
    c2, cb2, mo2, s = BF.biofilm_step(cls, np.ones(flat.size), cb, mo, _bp(q_max=0.0),
                                      dict(FP, k_ata=0), 11)
    assert s["spread"] > 10
    assert _totals(cb2, mo2) == pytest.approx(_totals(cb, mo), rel=1e-13)
    assert int((c2 == O.BIOFILM).sum()) == int((cls == O.BIOFILM).sum()) + s["spread"]
    # nothing lands in the inlet or outlet column
    assert not np.any(c2[:, 0] == O.BIOFILM) and not np.any(c2[:, -1] == O.BIOFILM)


def test_long_walks_move_values_along_a_simple_path():
    """A 9 x 9 block: walks from its centre revisit cells on their way out,
    and only a loop-erased (simple) path moves each value exactly once."""
    cls = _channel(30, 17)
    cls[4:13, 10:19] = O.BIOFILM
    flat = cls.reshape(-1)
    rng = np.random.default_rng(5)
    cb = np.where(flat == O.BIOFILM, rng.uniform(100, 400, flat.size), 0.0)
    mo = np.where(cb > 0, rng.uniform(0, 0.05, flat.size), 0.0)
    centre = 14 + 30 * 8
    cb[centre] = 800.0
    for seed in range(12):
        c2, cb2, mo2, s = BF.biofilm_step(cls, np.ones(flat.size), cb, mo, _bp(q_max=0.0),
                                          dict(FP, k_ata=0), 100 + seed)
        assert s["walks"] == 1 and s["spread"] == 1
        old = sorted(zip(cb[cb > 0], mo[cb > 0]))
        old.remove((800.0, mo[centre]))
        old += [(480.0, mo[centre]), (320.0, mo[centre])]
        assert sorted(zip(cb2[cb2 > 0], mo2[cb2 > 0])) == sorted(old), seed


def test_attachment_draws_every_front_cell():
    """One cell per interval: over many seeds each front cell is drawn."""
    cls = _channel(16, 10)
    cls[4:6, 7:9] = O.SOLID
    front = ndimage.binary_dilation(cls == O.SOLID, structure=np.ones((3, 3), bool)) & (cls == O.FLUID)
    z = np.zeros(cls.size)
    seen = set()
    for seed in range(600):
        c2 = BF.biofilm_step(cls, np.ones(cls.size), z, z, _bp(q_max=0.0), dict(FP, k_ata=1), seed)[0]
        seen |= set(np.flatnonzero((c2 == O.BIOFILM).reshape(-1)).tolist())
    assert seen == set(np.flatnonzero(front.reshape(-1)).tolist())


def test_no_biomass_enters_the_inlet_or_outlet_column():
    """Electrode cells next to the boundary columns: their front there is
    not attachable, and a full cell beside the outlet column spreads
    elsewhere."""
    cls = _channel(10, 8)
    cls[2:6, 1] = O.SOLID
    cls[2:6, 8] = O.BIOFILM
    z = np.zeros(cls.size)
    c2, _, _, s = BF.biofilm_step(cls, np.ones(cls.size), z, z, _bp(q_max=0.0),
                                  dict(FP, k_ata=100), 3)
    assert s["attached"] > 0
    assert not np.any(c2[:, 0] == O.BIOFILM) and not np.any(c2[:, -1] == O.BIOFILM)
    flat = cls.reshape(-1)
    cb = np.where(flat == O.BIOFILM, 900.0, 0.0)
    mo = np.where(cb > 0, 0.02, 0.0)
    for seed in range(20):
        c3, _, _, s = BF.biofilm_step(cls, np.ones(cls.size), cb, mo, _bp(q_max=0.0),
                                      dict(FP, k_ata=0), seed)
        assert s["spread"] == 4
        assert not np.any(c3[:, -1] == O.BIOFILM)

"""Served form on the GPU: continuous batching of 2-D steady solves.

What is checked, through the C ABI:
  * a request's result equals that of the single-solve path with the same
    storage (iterations, statuses and the FP64 fluxes of the final states
    exactly; fields to the output rounding), for a mix larger than the pool
    so that admission by footprint, slot reuse and queueing take part;
  * a request's result is bit-identical alone and inside a mix;
  * the captured graph and direct launches agree bit for bit;
  * a served request agrees with the FP64 oracle run for the same number of
    steps (1e-4 relative L2 for the FP32 forms);
  * FP16-storage served results stay within 5e-3 relative L2 of the plain
    FP32 single solve run for the same numbers of steps;
  * rejections (bad parameters, a pool too small, a medium that does not
    percolate) and max_iter endings;
  * the solo lane: a request routed to the single-domain solver returns
    what the batch returns, bit for bit; an escalated request returns the
    FP32-shifted single solve, with the batched attempt's status and counts.
"""
import numpy as np
import pytest

import oracle as O
from helpers import rel_l2

pytestmark = pytest.mark.gpu

FP32, FP32S, FP16S = 0, 1, 2

# (nx, ny, solid share, tau, u_in, seed): small domains that converge in
# 5e3 - 8e4 steps; 66 x 33 has ragged tiles in x and y
DIVERGING = (96, 48, 0.4, 0.6, 0.02, 12)  # |u| passes 0.3 in a narrow pore
MIX = [
    (64, 32, 0.3, 0.8, 0.01, 11),
    (96, 48, 0.4, 0.7, 0.01, 12),
    (66, 33, 0.2, 1.0, 0.015, 13),
    (128, 64, 0.3, 0.7, 0.01, 14),
    (80, 40, 0.45, 0.9, 0.005, 19),
]
D_SUB, K_SINK = 0.1 / 3.0, 1e-3


@pytest.fixture(scope="module")
def srv_env(gpu_lib):
    lbm = gpu_lib
    ctx = lbm.lbm_ctx_create(0)
    yield lbm, ctx
    lbm.lbm_ctx_destroy(ctx)


def _mask(lbm, nx, ny, solid, seed, layer=1):
    st, cls, _ = lbm.lbm_geom_discs(nx, ny, 3, 6, solid, 1, seed)
    assert st == 0
    return lbm.lbm_biofilm_layer(cls) if layer else cls


def _request(lbm, spec, user=0, tol=1e-6, max_iter=400000, **kw):
    nx, ny, solid, tau, u_in, seed = spec
    return lbm.make_request(nx, ny, r_min=3, r_max=6, solid_frac=solid, overlap=1, seed=seed,
                            layer=1, tau=tau, u_in=u_in, D=D_SUB, c_in=1.0, k_sink=K_SINK,
                            tol=tol, max_iter=max_iter, user=user, **kw)


def _serve(lbm, ctx, specs, storage, pool=None, slots=8, order=None, **cfgkw):
    """Submit specs (in `order`) to a fresh server; results by spec index."""
    need = [lbm.lbm_server_footprint(s[0], s[1], storage) for s in specs]
    cfg = lbm.make_server_cfg(pool or 4 * sum(need), max_slots=slots, storage=storage, **cfgkw)
    srv = lbm.lbm_server_create(ctx, cfg)
    try:
        tickets = {}
        for i in (order or range(len(specs))):
            st, t = lbm.lbm_server_submit(srv, _request(lbm, specs[i], user=i))
            assert st == 0, lbm.lbm_server_error(srv)
            tickets[t] = i
        assert lbm.lbm_server_drain(srv, 300.0) == 0
        res = {}
        while len(res) < len(specs):
            for r in lbm.lbm_server_poll(srv, 16, 1.0):
                res[tickets[r["ticket"]]] = r
        stats = lbm.lbm_server_stats(srv)
    finally:
        lbm.lbm_server_destroy(srv)
    return res, stats, need


def _single(lbm, ctx, spec, storage, tol=1e-6, max_iter=400000, check_every=0):
    nx, ny, solid, tau, u_in, seed = spec
    cls = _mask(lbm, nx, ny, solid, seed)
    p = lbm.make_params(tau=tau, u_in=u_in, D=D_SUB, c_in=1.0, k_sink=K_SINK, storage=storage,
                        check_every=check_every)
    s = lbm.lbm_solver_create(ctx, cls, p)
    try:
        sf, fi = lbm.lbm_solver_fluid(s, tol, max_iter)
        sa, ai = (None, None) if sf == lbm.LBM_EDIVERGED else lbm.lbm_solver_ad(s, tol, max_iter)
        U = lbm.lbm_solver_get(s, lbm.LBM_FIELD_U, (nx, ny, 1))
        C = None if sa is None else lbm.lbm_solver_get(s, lbm.LBM_FIELD_C, (nx, ny, 1))
    finally:
        lbm.lbm_solver_destroy(s)
    return dict(cls=cls, sf=sf, sa=sa, fi=fi, ai=ai, U=U, C=C)


@pytest.mark.parametrize("storage,K", [(FP32, 100), (FP32S, 100), (FP32S, 40), (FP16S, 100)],
                         ids=["fp32", "fp32s", "fp32s-K40", "fp16s"])
def test_server_matches_single_solve(srv_env, storage, K):
    """FP32 forms are served over 64 x 16 tiles, four steps per launch (a
    chunk of K = 100 opens with two two-step launches, K = 40 has four-step
    launches only); FP16 over 64 x 4 tiles, two steps per launch.  The
    single solves of these small domains take 64 x 4 tiles and two steps."""
    lbm, ctx = srv_env
    specs = MIX[:4]
    need = [lbm.lbm_server_footprint(s[0], s[1], storage) for s in specs]
    pool = max(need) + sorted(need)[-2] + 4096  # at most two largest at once
    print("server vs single solve, storage", storage, "K", K, "pool", pool, flush=True)
    res, stats, _ = _serve(lbm, ctx, specs, storage, pool=pool, slots=3, check_every=K)
    assert sum(need) > pool and stats["pool_peak"] <= pool
    assert stats["finished"] == len(specs) and stats["rejected"] == 0
    for i, spec in enumerate(specs):
        r, s = res[i], _single(lbm, ctx, spec, storage, check_every=K)
        assert r["status_fluid"] == s["sf"] and r["status_ad"] == s["sa"], (i, r, s["sf"], s["sa"])
        assert r["iters_fluid"] == s["fi"]["iters"] and r["iters_ad"] == s["ai"]["iters"]
        assert r["active_fluid"] == s["fi"]["active_nodes"] and r["active_ad"] == s["ai"]["active_nodes"]
        # FP64 sums over the final stored states: equal only if the states are
        assert r["flux"][0] == s["fi"]["flux_in"] and r["flux"][1] == s["fi"]["flux_out"]
        assert r["flux"][2] == s["ai"]["flux_in"] and r["flux"][3] == s["ai"]["flux_out"]
        assert r["flux"][4] == s["ai"]["sink_total"]
        # fields: the server returns FP32 exports, the solver FP64 ones
        assert np.abs(r["u"] - s["U"]).max() <= 1e-6 * max(np.abs(s["U"]).max(), 1e-30)
        assert np.abs(r["c"] - s["C"]).max() <= 1e-6
        assert r["t_submit"] <= r["t_admit"] <= r["t_finish"]


@pytest.mark.parametrize("storage", [FP32S, FP16S], ids=["fp32s", "fp16s"])
def test_server_alone_equals_in_mix(srv_env, storage):
    lbm, ctx = srv_env
    x = MIX[2]
    alone, _, _ = _serve(lbm, ctx, [x], storage)
    mix = [MIX[0], MIX[1], x, MIX[3], MIX[4]]
    print("alone vs mix, storage", storage, flush=True)
    inmix, _, _ = _serve(lbm, ctx, mix, storage, slots=4, order=[3, 0, 2, 4, 1])
    a, b = alone[0], inmix[2]
    assert a["iters_fluid"] == b["iters_fluid"] and a["iters_ad"] == b["iters_ad"]
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["c"], b["c"])
    assert np.array_equal(a["flux"], b["flux"])


def test_server_graph_equals_direct_launch(srv_env):
    lbm, ctx = srv_env
    specs = [MIX[0], MIX[2]]
    g, _, _ = _serve(lbm, ctx, specs, FP32S)
    d, _, _ = _serve(lbm, ctx, specs, FP32S, direct_launch=1, inflight=1)
    for i in range(len(specs)):
        assert g[i]["iters_fluid"] == d[i]["iters_fluid"] and g[i]["iters_ad"] == d[i]["iters_ad"]
        assert np.array_equal(g[i]["u"], d[i]["u"]) and np.array_equal(g[i]["c"], d[i]["c"])


def _burst(lbm, ctx, specs, prep_threads):
    """Submit every spec at once (tol 0, 600 + 600 steps each) and return
    the results by spec index; every ticket must come back exactly once."""
    need = [lbm.lbm_server_footprint(s[0], s[1], FP32S) for s in specs]
    cfg = lbm.make_server_cfg(sum(sorted(need)[-6:]), max_slots=6, storage=FP32S, check_every=100,
                              prep_threads=prep_threads, solo_nodes=-1)
    srv = lbm.lbm_server_create(ctx, cfg)
    try:
        tickets = {}
        for i, spec in enumerate(specs):
            st, t = lbm.lbm_server_submit(srv, _request(lbm, spec, user=i, tol=0.0, max_iter=600))
            assert st == 0, lbm.lbm_server_error(srv)
            tickets[t] = i
        assert lbm.lbm_server_drain(srv, 120.0) == 0, lbm.lbm_server_stats(srv)
        res = {}
        for _ in range(200):
            for r in lbm.lbm_server_poll(srv, 16, 0.1):
                assert tickets[r["ticket"]] not in res, "a request came back twice"
                res[tickets[r["ticket"]]] = r
            if len(res) == len(specs):
                break
        stats = lbm.lbm_server_stats(srv)
    finally:
        lbm.lbm_server_destroy(srv)
    assert len(res) == len(specs) and stats["finished"] == len(specs) and stats["pool_used"] == 0
    return res


def test_server_burst_prepared_out_of_order(srv_env):
    """Regression test of admission: preparation threads finish out of
    ticket order (large masks take longer than small ones), and a request
    prepared while the worker admitted a later ticket was once dropped (the
    drain never returned) while the admitted one ran twice.  A burst of
    mixed sizes is served with four preparation threads and again with one;
    every request comes back once, with the same steps and fields."""
    lbm, ctx = srv_env
    rng = np.random.default_rng(31)
    specs = []
    for i in range(36):
        nx = int(rng.choice([48, 64, 96, 160, 224]))
        specs.append((nx, nx // 2, 0.3, 0.8, 0.01, 100 + i))
    print("burst of", len(specs), "requests, 4 then 1 preparation threads", flush=True)
    a = _burst(lbm, ctx, specs, 4)
    b = _burst(lbm, ctx, specs, 1)
    rejected = 0
    for i in range(len(specs)):
        ra, rb = a[i], b[i]
        nx, ny, solid, _, _, seed = specs[i]
        if not lbm.lbm_percolates(_mask(lbm, nx, ny, solid, seed)):
            assert ra["status"] == rb["status"] == lbm.LBM_EINVAL
            rejected += 1
            continue
        assert ra["status"] == rb["status"] == lbm.LBM_NOT_CONVERGED, (i, ra["status"], rb["status"])
        assert ra["iters_fluid"] == rb["iters_fluid"] == 600 and ra["iters_ad"] == rb["iters_ad"] == 600
        assert np.array_equal(ra["u"], rb["u"]) and np.array_equal(ra["c"], rb["c"])
        assert np.array_equal(ra["flux"], rb["flux"])
    assert 0 < rejected < len(specs) // 4  # media that do not percolate take the rejection path


def test_served_request_matches_oracle(srv_env):
    lbm, ctx = srv_env
    spec = MIX[0]
    nx, ny, solid, tau, u_in, seed = spec
    res, _, _ = _serve(lbm, ctx, [spec], FP32S)
    r = res[0]
    assert r["status"] == 0, r
    # the oracle builds the same mask and runs the same step counts
    st, cls, _ = O.geom_discs(nx, ny, 3, 6, solid, 1, seed)
    assert st == "OK"
    cls = O.biofilm_layer(cls)
    f, _, _ = O.fluid_run(cls, O.fluid_init(cls), tau, u_in, r["iters_fluid"])
    U, _ = O.fluid_moments(cls, f)
    g, _ = O.ad_run(cls, O.ad_init(cls, U, 1.0), U, D_SUB, 1.0, K_SINK, r["iters_ad"])
    C = O.ad_moment(cls, g, K_SINK)
    flat = cls.reshape(-1)
    fl = flat == 0
    act = (flat == 0) | (flat == 3)
    assert rel_l2(r["u"], U.reshape(2, -1), fl) < 1e-4
    assert rel_l2(r["c"], C.reshape(-1), act) < 1e-4


def test_served_fp16_within_5e_3_of_plain_fp32(srv_env):
    """Precision of the served FP16 form: the plain FP32 single solve run for
    the same numbers of steps (tol 0, max_iter = the served counts), so that
    only the storage differs.  (At a tolerance the two forms stop at
    different points of slow transients: FP16 reaches a stochastic-rounding
    floor of the per-node residual first.)  The shift removes w_i * 1, not
    the pressure drop: with u_in = 0.005 and a density excess ~0.08 at the
    inlet (MIX[4]) the FP16 ulp of the stored values is ~1e-5 against
    velocities ~5e-3, and the momentum noise that stochastic rounding injects
    decays only viscously -- ~2% velocity error; these cases use u_in >= 0.01."""
    lbm, ctx = srv_env
    specs = [MIX[0], MIX[3]]
    res, _, _ = _serve(lbm, ctx, specs, FP16S)
    for i, spec in enumerate(specs):
        nx, ny, solid, tau, u_in, seed = spec
        r = res[i]
        cls = _mask(lbm, nx, ny, solid, seed)
        p = lbm.make_params(tau=tau, u_in=u_in, D=D_SUB, c_in=1.0, k_sink=K_SINK, storage=FP32,
                            stall_checks=-1)
        s = lbm.lbm_solver_create(ctx, cls, p)
        try:
            sf, fi = lbm.lbm_solver_fluid(s, 0.0, r["iters_fluid"])
            sa, ai = lbm.lbm_solver_ad(s, 0.0, r["iters_ad"])
            U = lbm.lbm_solver_get(s, lbm.LBM_FIELD_U, (nx, ny, 1))
            C = lbm.lbm_solver_get(s, lbm.LBM_FIELD_C, (nx, ny, 1))
        finally:
            lbm.lbm_solver_destroy(s)
        assert fi["iters"] == r["iters_fluid"] and ai["iters"] == r["iters_ad"]
        flat = cls.reshape(-1)
        fl = flat == 0
        act = (flat == 0) | (flat == 3)
        eu = rel_l2(r["u"], U, fl)
        ec = rel_l2(r["c"], C, act)
        print("fp16 served vs fp32 single", i, r["status"], r["iters_fluid"], r["iters_ad"], eu, ec,
              flush=True)
        assert eu < 5e-3 and ec < 5e-3


def test_server_max_iter_and_rejections(srv_env):
    lbm, ctx = srv_env
    spec = MIX[3]
    cfg = lbm.make_server_cfg(4 << 20, max_slots=2, storage=FP32S, solo_nodes=-1)
    srv = lbm.lbm_server_create(ctx, cfg)
    try:
        # parameters checked at submission
        bad = _request(lbm, spec)
        bad[0].tau = 0.5
        assert lbm.lbm_server_submit(srv, bad)[0] == lbm.LBM_EINVAL
        assert "tau" in lbm.lbm_server_error(srv)
        big = lbm.make_request(2048, 1024)
        assert lbm.lbm_server_submit(srv, big)[0] == lbm.LBM_EINVAL
        # a blocked medium: rejected when prepared, reported as a result
        cls = np.zeros((32, 64), np.uint8)
        cls[0, :] = cls[-1, :] = lbm.LBM_WALL
        cls[1:-1, 30] = lbm.LBM_SOLID
        st, t_block = lbm.lbm_server_submit(srv, lbm.make_request(64, 32, cls=cls))
        assert st == 0
        # max_iter 250 is rounded up to the check cadence (300 steps)
        st, t_cap = lbm.lbm_server_submit(srv, _request(lbm, spec, max_iter=250))
        assert st == 0
        st, t_div = lbm.lbm_server_submit(srv, _request(lbm, DIVERGING))
        assert st == 0
        assert lbm.lbm_server_drain(srv, 120.0) == 0
        got = {r["ticket"]: r for r in lbm.lbm_server_poll(srv, 8, 1.0)}
        stats = lbm.lbm_server_stats(srv)
    finally:
        lbm.lbm_server_destroy(srv)
    assert got[t_block]["status"] == lbm.LBM_EINVAL and "connect" in got[t_block]["message"]
    r = got[t_cap]
    assert r["status"] == lbm.LBM_NOT_CONVERGED
    assert r["iters_fluid"] == 300 and r["iters_ad"] == 300
    assert stats["rejected"] == 1 and stats["finished"] == 3
    s = _single(lbm, ctx, spec, FP32S, max_iter=300)
    assert s["sf"] == lbm.LBM_NOT_CONVERGED and s["fi"]["iters"] == 300
    assert r["flux"][0] == s["fi"]["flux_in"] and r["flux"][4] == s["ai"]["sink_total"]
    # a diverging fluid solve ends the request: no substrate solve
    r = got[t_div]
    s = _single(lbm, ctx, DIVERGING, FP32S)
    assert r["status"] == r["status_fluid"] == s["sf"] == lbm.LBM_EDIVERGED
    assert r["iters_fluid"] == s["fi"]["iters"] and r["iters_ad"] == 0
    assert not np.any(r["c"]) and r["flux"][0] == s["fi"]["flux_in"]


@pytest.mark.parametrize("storage", [FP32S, FP16S], ids=["fp32s", "fp16s"])
@pytest.mark.parametrize("spec", [(1024, 512, 0.3, 0.8, 0.01, 21), (512, 256, 0.3, 0.8, 0.01, 22)],
                         ids=["1024x512-wide", "512x256-middle"])
def test_server_matches_wide_single_solve(srv_env, spec, storage):
    """Large requests, whose single solves take other launch forms than the
    server.  Shifted FP32: served four steps per launch over 64 x 16 tiles;
    the single solve takes four-step launches over 64 x 16 tiles on 1024 x
    512 and over 64 x 8 tiles on 512 x 256.  FP16: served by paired
    launches over 64 x 4 tiles; the single solve fuses pairs of them into
    four-step launches over 64 x 16 or 64 x 8 tiles, rounding in LDS as the
    paired store would.  All make the same multiply-add choices (fused per source
    expression), so the states stay equal bit for bit: 400 steps of each
    solver (checks, and FP16's reference moves, every 100), then statuses,
    counts and the FP64 fluxes of the final states."""
    lbm, ctx = srv_env
    need = lbm.lbm_server_footprint(spec[0], spec[1], storage)
    cfg = lbm.make_server_cfg(need + 4096, max_slots=1, storage=storage, check_every=100, solo_nodes=-1)
    srv = lbm.lbm_server_create(ctx, cfg)
    print("server vs single solve %dx%d storage %d" % (spec[0], spec[1], storage), flush=True)
    try:
        st, t = lbm.lbm_server_submit(srv, _request(lbm, spec, max_iter=400))
        assert st == 0, lbm.lbm_server_error(srv)
        assert lbm.lbm_server_drain(srv, 120.0) == 0
        r = lbm.lbm_server_poll(srv, 1, 1.0)[0]
    finally:
        lbm.lbm_server_destroy(srv)
    s = _single(lbm, ctx, spec, storage, max_iter=400, check_every=100)
    assert r["status_fluid"] == s["sf"] == lbm.LBM_NOT_CONVERGED
    assert r["iters_fluid"] == s["fi"]["iters"] == 400 and r["iters_ad"] == s["ai"]["iters"] == 400
    assert r["flux"][0] == s["fi"]["flux_in"] and r["flux"][1] == s["fi"]["flux_out"]
    assert r["flux"][2] == s["ai"]["flux_in"] and r["flux"][3] == s["ai"]["flux_out"]
    assert r["flux"][4] == s["ai"]["sink_total"]


@pytest.mark.parametrize("storage", [FP32S, FP16S], ids=["fp32s", "fp16s"])
def test_solo_lane_equals_batch(srv_env, storage):
    """A request of at least solo_nodes nodes is solved by the single-domain
    solver on the solo lane (wider multi-step launches, its own stream, next
    to the batch): statuses, counts, fluxes and the FP32 fields equal the
    batch's bit for bit."""
    lbm, ctx = srv_env
    specs = [MIX[0], MIX[3]]  # 2,048 and 8,192 nodes
    print("solo lane vs batch, storage", storage, flush=True)
    batch, bstats, _ = _serve(lbm, ctx, specs, storage, solo_nodes=-1)
    solo, sstats, _ = _serve(lbm, ctx, specs, storage, solo_nodes=4096)
    assert bstats["solo"] == 0 and sstats["solo"] == 1 and sstats["escalated"] == 0
    assert [batch[i]["lane"] for i in (0, 1)] == [lbm.LBM_LANE_BATCH] * 2
    assert [solo[i]["lane"] for i in (0, 1)] == [lbm.LBM_LANE_BATCH, lbm.LBM_LANE_SOLO]
    for i in (0, 1):
        a, b = batch[i], solo[i]
        for k in ("status", "status_fluid", "status_ad", "iters_fluid", "iters_ad", "active_fluid",
                  "active_ad"):
            assert a[k] == b[k], (i, k, a[k], b[k])
        assert np.array_equal(a["flux"], b["flux"])
        assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["c"], b["c"])
        assert b["t_submit"] <= b["t_admit"] <= b["t_finish"]


@pytest.mark.parametrize("solo", [0, 1], ids=["batched", "solo"])
def test_escalation_resolves_in_fp32_shifted(srv_env, solo):
    """FP16 server with escalation: a request whose FP16 solves (batched, or
    on a solo lane) end NOT_CONVERGED (max_iter 200) is solved again from
    rest in FP32-shifted storage -- the result is that single solve's,
    marked escalated, with the first attempt's status and step counts; a
    request that ends OK keeps its FP16 result."""
    lbm, ctx = srv_env
    a_spec, b_spec = MIX[0], MIX[2]
    need = sum(lbm.lbm_server_footprint(s[0], s[1], FP16S) for s in (a_spec, b_spec))
    cfg = lbm.make_server_cfg(4 * need, max_slots=4, storage=FP16S, check_every=100, escalate=1,
                              solo_nodes=solo or -1)
    srv = lbm.lbm_server_create(ctx, cfg)
    print("escalation", flush=True)
    try:
        st, ta = lbm.lbm_server_submit(srv, _request(lbm, a_spec, max_iter=200))
        assert st == 0
        st, tb = lbm.lbm_server_submit(srv, _request(lbm, b_spec, tol=1e-3))
        assert st == 0
        assert lbm.lbm_server_drain(srv, 120.0) == 0
        got = {r["ticket"]: r for r in lbm.lbm_server_poll(srv, 4, 1.0)}
        stats = lbm.lbm_server_stats(srv)
    finally:
        lbm.lbm_server_destroy(srv)
    assert stats["finished"] == 2 and stats["solo"] == 1 + solo and stats["escalated"] == 1
    ra, rb = got[ta], got[tb]
    assert ra["lane"] == lbm.LBM_LANE_ESCALATED
    assert ra["first_status"] == lbm.LBM_NOT_CONVERGED
    assert ra["first_iters_fluid"] == 200 and ra["first_iters_ad"] == 200
    s = _single(lbm, ctx, a_spec, FP32S, max_iter=200)
    assert ra["status_fluid"] == s["sf"] == lbm.LBM_NOT_CONVERGED
    assert ra["iters_fluid"] == s["fi"]["iters"] == 200 and ra["iters_ad"] == s["ai"]["iters"] == 200
    assert ra["flux"][0] == s["fi"]["flux_in"] and ra["flux"][1] == s["fi"]["flux_out"]
    assert ra["flux"][2] == s["ai"]["flux_in"] and ra["flux"][4] == s["ai"]["sink_total"]
    assert np.abs(ra["u"] - s["U"]).max() <= 1e-6 * max(np.abs(s["U"]).max(), 1e-30)
    assert np.abs(ra["c"] - s["C"]).max() <= 1e-6
    assert rb["lane"] == (lbm.LBM_LANE_SOLO if solo else lbm.LBM_LANE_BATCH) and rb["status"] == lbm.LBM_OK
    assert rb["first_status"] == 0 and rb["first_iters_fluid"] == 0
    s = _single(lbm, ctx, b_spec, FP16S, tol=1e-3, check_every=100)
    assert rb["iters_fluid"] == s["fi"]["iters"] and rb["iters_ad"] == s["ai"]["iters"]
    assert rb["flux"][0] == s["fi"]["flux_in"] and rb["flux"][4] == s["ai"]["sink_total"]


def test_concurrent_solo_lanes_equal_batch(srv_env):
    """Four solo lanes solving five requests at once, each lane a solver on
    its own stream and host thread: every result equals the batch's bit for
    bit.  (Uploads that ran on the null stream were not ordered against a
    lane's non-blocking stream: under concurrency a solve could start on
    descriptors still landing.)"""
    lbm, ctx = srv_env
    specs = MIX[:5]
    batch, _, _ = _serve(lbm, ctx, specs, FP32S, solo_nodes=-1)
    solo, stats, _ = _serve(lbm, ctx, specs, FP32S, solo_nodes=1, solo_lanes=4)
    assert stats["solo"] == len(specs)
    for i in range(len(specs)):
        a, b = batch[i], solo[i]
        assert b["lane"] == lbm.LBM_LANE_SOLO
        assert (a["status"], a["iters_fluid"], a["iters_ad"]) == (b["status"], b["iters_fluid"], b["iters_ad"]), i
        assert np.array_equal(a["flux"], b["flux"])
        assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["c"], b["c"])

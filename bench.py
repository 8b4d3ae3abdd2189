"""Benchmark: coupled steady solves of the anode-compartment LBM on one GPU.

One step = one pass of the hot path over the workload: fluid steady solve
from rest (D2Q9 / D3Q19 BGK with bounce-back, velocity inlet, pressure
outlet) to the residual tolerance, export of the velocity, then the
substrate steady solve (D2Q5 / D3Q7 advection-diffusion with the biofilm
sink) in that velocity, and the FP64 fluxes.  The electrode mask is built
before the timed region (inputs resident in HBM).  value = lattice-node
updates of both solvers per second over the timed steps, in MLUPS.

Prints one JSON line with a roofline object for the dominant kernel (the
fluid stream-collide step) and the FP64 CPU oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--storage fp32s]
    python bench.py --workload served --storage fp16s [--requests 48] [--rate 50]
    python bench.py --workload c5 [--updates 200] [--compare-storage fp16s]

The served mode replays the seeded request stream (Poisson arrivals, 2-D
domains log-uniform in size) into one server in real time and reports the
p50/p99 solve latency and the aggregate MLUPS beside the plain FP32 single
solves of the same requests, run one at a time on the same GPU.
"""
import argparse
import hashlib
import collections
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM peak (fluid+AD LBM); served p50/p99 steady-solve latency"
HBM_PEAK_GBS = 8000.0
STORAGES = {"fp32": 0, "fp32s": 1, "fp16s": 2, "fp64": 3, "fp32s-f64": 4}
DTYPES = {"fp32": "f32", "fp32s": "f32", "fp16s": "f32 (f16 storage)", "fp64": "f64",
          "fp32s-f64": "f64 (f32 storage)"}
# the step kernels' sources, the solver that picks their launch shapes
# (tile heights, z-segments, steps per launch) and the compiler flags:
# counters taken for other code are not reported
KERNEL_SRC = (os.path.join(ROOT, "paper_1802_07525_amd", "csrc", "kernels.hip"),
              os.path.join(ROOT, "paper_1802_07525_amd", "csrc", "lbm_kernels.h"),
              os.path.join(ROOT, "paper_1802_07525_amd", "csrc", "solver.cpp"))
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def _code_only(text):
    """Source text without comments, blank space and roctx range statements
    (comment edits and host-side trace ranges change neither the kernels
    nor their launch shapes)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = re.sub(r"\bRange rg\([^;]*\);", " ", text)
    return " ".join(text.split())


def kernel_sha():
    from paper_1802_07525_amd import build as libbuild
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path) as fh:
            h.update(_code_only(fh.read()).encode())
    h.update(repr((libbuild.COMMON[:4], libbuild.DEVICE)).encode())
    return h.hexdigest()[:16]


def algo_bytes(q, sb, extra=0):
    """per active-node update: q populations read + q written, 1-byte class"""
    return 2 * q * sb + 1 + extra


def traffic_for(kernel, workload, storage):
    try:
        with open(TRAFFIC) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get("%s|%s|%s" % (kernel, workload, storage))
    if not rec or rec.get("kernel_sha") != kernel_sha():
        return None
    # HBM-side bytes per lattice step of the kernel's launches
    return rec.get("hbm_bytes_per_launch") / rec.get("steps_per_launch", 1)


def default_k(storage_name):
    """The library's residual check interval for a storage form."""
    return 1000 if storage_name == "fp16s" else 100


def _omp():
    """OpenMP runtime the oracle library runs on (same process)."""
    import ctypes
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def _oracle_rate(cls, w, seconds):
    """FP64 oracle MLUPS on the mask: fluid segments from rest, then
    substrate segments from equilibrium in the last velocity, each for about
    seconds / 2.  Segments are 100 steps (2-D) or 10 (3-D)."""
    import numpy as np
    import oracle as O
    seg = 10 if w["nz"] > 1 else 100
    f = O.fluid_init(cls)
    n_f = int(O.flow_domain(cls).sum())
    n_a = int(np.isin(cls, [O.FLUID, O.BIOFILM]).sum())
    t0 = time.perf_counter()
    steps = 0
    U = None
    while True:
        f, U, _ = O.fluid_run(cls, f, w["tau"], w["u_in"], seg)
        steps += seg
        if time.perf_counter() - t0 >= seconds / 2:
            break
    tf = time.perf_counter() - t0
    g = O.ad_init(cls, U, w["c_in"])
    t1 = time.perf_counter()
    asteps = 0
    while True:
        g, _ = O.ad_run(cls, g, U, w["D"], w["c_in"], w["k"], seg)
        asteps += seg
        if time.perf_counter() - t1 >= seconds / 2:
            break
    ta = time.perf_counter() - t1
    return (steps * n_f + asteps * n_a) / (tf + ta) / 1e6, steps, asteps, tf + ta


def cpu_baseline(cls, w, seconds=10.0):
    """FP64 oracle on a bounded sample of the same workload, with all the
    host's OpenMP threads and with one: fluid segments from rest, then
    substrate segments, about `seconds` per thread count."""
    omp = _omp()
    cores = omp.omp_get_max_threads() if omp else os.cpu_count()
    rate, fs, as_, el = _oracle_rate(cls, w, seconds)
    out = {"value": rate, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": "%d fluid + %d substrate FP64 steps from rest on the same %s mask "
                     "(%.1f s, %d threads)" % (fs, as_, w["name"], el, cores),
           "cpu_model": cpu_model()}
    if omp:
        omp.omp_set_num_threads(1)
        try:
            r1, fs1, as1, el1 = _oracle_rate(cls, w, seconds)
        finally:
            omp.omp_set_num_threads(cores)
        out["one_thread"] = {"value": r1, "unit": "MLUPS", "cores": 1,
                             "sample": "%d fluid + %d substrate FP64 steps (%.1f s)" % (fs1, as1, el1)}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def profile_main(args, lbm, ctx, cls, w, storage):
    """Short run for profilers: n fluid steps from rest, the velocity export,
    n substrate steps, then ten 1 GiB device copies by the library's plain
    copy kernel (the reference for counter calibration).  Per-launch HIP-event
    times of the step kernels are printed with the launch counts."""
    n = args.profile_steps
    p = lbm.make_params(tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"], k_sink=w["k"],
                        storage=storage)
    s = lbm.lbm_solver_create(ctx, cls, p)
    _, f_ms = lbm.lbm_solver_steps(s, 0, n, 1)
    lbm.lbm_solver_export_u(s)
    _, a_ms = lbm.lbm_solver_steps(s, 1, n, 1)
    lbm.lbm_solver_destroy(s)
    gbs, copy_ms = lbm.lbm_copy_bandwidth(ctx, 1 << 30, 10)
    lbm.lbm_ctx_destroy(ctx)
    nf = int(lbm.lbm_flow_domain(cls).sum())
    na = int(((cls == 0) | (cls == 3)).sum())
    print(json.dumps({"profile": w["name"], "storage": args.storage, "steps": n,
                      "fluid_nodes": nf, "ad_nodes": na, "grid_nodes": int(cls.size),
                      "fluid_ms_per_step": f_ms / n,
                      "ad_ms_per_step": a_ms / n, "copy_bytes": 1 << 30, "copy_ms": copy_ms,
                      "copy_gbs": gbs}), flush=True)


def coupled_main(args):
    """Coupled biofilm loop on the 512 x 256 anode: cold fluid and substrate
    solves, then `updates` growth steps, each followed by warm re-solves of
    both solvers to the tolerance; the consumed flux J is accumulated in
    FP64.  With --compare-storage the same biofilm history is re-solved in
    that storage and the J series are compared."""
    import numpy as np
    import torch

    import paper_1802_07525_amd as lbm
    from paper_1802_07525_amd import inputs

    assert torch.cuda.is_available(), "no GPU visible"
    lbm.load()
    w = inputs.WORKLOADS["c5"]
    st, cls, _ = lbm.lbm_geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                    w["overlap"], w["seed"])
    assert st == 0
    cls = lbm.lbm_biofilm_layer(cls)
    updates = args.updates or w["updates"]
    xi = inputs.growth_draws(updates, seed=w["seed"])
    ctx = lbm.lbm_ctx_create(0)

    def run(storage):
        p = lbm.make_params(tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"], k_sink=w["k"],
                            storage=storage, stall_checks=args.stall_checks)
        s = lbm.lbm_solver_create(ctx, cls, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stc, out = lbm.lbm_coupled_run(s, xi, w["tol"], args.max_iter or w["max_iter"])
        el = time.perf_counter() - t0
        lbm.lbm_solver_destroy(s)
        # updates completed: the loop stops at the first failing solve
        done = int(np.count_nonzero(out["iters_ad"])) - 1
        return stc, out, el, done

    storage = STORAGES[args.storage]
    stc, out, el, done = run(storage)
    # nodes updated per solve: the flow domain after each growth step (a
    # step can close a pore), and the substrate nodes (growth keeps them)
    flat = cls.reshape(-1).copy()
    nfs = [int(lbm.lbm_flow_domain(cls).sum())]
    for q in out["picked"][:done]:
        flat[q] = 3
        nfs.append(int(lbm.lbm_flow_domain(flat.reshape(cls.shape)).sum()))
    nfs += [0] * (updates + 1 - len(nfs))
    na = int(((cls == 0) | (cls == 3)).sum())
    upd = float(np.sum(out["iters_fluid"] * np.asarray(nfs)) + np.sum(out["iters_ad"] * na))
    res = {
        "metric": METRIC, "value": upd / el / 1e6, "unit": "MLUPS", "n_gpus": 1, "steps": updates,
        "warmup": 0, "ms_per_step": el / max(updates, 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.storage], "data": "synthetic",
        "config": {"workload": w["name"], "grid": [w["nx"], w["ny"], 1], "storage": args.storage,
                   "updates": updates, "tol": w["tol"], "seed": w["seed"],
                   "status": lbm.status_name(stc), "updates_done": done},
        "coupled": {"seconds": el, "J_accum": out["J_accum"], "J0": float(out["J"][0]),
                    "J_last": float(out["J"][-1]),
                    "fluid_iters_cold": int(out["iters_fluid"][0]),
                    "ad_iters_cold": int(out["iters_ad"][0]),
                    "fluid_iters_warm_mean": float(np.mean(out["iters_fluid"][1:])) if updates else 0.0,
                    "ad_iters_warm_mean": float(np.mean(out["iters_ad"][1:])) if updates else 0.0},
    }
    if args.compare_storage:
        # the same biofilm history (the first run's picks) in the other
        # storage: an independent loop would part at its first pick, a
        # discontinuous function of C
        p = lbm.make_params(tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"], k_sink=w["k"],
                            storage=STORAGES[args.compare_storage], stall_checks=args.stall_checks,
                            check_every=args.compare_check_every)
        s = lbm.lbm_solver_create(ctx, cls, p)
        mi = args.max_iter or w["max_iter"]
        J2, fail = [], None
        t0 = time.perf_counter()
        for m in range(done + 1):
            if m > 0:
                assert lbm.lbm_solver_update_cells(s, [out["picked"][m - 1]], [3]) == 0
            sf, _ = lbm.lbm_solver_fluid(s, w["tol"], mi, int(m > 0))
            sa, ai = lbm.lbm_solver_ad(s, w["tol"], mi, int(m > 0)) if sf >= 0 else (0, None)
            if sf < 0 or sa < 0:
                fail = {"update": m, "solver": "fluid" if sf < 0 else "substrate",
                        "status": lbm.status_name(sf if sf < 0 else sa)}
                break
            J2.append(ai["sink_total"])
        el2 = time.perf_counter() - t0
        lbm.lbm_solver_destroy(s)
        k = len(J2)
        J1 = np.asarray(out["J"][:k])
        J2 = np.asarray(J2)
        rel = np.abs(J2 - J1) / np.abs(J1)
        res["compare"] = {"storage": args.compare_storage, "seconds": el2, "updates": k - 1,
                          "check_every": args.compare_check_every or default_k(args.compare_storage),
                          "first_failure": fail,
                          "J_accum": float(J2[1:].sum()),
                          "J_accum_rel_diff": float(abs(J2[1:].sum() - J1[1:].sum()) / abs(J1[1:].sum()))
                          if k > 1 else None,
                          "J_rel_diff_max": float(rel.max()) if k else None,
                          "J_rel_diff_median": float(np.median(rel)) if k else None}
    lbm.lbm_ctx_destroy(ctx)
    print(json.dumps(res), flush=True)


def mfc_main(args):
    """The model loop of Sec. 2 on the 512 x 256 electrode, one hour per
    interval: fluid and substrate solves to 1e-6 (cold, then warm), the
    bio-electrochemical update (one work-group kernel) and the agent-based
    biofilm (host), Table 1's parameters.  Reports lattice updates per
    second over the loop, the time per stage and the V, I series' ends."""
    import numpy as np
    import torch

    import paper_1802_07525_amd as lbm
    from paper_1802_07525_amd import inputs

    assert torch.cuda.is_available(), "no GPU visible"
    lbm.load()
    w = inputs.WORKLOADS["mfc"]
    st, cls, _ = lbm.lbm_geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                    w["overlap"], w["seed"])
    assert st == 0
    hours = args.hours or w["hours"]
    ctx = lbm.lbm_ctx_create(0)
    p = lbm.make_params(tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"], k_sink=w["k"],
                        storage=STORAGES[args.storage], stall_checks=args.stall_checks)
    s = lbm.lbm_solver_create(ctx, cls, p)
    b = lbm.lbm_bio_create(s, lbm.make_bio_params(**inputs.bio_params(w["c_in"])), None, None, ctx)
    fp = lbm.make_biofilm_params(Y_bio=args.y_bio)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stc, series = lbm.lbm_mfc_run(b, fp, hours, w["seed"], w["tol"], args.max_iter or w["max_iter"])
    el = time.perf_counter() - t0
    lbm.lbm_bio_destroy(b)
    lbm.lbm_solver_destroy(s)
    lbm.lbm_ctx_destroy(ctx)
    done = [r for r in series if r["iters_ad"] > 0 and r["film"]["cells"] > 0]
    upd = float(sum(r["iters_fluid"] * r["nodes_fluid"] + r["iters_ad"] * r["nodes_ad"]
                    for r in series))
    I = [r["bio"]["I_cell"] for r in done]
    V = [r["bio"]["V_cell"] for r in done]
    res = {
        "metric": METRIC, "value": upd / el / 1e6, "unit": "MLUPS", "n_gpus": 1, "steps": hours,
        "warmup": 0, "ms_per_step": el / max(len(done), 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.storage], "data": "synthetic",
        "config": {"workload": w["name"], "grid": [w["nx"], w["ny"], 1], "storage": args.storage,
                   "hours": hours, "hours_done": len(done), "tol": w["tol"], "seed": w["seed"],
                   "Y_bio": args.y_bio, "status": lbm.status_name(stc)},
        "mfc": {"seconds": el,
                "seconds_solves": float(sum(r["seconds_solves"] for r in series)),
                "seconds_bio": float(sum(r["seconds_bio"] for r in series)),
                "seconds_film": float(sum(r["seconds_film"] for r in series)),
                "bio_ms_mean": float(np.mean([r["seconds_bio"] for r in done]) * 1e3) if done else None,
                "film_ms_mean": float(np.mean([r["seconds_film"] for r in done]) * 1e3) if done else None,
                "fluid_iters": [int(r["iters_fluid"]) for r in series],
                "ad_iters": [int(r["iters_ad"]) for r in series],
                "I_mA": [round(x * 1e3, 6) for x in I],
                "V_mV": [round(x * 1e3, 4) for x in V],
                "biofilm_cells": [int(r["film"]["cells"]) for r in done],
                "spread": int(sum(r["film"]["spread"] for r in done)),
                "walks": int(sum(r["film"]["walks"] for r in done))},
    }
    print(json.dumps(res), flush=True)


def _serve_stream(lbm, ctx, reqs, storage, args, max_iter):
    """Submit reqs in real time (Poisson arrivals) to a fresh server and
    collect every result: (results by request index, refusals, stats)."""
    import threading

    cfg = lbm.make_server_cfg(int(args.pool_gb * (1 << 30)), max_slots=args.slots, storage=storage,
                              prep_threads=4, stall_checks=args.stall_checks,
                              check_every=args.check_every, escalate=int(args.escalate),
                              solo_nodes=args.solo_nodes, solo_lanes=args.solo_lanes)
    srv = lbm.lbm_server_create(ctx, cfg)

    def request(r):
        return lbm.make_request(r["nx"], r["ny"], r_min=r["r_min"], r_max=r["r_max"],
                                solid_frac=1.0 - r["porosity"], overlap=r["overlap"],
                                seed=r["seed"], layer=0, tau=r["tau"], u_in=r["u_in"], D=r["D"],
                                c_in=r["c_in"], k_sink=r["k"], tol=r["tol"], max_iter=max_iter,
                                user=r["i"])

    results, refused = {}, []
    t_start = time.perf_counter()

    def feeder():
        for r in reqs:
            dt = r["arrival"] - (time.perf_counter() - t_start)
            if dt > 0:
                time.sleep(dt)
            st, _ = lbm.lbm_server_submit(srv, request(r))
            if st:
                refused.append((r["i"], lbm.status_name(st), lbm.lbm_server_error(srv)))

    th = threading.Thread(target=feeder)
    th.start()
    last = time.perf_counter()
    while len(results) + len(refused) < len(reqs):
        for d in lbm.lbm_server_poll(srv, 64, 0.5):
            results[d["user"]] = d
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            print("served: %d/%d finished after %.0f s" % (len(results), len(reqs), last - t_start),
                  file=sys.stderr, flush=True)
    th.join()
    stats = lbm.lbm_server_stats(srv)
    lbm.lbm_server_destroy(srv)
    return results, refused, stats


def _single(lbm, ctx, r, storage, max_iter, fixed=None):
    """One request as a plain single solve: to its tolerance, or (fixed =
    (fluid steps, substrate steps)) for exactly those steps.  Returns
    (seconds, updates, U, C, status pair) or None if the fluid diverged."""
    st, cls, _ = lbm.lbm_geom_discs(r["nx"], r["ny"], r["r_min"], r["r_max"], 1.0 - r["porosity"],
                                    r["overlap"], r["seed"])
    p = lbm.make_params(tau=r["tau"], u_in=r["u_in"], D=r["D"], c_in=r["c_in"], k_sink=r["k"],
                        storage=storage)
    ts = time.perf_counter()
    s = lbm.lbm_solver_create(ctx, cls, p)
    if fixed is None:
        sf, fi = lbm.lbm_solver_fluid(s, r["tol"], max_iter)
        if sf < 0:
            lbm.lbm_solver_destroy(s)
            return None
        sa, ai = lbm.lbm_solver_ad(s, r["tol"], max_iter)
        upd = fi["iters"] * fi["active_nodes"] + ai["iters"] * ai["active_nodes"]
        stat = (sf, sa)
    else:
        lbm.lbm_solver_steps(s, 0, fixed[0], 1)
        lbm.lbm_solver_export_u(s)
        lbm.lbm_solver_steps(s, 1, fixed[1], 1)
        nf = int(lbm.lbm_flow_domain(cls).sum())
        na = int(((cls == 0) | (cls == 3)).sum())
        upd = fixed[0] * nf + fixed[1] * na
        stat = (0, 0)
    grid = (r["nx"], r["ny"], 1)
    U = lbm.lbm_solver_get(s, lbm.LBM_FIELD_U, grid)
    C = lbm.lbm_solver_get(s, lbm.LBM_FIELD_C, grid)
    lbm.lbm_solver_destroy(s)
    return time.perf_counter() - ts, upd, U, C, stat, cls


def served_main(args):
    """Served stream: the seeded requests with Poisson arrivals, submitted in
    real time to one server (continuous batching) at each rate of the sweep
    (one JSON line per rate: p50/p99 latency, throughput).  Then the same
    requests as plain single solves one at a time on the same GPU in FP32
    shifted storage: to their tolerance (throughput), and for exactly the
    served solves' step counts (equal work; field errors of the served
    results against them)."""
    import numpy as np
    import torch

    import paper_1802_07525_amd as lbm
    from paper_1802_07525_amd import inputs

    assert torch.cuda.is_available(), "no GPU visible"
    lbm.load()
    storage = STORAGES[args.storage]
    max_iter = args.max_iter or 2_000_000
    rates = [float(x) for x in args.rates.split(",")] if args.rates else [args.rate]
    ctx = lbm.lbm_ctx_create(0)
    sb = {0: 4, 1: 4, 2: 2, 4: 4}[storage]
    last_results = None
    for rate in rates:
        reqs = inputs.serve_requests(args.requests, rate)
        results, refused, stats = _serve_stream(lbm, ctx, reqs, storage, args, max_iter)
        done = [d for d in results.values() if d["status"] >= 0]
        lat = np.array([d["t_finish"] - d["t_submit"] for d in done])
        t0 = min(d["t_submit"] for d in results.values())
        t1 = max(d["t_finish"] for d in results.values())
        makespan = t1 - t0
        upd = sum(d["iters_fluid"] * d["active_fluid"] + d["iters_ad"] * d["active_ad"] for d in done)
        algo = sum(d["iters_fluid"] * d["active_fluid"] * algo_bytes(9, sb)
                   + d["iters_ad"] * d["active_ad"] * algo_bytes(5, sb, 8) for d in done)
        achieved = algo / stats["busy_seconds"] / 1e9 if stats["busy_seconds"] > 0 else 0.0
        line = {
            "metric": METRIC, "value": upd / makespan / 1e6, "unit": "MLUPS", "n_gpus": 1,
            "steps": len(reqs), "warmup": 0, "ms_per_step": makespan / len(reqs) * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": DTYPES[args.storage], "data": "synthetic",
            "config": {"workload": "served stream: first %d requests of the seeded stream, Poisson "
                                   "%g req/s, 2-D D2Q9+D2Q5, nx log-uniform 64..2048, ny = nx/2"
                                   % (len(reqs), rate),
                       "rate": rate, "storage": args.storage, "pool_gb": args.pool_gb,
                       "check_every": args.check_every or default_k(args.storage),
                       "slots": args.slots, "seed": inputs.SERVE_SEED,
                       "escalate": bool(args.escalate), "solo_nodes": args.solo_nodes or 262144,
                       "solo_lanes": args.solo_lanes or 2},
            "served": {"completed": len(done), "failed": len(results) - len(done) + len(refused),
                       "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                       "p50_by_lane_s": {name: float(np.percentile([d["t_finish"] - d["t_submit"] for d in done
                                                                    if d["lane"] == k], 50))
                                         for k, name in ((0, "batch"), (1, "solo"), (2, "escalated"))
                                         if any(d["lane"] == k for d in done)},
                       "mean_s": float(lat.mean()), "makespan_s": makespan,
                       "req_per_s": len(done) / makespan, "busy_s": stats["busy_seconds"],
                       "chunks": stats["chunks"], "chunks_wide": stats["chunks_wide"],
                       "pool_peak_gb": stats["pool_peak"] / 2 ** 30,
                       "lanes": {"batch": int(sum(1 for d in results.values() if d["lane"] == 0)),
                                 "solo": int(sum(1 for d in results.values() if d["lane"] == 1)),
                                 "escalated": int(sum(1 for d in results.values() if d["lane"] == 2))},
                       "escalated": {"%s->%s" % (lbm.status_name(a), lbm.status_name(b)): int(n)
                                     for (a, b), n in sorted(collections.Counter(
                                         (d["first_status"], d["status"]) for d in results.values()
                                         if d["lane"] == 2).items())},
                       "requests": [[int(d["user"]), int(d["status"]), int(d["lane"]), int(d["iters_fluid"]),
                                     int(d["iters_ad"])] for d in sorted(results.values(),
                                                                         key=lambda d: d["user"])],
                       "statuses": {lbm.status_name(k): int(sum(1 for d in results.values()
                                                                if d["status"] == k))
                                    for k in sorted({d["status"] for d in results.values()})}},
            "roofline": {"bound": "hbm", "kernel": "k_srv_step (batched fluid+substrate)",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "note": "algorithmic bytes of the returned solves (batch and solo lane; "
                                 "not the discarded first attempts of escalated requests) / "
                                 "device-busy time of either lane"},
        }
        print(json.dumps(line), flush=True)
        last_results = (reqs, results, makespan, upd)
    if args.no_single:
        lbm.lbm_ctx_destroy(ctx)
        return
    reqs, results, makespan, upd = last_results
    done = sorted((d for d in results.values() if d["status"] >= 0), key=lambda d: d["user"])
    # single FP32-shifted solves to tolerance (throughput), then at the served
    # step counts (equal work: field errors)
    single_s, single_upd, fail = 0.0, 0.0, 0
    eq_s, eq_upd, eu, ec, n_ok, detail = 0.0, 0.0, [], [], 0, []
    last = time.perf_counter()
    for d in done:
        if time.perf_counter() - last > 20:
            last = time.perf_counter()
            print("single FP32S: request %d of %d" % (d["user"], len(reqs)), file=sys.stderr, flush=True)
        r = reqs[d["user"]]
        a = _single(lbm, ctx, r, STORAGES["fp32s"], max_iter)
        if a is None:
            fail += 1
        else:
            single_s += a[0]
            single_upd += a[1]
        b = _single(lbm, ctx, r, STORAGES["fp32s"], max_iter, fixed=(d["iters_fluid"], d["iters_ad"]))
        eq_s += b[0]
        eq_upd += b[1]
        U, C, cls = b[2], b[3], b[5]
        flat = cls.reshape(-1)
        fl, act = flat == 0, (flat == 0) | (flat == 3)
        eu.append(float(np.linalg.norm(d["u"][:, fl] - U[:, fl]) / np.linalg.norm(U[:, fl])))
        ec.append(float(np.linalg.norm(d["c"][act] - C[act]) / np.linalg.norm(C[act])))
        n_ok += d["status"] == 0
        detail.append({"user": int(d["user"]), "status": lbm.status_name(d["status"]),
                       "porosity": round(r["porosity"], 3), "nx": r["nx"],
                       "u": round(eu[-1], 6), "c": round(ec[-1], 6)})
    lbm.lbm_ctx_destroy(ctx)
    eu, ec = np.array(eu), np.array(ec)
    within = (eu < 5e-3) & (ec < 5e-3)
    print(json.dumps({
        "compare": "served %s (last rate) against single FP32-shifted solves of the same %d requests "
                   "on the same GPU" % (args.storage, len(done)),
        "served_makespan_s": makespan, "served_mlups": upd / makespan / 1e6,
        "served_ok": int(n_ok),
        "single_fp32s_to_tol": {"seconds": single_s, "mlups": single_upd / single_s / 1e6,
                                "failed": fail, "req_per_s": (len(done) - fail) / single_s},
        "single_fp32s_equal_steps": {"seconds": eq_s, "mlups": eq_upd / eq_s / 1e6,
                                     "speedup_served": eq_s / makespan},
        "fields_vs_equal_steps": {"u_rel_l2_median": float(np.median(eu)), "u_rel_l2_max": float(eu.max()),
                                  "c_rel_l2_median": float(np.median(ec)), "c_rel_l2_max": float(ec.max()),
                                  "frac_within_5e-3": float(within.mean()),
                                  "frac_within_5e-3_of_ok": float(within[[d["status"] == 0 for d in done]].mean())
                                  if n_ok else None,
                                  "outside": [x for x, ok in zip(detail, within) if not ok]}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--storage", default="fp32s", choices=sorted(STORAGES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-iter", type=int, default=0)
    ap.add_argument("--requests", type=int, default=48, help="served stream length")
    ap.add_argument("--rate", type=float, default=50.0, help="served arrivals per second")
    ap.add_argument("--rates", default="", help="served: comma-separated arrival rates (a sweep)")
    ap.add_argument("--no-single", action="store_true", help="served: skip the single-solve comparison")
    ap.add_argument("--check-every", type=int, default=0,
                    help="residual check interval of the solves or the server (0: the library "
                         "default, 100, or 1000 with FP16 storage)")
    ap.add_argument("--pool-gb", type=float, default=32.0)
    ap.add_argument("--escalate", action="store_true",
                    help="served: re-solve failed reduced-storage requests in FP32-shifted storage")
    ap.add_argument("--solo-nodes", type=int, default=0,
                    help="served: requests of at least this many nodes go to the solo lanes "
                         "(0: the library default, 262,144; -1: none)")
    ap.add_argument("--solo-lanes", type=int, default=0, help="served: solo-lane threads (0: 2)")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--stall-checks", type=int, default=0,
                    help="stall window in checks (0: the library default)")
    ap.add_argument("--updates", type=int, default=0, help="coupled loop: growth updates")
    ap.add_argument("--hours", type=int, default=0, help="model loop: intervals (0: 72)")
    ap.add_argument("--y-bio", type=float, default=1.0,
                    help="model loop: biomass yield on the consumed substrate")
    ap.add_argument("--compare-storage", default="", choices=[""] + sorted(STORAGES),
                    help="coupled loop: repeat in this storage and compare")
    ap.add_argument("--compare-check-every", type=int, default=0,
                    help="coupled loop: residual check interval of the compared run (0: the "
                         "library default)")
    ap.add_argument("--ad-lattice", default="d2q5", choices=["d2q5", "d2q9"],
                    help="2-D substrate lattice: D2Q5 with the linear equilibrium, or the "
                         "paper's D2Q9 with the Eq. 5 equilibrium")
    ap.add_argument("--k-half", type=float, default=0.0,
                    help="Monod half-saturation of the biofilm sink (0: first order)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="profiling run: this many fluid and substrate steps of the workload "
                         "and a 1 GiB copy (counter calibration) instead of the solves")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the served stream and slab decomposition would shard across GPUs; "
              "they are not built).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "served":
        if args.storage == "fp64":
            sys.exit("the served form stores FP32 or FP16")
        return served_main(args)
    if args.workload == "c5":
        return coupled_main(args)
    if args.workload == "mfc":
        return mfc_main(args)

    import numpy as np
    import torch

    import paper_1802_07525_amd as lbm
    from paper_1802_07525_amd import inputs

    assert torch.cuda.is_available(), "no GPU visible"
    lbm.load()
    w = inputs.WORKLOADS[args.workload]
    storage = STORAGES[args.storage]
    if w["nz"] > 1:
        st, cls, _ = lbm.lbm_geom_fibres(w["nx"], w["ny"], w["nz"], w["r_min"], w["r_max"],
                                         w["solid"], w["seed"])
    else:
        st, cls, _ = lbm.lbm_geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                        w["overlap"], w["seed"])
    assert st == 0
    if w.get("layer", True):
        cls = lbm.lbm_biofilm_layer(cls)
    max_iter = args.max_iter or w["max_iter"]
    ctx = lbm.lbm_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    if args.profile_steps:
        return profile_main(args, lbm, ctx, cls, w, storage)
    ad9 = args.ad_lattice == "d2q9"
    if ad9 and w["nz"] > 1:
        sys.exit("--ad-lattice d2q9 is a 2-D option")
    p = lbm.make_params(tau=w["tau"], u_in=w["u_in"], D=w["D"], c_in=w["c_in"], k_sink=w["k"],
                        storage=storage, stall_checks=args.stall_checks, k_half=args.k_half,
                        ad_lattice=int(ad9), check_every=args.check_every)
    s = lbm.lbm_solver_create(ctx, cls, p)

    def one_step():
        sf, fi = lbm.lbm_solver_fluid(s, w["tol"], max_iter, 0)
        if sf < 0:
            raise RuntimeError("fluid solve failed: %s %s" % (lbm.status_name(sf),
                                                              lbm.lbm_last_error(ctx)))
        sa, ai = lbm.lbm_solver_ad(s, w["tol"], max_iter, 0)
        if sa < 0:
            raise RuntimeError("substrate solve failed: %s %s" % (lbm.status_name(sa),
                                                                  lbm.lbm_last_error(ctx)))
        return sf, fi, sa, ai

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [one_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    upd = sum(fi["iters"] * fi["active_nodes"] + ai["iters"] * ai["active_nodes"]
              for _, fi, _, ai in recs)
    value = upd / el / 1e6
    sf, fi, sa, ai = recs[-1]
    dim = 3 if w["nz"] > 1 else 2
    qf, qa = (19, 7) if dim == 3 else (9, 9 if ad9 else 5)
    sb = {0: 4, 1: 4, 2: 2, 3: 8, 4: 4}[storage]
    cb = 8 if storage == 3 else 4
    # Per solver: HIP-event time over its launches in the timed region (on
    # the library's stream).  A launch advances several steps -- two in 3-D
    # (z-marching blocks), two or four in 2-D -- so the algorithmic bytes of
    # a launch are the per-step figure times the solve's steps per launch.
    copy_gbs, _ = lbm.lbm_copy_bandwidth(ctx, 1 << 30, 10)

    def kernel_figures(which, q, extra, idx, name):
        ms = sum(r[idx]["kernel_ms"] for r in recs)
        nl = sum(r[idx]["launches"] for r in recs)
        spl = sum(r[idx]["iters"] for r in recs) / max(nl, 1)
        avg = ms / max(nl, 1)
        nodes = recs[-1][idx]["active_nodes"]
        algo = spl * algo_bytes(q, sb, extra) * nodes
        gbs = algo / (avg * 1e-3) / 1e9
        # isolated per-launch HIP-event timing on the same state
        _, iso = lbm.lbm_solver_time_steps(s, which, 300)
        per_step = traffic_for(name, args.workload, args.storage)
        traffic = None if per_step is None else per_step * spl
        rec = {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
               "algo_bytes_per_launch": algo, "steps_per_launch": spl, "avg_launch_ms": avg,
               "avg_launch_ms_isolated": iso, "launches": nl, "kernel_ms_total": ms,
               "copy_gbs": copy_gbs, "frac_of_copy": gbs / copy_gbs,
               # HBM bytes actually moved (counters) over the same launch time
               "hbm_gbs": None if traffic is None else traffic / (avg * 1e-3) / 1e9}
        rec["hbm_frac"] = None if traffic is None else rec["hbm_gbs"] / HBM_PEAK_GBS
        return rec

    form = lambda spl: ("3d2" if spl > 1.5 else "") if dim == 3 else ("N" if spl > 2.5 else "2")
    nl_f = sum(r[1]["launches"] for r in recs)
    nl_a = sum(r[3]["launches"] for r in recs)
    spl_f = sum(r[1]["iters"] for r in recs) / max(nl_f, 1)
    spl_a = sum(r[3]["iters"] for r in recs) / max(nl_a, 1)
    lat_f = "D3Q19" if dim == 3 else "D2Q9"
    lat_a = "D3Q7" if dim == 3 else ("D2Q9" if ad9 else "D2Q5")
    fl = kernel_figures(0, qf, 0, 1, "k_fluid_step%s<%s,%s>" % (form(spl_f), lat_f, args.storage))
    ad = kernel_figures(1, qa, dim * cb, 3, "k_ad_step%s<%s,%s>" % (form(spl_a), lat_a, args.storage))
    # the roofline object is the kernel with the larger share of GPU time
    dom, other = (fl, ad) if fl["kernel_ms_total"] >= ad["kernel_ms_total"] else (ad, fl)
    n_all = w["nx"] * w["ny"] * w["nz"]
    upd_all = sum((fi_["iters"] + ai_["iters"]) * n_all for _, fi_, _, ai_ in recs)
    layer = w.get("layer", True)
    out = {
        "metric": METRIC, "value": value, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[args.storage], "data": "synthetic",
        "config": {"workload": w["name"], "grid": [w["nx"], w["ny"], w["nz"]],
                   "storage": args.storage, "tau": w["tau"], "u_in": w["u_in"], "D": w["D"],
                   "biofilm_layer": layer, "k_sink": w["k"] if layer else None,
                   "k_half": args.k_half if layer else None,
                   "substrate_lattice": "d3q7" if dim == 3 else args.ad_lattice,
                   "tol": w["tol"], "seed": w["seed"],
                   "check_every": args.check_every or default_k(args.storage),
                   "fluid_status": lbm.status_name(sf), "fluid_iters": fi["iters"],
                   "ad_status": lbm.status_name(sa), "ad_iters": ai["iters"],
                   "fluid_nodes": fi["active_nodes"], "ad_nodes": ai["active_nodes"],
                   "fluid_seconds": fi["seconds"], "ad_seconds": ai["seconds"],
                   "mlups_all_nodes": upd_all / el / 1e6},
        "roofline": dom,
        "roofline_other": other,
    }
    lbm.lbm_solver_destroy(s)
    lbm.lbm_ctx_destroy(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cls, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

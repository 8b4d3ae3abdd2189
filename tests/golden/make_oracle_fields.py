"""Write the FP64 oracle's fields for a workload at its full size (test data).

    python tests/golden/make_oracle_fields.py <workload> <fluid_steps> <substrate_steps>

Builds the workload's electrode mask with the oracle's own generators, runs
the oracle's fluid solver from rest for <fluid_steps> steps (Sec. 2.1.1),
then its substrate solver from equilibrium at c_in in the resulting
velocity for <substrate_steps> steps (Sec. 2.1.2), and stores a sample of
the fields with the FP64 fluxes in
tests/golden/oracle_fields/<workload>_f<fluid_steps>_a<substrate_steps>.npz.

The step counts are those at which the GPU's FP32-shifted steady solves of
the workload stop at its tolerance, so that the parity tests compare fields
at matched iterations.  Only the oracle and the seeded workload settings are
used.  The sample is every eighth row of a 2-D grid, or the planes z = 32,
64 and 96 of a 3-D one; velocity, density and concentration are stored as
float32 (relative precision 6e-8, far below the 1e-4 and 5e-3 bounds they
are compared at).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1802_07525_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "oracle_fields")


def mask(w):
    if w["nz"] > 1:
        st, cls, _ = O.geom_fibres(w["nx"], w["ny"], w["nz"], w["r_min"], w["r_max"], w["solid"],
                                   w["seed"])
    else:
        st, cls, _ = O.geom_discs(w["nx"], w["ny"], w["r_min"], w["r_max"], w["solid"],
                                  w["overlap"], w["seed"])
    assert st == "OK"
    return O.biofilm_layer(cls) if w.get("layer", True) else cls


def sample_nodes(w):
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    if nz > 1:
        return idx[[32, 64, 96]].ravel()
    return idx[0, 3::8].ravel()


def path_for(name, nf, na):
    return os.path.join(OUT, "%s_f%d_a%d.npz" % (name, nf, na))


def main(name, nf, na):
    w = inputs.WORKLOADS[name]
    cls = mask(w)
    t0 = time.time()
    f, _, _ = O.fluid_run(cls, O.fluid_init(cls), w["tau"], w["u_in"], nf)
    U, rho = O.fluid_moments(cls, f)
    fin, fout = O.fluid_fluxes(cls, f, w["u_in"])
    t1 = time.time()
    print("fluid %d steps: %.0f s" % (nf, t1 - t0), flush=True)
    g, _ = O.ad_run(cls, O.ad_init(cls, U, w["c_in"]), U, w["D"], w["c_in"], w["k"], na)
    C = O.ad_moment(cls, g, w["k"])
    ain, aout, sink = O.ad_fluxes(cls, g, w["c_in"], w["k"])
    print("substrate %d steps: %.0f s" % (na, time.time() - t1), flush=True)
    nodes = sample_nodes(w)
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(path_for(name, nf, na), nodes=nodes.astype(np.int32),
                        U=U[:, nodes].astype(np.float32),
                        rho_m1=(rho[nodes] - 1.0).astype(np.float32),
                        C=C[nodes].astype(np.float32),
                        fluxes=np.array([fin, fout, ain, aout, sink]),
                        steps=np.array([nf, na]))
    print("wrote", path_for(name, nf, na), flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]))

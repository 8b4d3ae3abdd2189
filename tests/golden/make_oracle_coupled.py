"""Write the FP64 oracle's coupled biofilm loop at the workload's full size.

    python tests/golden/make_oracle_coupled.py [updates]

Runs the oracle's coupled loop (the model loop of Sec. 2 with the simplified
growth rule: cold fluid and substrate solves, then `updates` growth picks,
each followed by warm re-solves of both) on the 512 x 256 coupled-loop
workload, with the workload's seeded growth draws, and stores the growth
picks, the consumption series J, J_accum, the iteration counts and a sample
of the final fields in tests/golden/oracle_fields/c5_u<updates>.npz.  Only
the oracle and the seeded workload settings are used.  Sample: every eighth
row, float32.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle as O  # noqa: E402
from make_oracle_fields import OUT, mask, sample_nodes  # noqa: E402
from paper_1802_07525_amd import inputs  # noqa: E402


def path_for(updates):
    return os.path.join(OUT, "c5_u%d.npz" % updates)


def main(updates):
    w = inputs.WORKLOADS["c5"]
    cls = mask(w)
    xi = inputs.growth_draws(updates, seed=w["seed"])
    t0 = time.time()
    o = O.coupled_run(cls, w["tau"], w["u_in"], w["D"], w["c_in"], w["k"], w["tol"], w["max_iter"], xi)
    print("coupled loop, %d updates: %s in %.0f s" % (updates, o["status"], time.time() - t0), flush=True)
    assert o["status"] == "OK", o["status"]
    nodes = sample_nodes(w)
    os.makedirs(OUT, exist_ok=True)
    np.savez_compressed(path_for(updates), picked=o["picked"], J=o["J"], J_accum=np.array([o["J_accum"]]),
                        iters_fluid=o["iters_fluid"], iters_ad=o["iters_ad"], nodes=nodes.astype(np.int32),
                        U=o["U"][:, nodes].astype(np.float32), C=o["C"][nodes].astype(np.float32))
    print("wrote", path_for(updates), flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else inputs.WORKLOADS["c5"]["updates"])

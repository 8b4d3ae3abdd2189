"""MI355X (gfx950) lattice Boltzmann library for the anode compartment of a
microbial fuel cell (Tsompanas et al., arXiv 1802.07525, Sec. 2.1).

The lattice work runs in the HIP library ``_lbm.so`` behind the C ABI of
``include/lbm.h``; this package is its ctypes binding (same names) plus
the seeded workload definitions in ``inputs``.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import load, exported_symbols, Solver, LBMError  # noqa: F401

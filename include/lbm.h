/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for the
 * anode compartment of a microbial fuel cell, after Tsompanas et al.,
 * "Modelling Microbial Fuel Cells using lattice Boltzmann methods"
 * (arXiv 1802.07525).
 *
 * The library computes the two coupled steady states of the paper's model
 * loop (Sec. 2, steps 2 and 3): the BGK fluid flow through a porous anode
 * with bounce-back on electrode and biofilm nodes (Sec. 2.1.1, Eqs. 1-11),
 * and the advection-diffusion of substrate in that frozen flow with
 * zero-flux solids, a Dirichlet inlet and consumption on biofilm nodes
 * (Sec. 2.1.2, Eqs. 12-13).  Both are re-converged whenever the biofilm
 * changes (Sec. 2.3).  Everything that steps a lattice runs in hand-written
 * HIP kernels on one GPU; the host side only validates, builds masks and
 * decides when to stop.
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid: nx * ny * nz nodes (nz = 1 for 2-D), linear index
 *   n = x + nx * (y + ny * z), x fastest.  Flow enters at x = 0 and leaves
 *   at x = nx - 1 (Sec. 3: influent from the left, effluent to the right).
 * Node classes (uint8): LBM_FLUID, LBM_SOLID (electrode), LBM_WALL
 *   (chassis), LBM_BIOFILM.  Rows y = 0 and y = ny - 1 (and planes z = 0,
 *   nz - 1 in 3-D) must be WALL or SOLID; columns x = 0 and x = nx - 1 must
 *   hold no SOLID or BIOFILM.  The fluid sees SOLID, WALL and BIOFILM as
 *   blocked (the biofilm is impermeable, Sec. 2.3 and Sec. 4); the
 *   substrate sees only SOLID and WALL as blocked and is consumed on
 *   BIOFILM.
 * Lattices: D2Q9 / D2Q5 in 2-D, D3Q19 / D3Q7 in 3-D.  D2Q9 directions
 *   follow Eqs. 1-3 with 1=(1,0), 2=(0,1), 3=(-1,0), 4=(0,-1), 5=(1,1),
 *   6=(-1,1), 7=(-1,-1), 8=(1,-1) (opposites 1-3, 2-4, 5-7, 6-8 as Eq. 11
 *   pairs them); D2Q5 is 0..4 of that.  D3Q19: 0 rest; 1..6 = +x,-x,+y,-y,
 *   +z,-z; 7..18 = (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),
 *   (1,0,-1),(-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1); D3Q7 is 0..6.
 * Units: lattice units throughout.  tau > 1/2 is the fluid relaxation time
 *   of Eq. 4 (nu = (tau - 1/2)/3); D > 0 is the substrate diffusivity, and
 *   the substrate relaxation time of Eq. 12 is tau_D = 1/2 + D / c_s^2 with
 *   c_s^2 = 1/3 (D2Q5) or 1/4 (D3Q7) -- the relation Table 1's tau_D and D
 *   satisfy.
 * Memory: the caller owns every pointer it passes and keeps it valid for
 *   the call; the library never frees caller memory and copies what it
 *   keeps.  Handles are owned by the library until their destroy call.
 *   Array arguments are host (CPU) memory unless a call says otherwise.
 * Threads: a context (and the solvers made from it) is used by one host
 *   thread at a time.  Server calls are thread-safe.
 * Errors: every call that can fail returns lbm_status.  LBM_NOT_CONVERGED
 *   and LBM_STALLED still fill every output.  LBM_EDEVICE means a HIP call
 *   failed; lbm_last_error() then holds the HIP message.  No call aborts
 *   the process.
 * Tracing: with LBM_ROCTX=1 in the environment when the first range opens,
 *   the library marks its host phases as roctx ranges, which rocprofv3
 *   --marker-trace records: lbm.geometry (a generated electrode),
 *   lbm.fluid.steady, lbm.ad.steady (one steady solve), lbm.update_cells,
 *   lbm.coupled.initial and lbm.coupled.update (one step of the coupled
 *   loop), lbm.mfc.hour and lbm.biofilm.step (the hourly model loop), lbm.srv.prepare, lbm.srv.step, lbm.srv.solo and
 *   lbm.srv.escalated (the server's threads).  The marker library
 *   (librocprofiler-sdk-roctx.so.1, else libroctx64.so.4) is opened with
 *   dlopen; LBM_ROCTX=<path> names another one.  If it cannot be opened,
 *   one message goes to stderr and nothing else changes.  Unset or 0: no
 *   ranges.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_NOT_CONVERGED = 1, /* max_iter reached; outputs hold the last state */
    LBM_STALLED = 2,       /* residual stopped improving above tol */
    LBM_EINVAL = -1,       /* bad argument, mask or geometry */
    LBM_ENOMEM = -2,       /* device or host allocation failed */
    LBM_EDEVICE = -3,      /* a HIP call failed (see lbm_last_error) */
    LBM_EDIVERGED = -4,    /* NaN/Inf, or |u| > 0.3 in the fluid */
    LBM_EBUSY = -5,        /* resource in use (server full, call in flight) */
    LBM_ENOTFOUND = -6     /* unknown ticket or field */
} lbm_status;

/* Population storage.  Arithmetic is FP64 for LBM_FP64 and
 * LBM_FP32_SHIFTED_F64 and FP32 for the others.  Shifted forms store
 * f_i - w_i rho0 (rho0 = 1) for the fluid and g_i - w_i c_ref (c_ref = c_in)
 * for the substrate, an exact change of variables that keeps the stored
 * values small. */
typedef enum {
    /* unshifted FP32 storage: each population at its full magnitude (~w_i
     * rho), whose round-to-nearest error recurs every step near a steady
     * state.  Fixed-step results hold the FP32 bounds, but converged fields
     * can drift past 1e-4 relative L2 (measured 1.4e-4 in velocity and
     * 5e-4 in concentration after 20,000 + 53,000 steps); it is kept for
     * comparison only.  LBM_FP32_SHIFTED is the FP32 form held to 1e-4. */
    LBM_FP32 = 0,
    /* FP32 arithmetic on FP32 shifted storage: the fastest FP32 form.  Its
     * rounding errors are deterministic functions of the state, and near a
     * steady state slow modes accumulate them: on the 1024 x 512 disc
     * medium at tau 0.6 (pore velocities to 0.23, density to 2.2) converged
     * fields differ from FP64 by 5e-4 relative L2 in velocity. */
    LBM_FP32_SHIFTED = 1,
    LBM_FP16_SHIFTED = 2,
    LBM_FP64 = 3,
    /* FP32 shifted storage -- the same bytes in memory as LBM_FP32_SHIFTED,
     * the same launches -- with each collision widened to FP64 and its
     * results rounded once to FP32: the FP32 form held to 1e-4 relative L2
     * against the FP64 fields on every workload. */
    LBM_FP32_SHIFTED_F64 = 4
} lbm_storage;

enum { LBM_FLUID = 0, LBM_SOLID = 1, LBM_WALL = 2, LBM_BIOFILM = 3 };

/* Substrate outlet: the paper names Dirichlet input and output (Sec. 2.1.2)
 * without an output value; the default is a zero-gradient outlet. */
typedef enum { LBM_OUT_ZERO_GRADIENT = 0, LBM_OUT_DIRICHLET = 1 } lbm_ad_outlet;

/* which solver a call addresses */
enum { LBM_SOLVER_FLUID = 0, LBM_SOLVER_AD = 1 };

/* fields for lbm_solver_get / lbm_solver_device_ptr */
typedef enum {
    LBM_FIELD_U = 0,       /* velocity, host double [dim][N]; 0 on blocked */
    LBM_FIELD_RHO = 1,     /* density, host double [N]; 0 on blocked */
    LBM_FIELD_C = 2,       /* concentration, host double [N]; 0 on SOLID/WALL */
    LBM_FIELD_CLASS = 3,   /* uint8 [N] */
    LBM_FIELD_LINKS_F = 4, /* fluid link mask, uint16 (2-D) / uint32 (3-D) [N] */
    LBM_FIELD_LINKS_C = 5, /* substrate link mask, uint8 [N] */
    LBM_FIELD_F = 6,       /* fluid populations f*, host double [Q][N], unshifted */
    LBM_FIELD_G = 7,       /* substrate populations g*, host double [Q][N], unshifted */
    LBM_FIELD_U_DEVICE = 8, /* device velocity buffer the AD solve reads (see device_ptr) */
    LBM_FIELD_DESC = 9     /* node descriptor words as the kernels read them, copied back
                            * from the device, uint32 [N] (diagnostic).  With qf, qa the
                            * fluid and substrate direction counts: bit 0 flow-domain
                            * node; bits 1..qf-1 blocked fluid pull sources; bits
                            * qf..qf+qa-2 blocked substrate pull sources (i = 1..qa-1);
                            * bit qf+qa-1 substrate-active (FLUID or BIOFILM); bit qf+qa
                            * BIOFILM; bit qf+qa+1 the column's reference node */
} lbm_field;

typedef struct {
    int32_t nx, ny, nz; /* nz = 1 for 2-D */
} lbm_grid;

typedef struct {
    double tau;           /* fluid relaxation time, > 1/2 */
    double u_in;          /* inlet plug velocity, |u_in| < 0.1 */
    double D;             /* substrate diffusivity, > 0 */
    double c_in;          /* inlet concentration (also the shift reference) */
    double k_sink;        /* first-order consumption on BIOFILM, 0 <= k < 1 */
    int32_t outlet;       /* lbm_ad_outlet */
    double c_out;         /* outlet value for LBM_OUT_DIRICHLET */
    int32_t storage;      /* lbm_storage */
    int32_t check_every;  /* residual cadence K, even and >= 2.  0: 100, or 1000
                             with FP16 storage, whose tile-mean residual carries
                             stochastic-rounding noise that falls with K: at
                             100 its floor sits above 1e-6 on most media */
    int32_t stall_checks; /* stall window in checks; 0: 1000, or with FP16 storage
                             the checks that span 10,000 steps (10 at K = 1000);
                             < 0 disables */
    double k_half;        /* 0: first-order sink k_sink C per step on BIOFILM nodes.
                             > 0: the Monod form of the consumption rate (Eq. 16,
                             its mediator factor folded into k_sink), k_sink C /
                             (C + k_half), C the concentration a step collides with;
                             needs k_sink < k_half.  Zero-initialised parameters keep
                             the first-order sink. */
    int32_t ad_lattice;   /* 0: D2Q5 (2-D) / D3Q7 (3-D) substrate with the linear
                             equilibrium.  1 (2-D only): the paper's substrate LBM,
                             D2Q9 with the equilibrium of Eq. 5 (C for rho); its
                             Dirichlet faces impose twice the even part of that
                             equilibrium, w_i c (1 + 9/2 (c.u)^2 - 3/2 u^2).  Not
                             offered by the server. */
} lbm_params;

typedef struct {
    int64_t iters;        /* steps taken by this solve */
    double residual;      /* residual at the last check (NaN if none) */
    int64_t checks;       /* residual checks performed */
    int64_t active_nodes; /* nodes the solver updates */
    double seconds;       /* wall time of the solve, device-synchronous */
    double kernel_ms;     /* HIP-event time over the step-kernel launches */
    int64_t launches;     /* step-kernel launches covered by kernel_ms.  A
                             launch advances two steps in 3-D (one with FP64
                             storage; FP16 storage takes its check and the
                             step before it as single steps); in 2-D two, or
                             three to four with FP32 storage on grids of at
                             least 256 tiles of 64 x 8 nodes */
    double mlups;         /* active-node updates per second / 1e6 */
    double gbps;          /* algorithmic bytes / kernel_ms: per active-node update,
                             each population read and written once, the 1-byte
                             node class, and (substrate) the velocity read */
    double flux_in;       /* per step, on the final state, FP64 */
    double flux_out;
    double sink_total;    /* substrate consumed per step (AD solves) */
} lbm_info;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_solver lbm_solver;

/* ---------------------------------------------------------------- misc */
const char *lbm_status_str(int status);
const char *lbm_version(void);

/* Context on GPU `device`.  hip_stream: a hipStream_t to enqueue on (e.g.
 * torch's current stream), or NULL for a stream the context creates (at the
 * default priority).  Errors: EINVAL (bad device), EDEVICE. */
lbm_status lbm_ctx_create(int device, void *hip_stream, lbm_ctx **out);
void lbm_ctx_destroy(lbm_ctx *ctx);
/* Last error text of this context ("" if none); valid until the next call. */
const char *lbm_last_error(const lbm_ctx *ctx);
/* hipStream_t the context enqueues on. */
void *lbm_ctx_stream(lbm_ctx *ctx);

/* ------------------------------------------------ geometry (host only) */
/* These run on the CPU with integer arithmetic and are bit-exact by
 * specification; they need no GPU and no context. */

/* Seeded random porous electrode (the paper's "random geometry", Sec. 3):
 * discs in the region [nx/4, 3nx/4) x [1, ny-1), radius drawn in
 * [r_min, r_max], placed until the SOLID share of the region reaches
 * solid_frac.  overlap = 0 keeps discs strictly apart; 1 allows overlap.
 * Draw order per attempt: centre x, centre y, radius (SplitMix64, integer
 * in [lo, hi] = lo + next mod (hi - lo + 1)).  cls_out: uint8 [N], written
 * whole (chassis rows WALL).  achieved (may be NULL): SOLID share reached.
 * EINVAL on bad sizes or when 10^6 attempts do not reach the target. */
typedef struct {
    int32_t r_min, r_max;
    double solid_frac;
    int32_t overlap;
} lbm_disc_params;
lbm_status lbm_geom_discs(lbm_grid g, const lbm_disc_params *p, uint64_t seed,
                          uint8_t *cls_out, double *achieved);

/* Seeded fibrous electrode (3-D): infinite cylinders through points of
 * [nx/4, 3nx/4) x [1, ny-1) x [1, nz-1) with integer directions in
 * [-4, 4]^3 \ {0} and radius in [r_min, r_max]; voxel p is SOLID iff
 * |(p - q) x d|^2 <= r^2 |d|^2.  Same stop rule and errors as discs. */
typedef struct {
    int32_t r_min, r_max;
    double solid_frac;
} lbm_fibre_params;
lbm_status lbm_geom_fibres(lbm_grid g, const lbm_fibre_params *p, uint64_t seed,
                           uint8_t *cls_out, double *achieved);

/* One-cell biofilm layer: every FLUID node with a SOLID lattice neighbour
 * (D2Q9 / D3Q19 directions) becomes BIOFILM, judged on the input mask. */
lbm_status lbm_biofilm_layer(lbm_grid g, uint8_t *cls_inout);

/* Link mask: bit i of word n is set iff the pull source n - c_i is inside
 * the grid and blocked for that solver.  which = LBM_SOLVER_FLUID writes
 * uint16 (2-D) or uint32 (3-D) words; LBM_SOLVER_AD writes uint8 words. */
lbm_status lbm_links(lbm_grid g, const uint8_t *cls, int which, void *links_out);

/* Link list: the set bits of lbm_links as ascending pairs
 * (n, i) -> out[2k] = n, out[2k+1] = i, for at most cap pairs.  Returns the
 * total count (which may exceed cap), or a negative lbm_status. */
int64_t lbm_link_list(lbm_grid g, const uint8_t *cls, int which, int64_t *out, int64_t cap);

/* 1 iff FLUID nodes of column 0 connect to column nx-1 along fluid-lattice
 * links (breadth-first search); 0 otherwise; negative on bad arguments. */
int lbm_percolates(lbm_grid g, const uint8_t *cls);

/* Flow domain (Sec. 2.1.1 boundary conditions on the Sec. 3 pore space):
 * out[n] = 1 iff node n is FLUID and a chain of fluid-lattice links between
 * FLUID nodes joins it to a FLUID node of the outlet column x = nx-1, else 0.
 * The fluid solver updates exactly these nodes.  FLUID nodes outside it (a
 * closed pore, or a pocket open to the inlet alone) carry no steady flow:
 * they report u = 0 and rho = 0, and the substrate solver treats them as
 * still fluid.  cls and out are host arrays of nx*ny*nz bytes; LBM_EINVAL on
 * null pointers or an empty grid. */
lbm_status lbm_flow_domain(lbm_grid g, const uint8_t *cls, uint8_t *out);

/* Biofilm growth pick of the coupled loop: among FLUID nodes with
 * 1 <= x <= nx-2 and a BIOFILM lattice neighbour (ascending n), weight
 * max(C, 0), pick the first whose running weight exceeds xi * W (W the
 * total); W = 0 picks candidate floor(xi * count).  C: host double [N].
 * Returns the node index, or -1 if there is no candidate. */
int64_t lbm_growth_pick(lbm_grid g, const uint8_t *cls, const double *C, double xi);

/* SplitMix64 stream of `seed`: out[k] = k-th output. */
void lbm_splitmix64(uint64_t seed, int64_t count, uint64_t *out);

/* ---------------------------------------------------- one-shot solves */
/* Steady fluid flow (Sec. 2.1.1) from rest on the mask cls (host uint8 [N]),
 * run until the residual -- the largest velocity change per step over the
 * check interval K (100; 1000 with FP16 storage), max |U(t) - U(t-K)| /
 * (K |u_in|) over FLUID nodes, evaluated at t = K, 2K, ... -- is <= tol, or
 * max_iter steps.
 * With LBM_FP16_SHIFTED storage the per-node changes are replaced by their
 * means over 64 x 4-node tiles (per z-plane): stochastic rounding injects
 * zero-mean momentum noise that would otherwise set a residual floor above
 * ordinary tolerances; the mean keeps the smooth evolution of the flow.
 * (The substrate residual below is treated the same way.)
 * Also stops on NaN/Inf or |u| > 0.3 (EDIVERGED), and (STALLED) after
 * stall_checks consecutive checks that set neither a new maximum of the
 * residual nor a new minimum since its last maximum -- a residual flat on a
 * round-off floor above tol; a transient that rises before it decays does
 * not count as a stall.  u_out: host double
 * [dim][N] (0 on blocked nodes).  info may be NULL. */
lbm_status lbm_fluid_steady(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, double tau,
                            double u_in, double tol, int64_t max_iter, int storage,
                            double *u_out, lbm_info *info);

/* Steady substrate field (Sec. 2.1.2) in the frozen velocity u (host double
 * [dim][N]), started from equilibrium at c_in; residual
 * max |C(t) - C(t-K)| / (K |c_in|) over FLUID and BIOFILM nodes.
 * c_field: host double [N] (0 on SOLID/WALL).  info may be NULL. */
lbm_status lbm_ad_steady(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const double *u,
                         double D, double c_in, double k_sink, int outlet, double c_out,
                         double tol, int64_t max_iter, int storage, double *c_field,
                         lbm_info *info);

/* Device-pointer forms of the two one-shot solves, for callers that hold
 * the mask and the fields in device memory (e.g. torch tensors): the same
 * arguments and results, but cls (uint8 [N]), u (double [dim][N]), u_out
 * and c_field are device pointers on the context's device.  The mask and
 * the input velocity are read back to the host once (geometry and link
 * words are built on the host); the outputs are written device to device
 * on the context's stream, which is synchronised before return. */
lbm_status lbm_fluid_steady_dev(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, double tau,
                                double u_in, double tol, int64_t max_iter, int storage,
                                double *u_out, lbm_info *info);
lbm_status lbm_ad_steady_dev(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const double *u,
                             double D, double c_in, double k_sink, int outlet, double c_out,
                             double tol, int64_t max_iter, int storage, double *c_field,
                             lbm_info *info);

/* No-allocation form of lbm_fluid_steady_dev, for callers that cannot
 * allocate device memory (code around stream capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments (device pointers) and
 * the same results bit for bit: the same kernels in the same order.  Every
 * device buffer of the solve is carved from a device scratch array of
 * LBM_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it has run
 * this call on, until the process ends; the call makes no device or pinned
 * allocation and creates no events.  The solve needs about 90 bytes per
 * node in 2-D with FP32 storage (about 700,000 nodes fit; 170 with FP64) and
 * about 190 in 3-D: EINVAL, with the sizes in lbm_last_error, if the grid
 * does not fit.  Calls that overlap on one GPU share its array and race:
 * the caller serialises them.  info->kernel_ms and info->gbps are 0 (no
 * events).  The context's stream is synchronised before return. */
#define LBM_NOALLOC_SCRATCH_BYTES (64u << 20)
lbm_status lbm_fluid_steady_dev_noalloc(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, double tau,
                                        double u_in, double tol, int64_t max_iter, int storage,
                                        double *u_out, lbm_info *info);

/* ----------------------------------------------------- stateful solver */
/* A solver owns the device state of one domain: both solvers' populations
 * (A/B pull buffers), the velocity the substrate solve reads, the node
 * descriptors and the residual/flux scratch.  Validates the mask (EINVAL,
 * including a medium that does not percolate) and parameters; ENOMEM if
 * the device buffers do not fit. */
lbm_status lbm_solver_create(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls,
                             const lbm_params *p, lbm_solver **out);
void lbm_solver_destroy(lbm_solver *s);

/* Steady solves.  warm = 0 starts the fluid at rest (rho = 1, u = 0) and
 * the substrate at equilibrium with c_in in the current velocity; warm = 1
 * continues from the retained state.  The fluid solve ends by exporting
 * its velocity to the buffer the substrate solve reads.  info may be NULL. */
lbm_status lbm_solver_fluid(lbm_solver *s, double tol, int64_t max_iter, int warm,
                            lbm_info *info);
lbm_status lbm_solver_ad(lbm_solver *s, double tol, int64_t max_iter, int warm,
                         lbm_info *info);

/* Exactly nsteps steps of one solver with no residual checks (cold = 1:
 * initialise first).  kernel_ms (may be NULL): HIP-event time over the
 * launches.  For the fluid this does not export the velocity; call
 * lbm_solver_export_u for that. */
lbm_status lbm_solver_steps(lbm_solver *s, int which, int64_t nsteps, int cold,
                            double *kernel_ms);
/* Per-launch timing: the launches covering nsteps steps of one solver
 * (state must be initialised; in 2-D a launch advances two steps, four
 * with FP32 storage on grids of at least 512 tiles of 64 x 16 nodes, and
 * nsteps is rounded up to whole launches), each bracketed by its own pair
 * of HIP events on
 * the context's stream; *avg_ms = mean event-to-event time per launch. */
lbm_status lbm_solver_time_steps(lbm_solver *s, int which, int nsteps, double *avg_ms);
/* Recompute the substrate solve's velocity from the stored fluid state. */
lbm_status lbm_solver_export_u(lbm_solver *s);
/* Replace the substrate solve's velocity: host double [dim][N]. */
lbm_status lbm_solver_set_u(lbm_solver *s, const double *u);

/* Copy a field to host memory (layout and type in lbm_field). */
lbm_status lbm_solver_get(lbm_solver *s, int field, void *dst);
/* Set populations from host double [Q][N] (unshifted values), field
 * LBM_FIELD_F or LBM_FIELD_G; blocked nodes are zeroed. */
lbm_status lbm_solver_put(lbm_solver *s, int field, const double *src);
/* Device pointer and byte size of LBM_FIELD_U_DEVICE (float [dim][N], or
 * double for LBM_FP64), valid until the solver is destroyed. */
lbm_status lbm_solver_device_ptr(lbm_solver *s, int field, void **ptr, size_t *bytes);

/* FP64 fluxes per step on the current states: out[0] fluid inflow,
 * out[1] fluid outflow, out[2] substrate inflow, out[3] substrate outflow,
 * out[4] substrate consumed on BIOFILM (deterministic two-pass sums). */
lbm_status lbm_solver_fluxes(lbm_solver *s, double *out5);

/* Change node classes (e.g. FLUID -> BIOFILM as the biofilm grows,
 * Sec. 2.3).  idx: host int64 [n] node indices, new_cls: host uint8 [n].
 * Nodes that become blocked for a solver lose its populations; nodes that
 * become active start from rest (fluid) or equilibrium at c_in (substrate).
 * Link masks of the neighbourhood are rebuilt.  EINVAL if a change breaks
 * the mask rules or percolation (the solver is then left unchanged). */
lbm_status lbm_solver_update_cells(lbm_solver *s, const int64_t *idx, const uint8_t *new_cls,
                                   int64_t n);

/* Checkpoint: the stored populations of both solvers, the velocity buffer
 * and the class mask, with a header naming grid, storage and parameters.
 * Restoring it resumes bit-exactly (the kernels are deterministic). */
lbm_status lbm_solver_state_size(lbm_solver *s, size_t *bytes);
lbm_status lbm_solver_get_state(lbm_solver *s, void *dst, size_t bytes);
lbm_status lbm_solver_put_state(lbm_solver *s, const void *src, size_t bytes);

/* Coupled biofilm loop (model loop of Sec. 2 with Sec. 2.3's re-solves;
 * simplified growth): cold fluid and substrate solves, then n_updates
 * times pick a new biofilm cell with lbm_growth_pick on the current C and
 * xi[m] (host double [n_updates] in [0, 1)), mark it BIOFILM, re-converge
 * fluid then substrate warm to tol (max_iter each), and add that update's
 * sink_total to *J_accum (FP64).  picked: int64 [n_updates]; J: double
 * [n_updates + 1] (J[0] before any growth); iters_fluid / iters_ad: int64
 * [n_updates + 1].  Any output pointer except J_accum may be NULL. */
lbm_status lbm_coupled_run(lbm_solver *s, int n_updates, const double *xi, double tol,
                           int64_t max_iter, int64_t *picked, double *J, double *J_accum,
                           int64_t *iters_fluid, int64_t *iters_ad);

/* ------------------------------------------------- bio-electrochemistry */
/* The MFC outputs of Sec. 2.2 (Eqs. 14-21), computed once per model
 * interval (one hour, Sec. 3) after the two steady solves (model loop of
 * Sec. 2, step 4).  Every cell holding biomass carries its biomass
 * concentration C_bio and its oxidised intracellular mediator M_ox (per unit
 * biomass; M_red = M_total - M_ox, Eq. 14).  One interval, from the
 * solver's current substrate field C:
 *   - double-Monod consumption (Eq. 16) q_a = q_max S/(S + K_s) *
 *     M_ox/(M_ox + K_Mox), with S = c_scale * max(C, 0) in mg/L;
 *   - the mediator balance of Eq. 15 over the interval with q_a and the
 *     current taken at the new state: per cell M = M0 - Y q_a(M) dt +
 *     gamma I dt / (m F B), B = sum of C_bio * V_a / N over the cells (the
 *     total biomass, N the lattice cells), capped at M_total;
 *   - the cell current of Eq. 20 with the overpotentials of Eqs. 18-19 at
 *     the biomass-weighted mean mediator: the unique root of I = max(0,
 *     I_20(I)) on [0, E0 / (R_int + R_ext)], by bisection (at most 80
 *     halvings, to adjacent doubles).
 * Units: mg, L, day (q_max), hour (dt_hours), A, V, ohm, m^2, K. */
typedef struct {
    double q_max;     /* maximum consumption rate, mg substrate / (mg biomass day) */
    double K_s;       /* substrate half-saturation, mg/L, > 0 */
    double M_total;   /* total intracellular mediator, mg mediator / mg biomass, > 0 */
    double K_Mox;     /* oxidised-mediator half-saturation, same unit, > 0 */
    double Y;         /* mediator yield, mg mediator / mg substrate */
    double gamma;     /* mediator molar mass, mg / mol */
    double m;         /* electrons per mediator reduction */
    double I0;        /* exchange current density, A / m^2 */
    double E0;        /* open-circuit voltage, V */
    double R_ext;     /* external load, ohm */
    double R_int;     /* internal resistance, ohm */
    double A_a;       /* anode surface area, m^2 */
    double V_a;       /* anode compartment volume, L */
    double T;         /* temperature, K */
    double eps;       /* current bound at low M_red (Eq. 20), mg mediator / mg biomass, >= 0 */
    double C0_bio;    /* biomass given to BIOFILM cells when none is passed, mg/L */
    double c_scale;   /* mg/L per lattice concentration unit */
    double dt_hours;  /* model interval, h */
} lbm_bio_params;

typedef struct {
    double I_cell;    /* A */
    double V_cell;    /* load voltage I R_ext, V (the left side of Eq. 17) */
    double V_total;   /* I (R_int + R_ext), V (Eq. 21) */
    double n_conc;    /* Eq. 18, V (+inf when no mediator is reduced) */
    double n_act;     /* Eq. 19, V */
    double M_ox;      /* biomass-weighted mean after the interval */
    double M_red;     /* M_total - M_ox */
    double biomass;   /* B, mg */
    double q_total;   /* substrate consumed at the new state, mg / h */
    int32_t n_cells;  /* cells holding biomass */
    int32_t root_iters; /* bisection halvings taken */
} lbm_bio_out;

typedef struct lbm_bio lbm_bio;
enum { LBM_BIO_CBIO = 0, LBM_BIO_MOX = 1 };

/* Attach a bio-electrochemical state to solver s (which must outlive it).
 * c_bio: host double [N] biomass in mg/L, >= 0, nonzero only on BIOFILM
 * nodes, or NULL for C0_bio on every BIOFILM node.  m_ox: host double [N]
 * in [0, M_total] where c_bio > 0, or NULL for M_total (fully oxidised).
 * EINVAL for invalid parameters or fields; ENOMEM if device memory is
 * short.  Device memory: 28 bytes per biomass cell plus 8 per node. */
lbm_status lbm_bio_create(lbm_solver *s, const lbm_bio_params *p, const double *c_bio,
                          const double *m_ox, lbm_bio **out);
/* One interval on the solver's current substrate state (EINVAL before any
 * substrate solve).  Updates M_ox of every biomass cell; *out may be NULL.
 * Synchronises the solver's stream. */
lbm_status lbm_bio_step(lbm_bio *b, lbm_bio_out *out);
/* Field LBM_BIO_CBIO or LBM_BIO_MOX as host double [N] (0 where no biomass). */
lbm_status lbm_bio_get(lbm_bio *b, int field, double *dst);
/* Set C_bio and M_ox of n nodes (host arrays; the same rules as create, and
 * c_bio = 0 removes a cell's biomass).  Call after growth has changed the
 * solver's cells. */
lbm_status lbm_bio_set(lbm_bio *b, const int64_t *nodes, const double *c_bio, const double *m_ox,
                       int64_t n);
void lbm_bio_destroy(lbm_bio *b);

/* ------------------------------------------------------ biofilm formation */
/* The agent-based biofilm of Sec. 2.3, once per model interval after the
 * bio-electrochemical update (model loop of Sec. 2, step 5), on the
 * solver's current substrate field and the bio state's biomass C_bio and
 * mediator M_ox:
 *   1. attachment: min(k_ata, front size) cells drawn without replacement
 *      (partial Fisher-Yates shuffle of the front in ascending node order)
 *      get C_bio = C0_bio and M_ox = M_total.  The front is the FLUID nodes
 *      with a SOLID neighbour among the fluid lattice's directions, outside
 *      the inlet and outlet columns;
 *   2. growth: C_bio += C_bio Y_bio q_a dt (q_a of Eq. 16, per day, at the
 *      current substrate and mediator; M_ox per unit biomass unchanged);
 *   3. spreading, one ascending pass over the nodes: a node whose C_bio
 *      exceeds C_max when visited passes fr_spr C_bio, with its M_ox, to a
 *      free neighbour drawn uniformly (free: FLUID outside the inlet and
 *      outlet columns).  With none free, a loop-erased random walk through
 *      BIOFILM nodes (uniform direction per step; a step into SOLID, WALL or
 *      off the grid is spent in place) finds a free node within max_walk
 *      steps, the biomass and mediator along its path move one node outward,
 *      and the initial node's neighbour on the path receives the share;
 *      otherwise nothing spreads.
 * Every node that gains biomass becomes BIOFILM (lbm_solver_update_cells).
 * Random numbers: the SplitMix64 stream of `seed` in the order above,
 * u = (x >> 11) 2^-53, an index in [0, m) is floor(u m). */
typedef struct {
    int32_t k_ata;     /* front cells attached per interval (Table 1: 200) */
    double C_max;      /* spreading threshold, mg/L (512.5) */
    double fr_spr;     /* fraction of the biomass a spreading moves (0.4) */
    int32_t max_walk;  /* random-walk steps before a spreading is given up */
    double Y_bio;      /* biomass per consumed substrate, mg/mg (not in Table 1;
                          1: the growth rate per unit biomass is q_a) */
} lbm_biofilm_params;

typedef struct {
    int32_t attached;    /* cells attached */
    int32_t spread;      /* spreading events */
    int32_t walks;       /* spreading attempts that needed a random walk */
    int32_t abandoned;   /* walks that found no free node */
    int32_t new_biofilm; /* nodes turned BIOFILM */
    int32_t cells;       /* nodes holding biomass afterwards */
    double biomass;      /* mg, afterwards */
} lbm_biofilm_stats;

/* One interval of attachment, growth and spreading.  EINVAL for bad
 * parameters, before any substrate solve, or when the new BIOFILM nodes
 * would stop the mask from percolating (nothing is changed then).
 * *st may be NULL. */
lbm_status lbm_biofilm_step(lbm_bio *b, const lbm_biofilm_params *p, uint64_t seed,
                            lbm_biofilm_stats *st);

typedef struct {
    int32_t status_fluid, status_ad;  /* lbm_status of the two solves */
    int64_t iters_fluid, iters_ad;
    int64_t nodes_fluid, nodes_ad;    /* nodes each solve updated per step */
    double seconds_solves;            /* wall time of the two solves */
    double seconds_bio;               /* of lbm_bio_step */
    double seconds_film;              /* of lbm_biofilm_step */
    lbm_bio_out bio;
    lbm_biofilm_stats film;
} lbm_mfc_interval;

/* The model loop of Sec. 2 for n_hours intervals (one hour each, Sec. 3):
 * fluid and substrate solves to tol (cold in the first interval, warm
 * after), lbm_bio_step, then lbm_biofilm_step with the interval's seed,
 * output h of the SplitMix64 stream of `seed`.  series: n_hours records.
 * Stops at the first error (a diverged solve, or growth that would close
 * the flow path: EINVAL), returning it; earlier records stay valid. */
lbm_status lbm_mfc_run(lbm_bio *b, const lbm_biofilm_params *p, int n_hours, uint64_t seed,
                       double tol, int64_t max_iter, lbm_mfc_interval *series);

/* ------------------------------------------------------------- serving */
/* Continuous batching of 2-D steady solves (D2Q9 fluid, then D2Q5
 * substrate in the exported velocity) -- the model loop's steps 2 and 3
 * (Sec. 2) for many independent domains at once, e.g. electrode-geometry
 * or parameter sweeps.  Requests are admitted in ticket order while a slot
 * is free and their device footprint (lbm_server_footprint) fits the pool;
 * every admitted request's populations stay resident and all of them are
 * stepped by the same kernel launches, each in its own phase, in chunks of
 * check_every steps captured once as HIP graphs (two steps per launch over
 * 64 x 4 tiles; for FP32 and FP32-shifted storage, while the batch holds at
 * least 256 tiles of 64 x 16 nodes and no solo lane is solving, four steps
 * per launch over such tiles, two in the first two launches when
 * check_every / 4 is odd -- the choice is made per chunk and does not
 * change any result).  The largest
 * request the server takes is bounded by pool_bytes and by
 * 2^31 / (64 * tile height) tiles in flight.  A request's arithmetic
 * is that of lbm_solver_fluid followed by lbm_solver_ad (cold, same
 * storage, same check cadence and stall window): its results are bit-equal
 * to that single solve and do not depend on what else is in flight.
 * max_iter is rounded up to a multiple of check_every.  A fluid solve that
 * ends NOT_CONVERGED or STALLED still proceeds to the substrate solve; one
 * that diverges ends the request (c is then 0).
 * Besides the batch the server runs solo lanes: host threads that each
 * solve one request at a time with a single-domain solver
 * (lbm_solver_fluid, then lbm_solver_ad, cold) on a stream of their own,
 * concurrently with the batch.  It takes (a) requests of at least
 * solo_nodes nodes, which fill the GPU on their own and there run the
 * single solver's wider multi-step launches, in the server's storage and
 * cadence -- bit-equal to what the batch would return -- and (b) with
 * escalate set and reduced storage (FP16 or unshifted FP32), every request
 * whose solves in that storage (batched or solo) did not both end OK: it is
 * solved again from rest with FP32-shifted storage (cadence and stall
 * window the lbm_params defaults), and that solve's result is returned,
 * marked in `lane`, with the first attempt's status and step counts
 * alongside.
 * All lbm_server_* calls are thread-safe. */
typedef struct lbm_server lbm_server;

typedef struct {
    size_t pool_bytes;     /* device memory for request state, one allocation */
    int32_t max_slots;     /* requests on the device at once, 1..64 (32 if 0) */
    int32_t storage;       /* any but LBM_FP64 */
    int32_t check_every;   /* K: steps per chunk and residual cadence, a multiple of 4
                              (if 0: 100, or 1000 with FP16 storage, as lbm_params) */
    int32_t stall_checks;  /* as lbm_params */
    int32_t inflight;      /* chunks enqueued ahead of the decisions, 1..6 (2 if 0) */
    int32_t prep_threads;  /* host threads that build masks, 1..16 (2 if 0) */
    int32_t direct_launch; /* 1: launch each chunk's kernels directly instead of the graph */
    int32_t escalate;      /* 1: re-solve failed reduced-storage requests in FP32-shifted
                              storage on the solo lane (see above) */
    int64_t solo_nodes;    /* requests of at least this many nodes go to the solo lanes
                              (0: 262,144, where a request fills the GPU alone;
                              < 0: none); such requests need not fit the pool */
    int32_t solo_lanes;    /* solo-lane threads, 1..8 (2 if 0) */
} lbm_server_cfg;

typedef struct {
    int32_t nx, ny;        /* 2-D grid; the mask rules of lbm_solver_create apply */
    const uint8_t *cls;    /* host uint8 [nx * ny] classes (copied), or NULL to build */
    lbm_disc_params discs; /* ... discs with lbm_geom_discs(discs, seed) */
    uint64_t seed;
    int32_t layer;         /* 1: then add lbm_biofilm_layer */
    double tau, u_in, D, c_in, k_sink;  /* as lbm_params */
    int32_t outlet;
    double c_out;
    double tol;            /* both solves */
    int64_t max_iter;      /* per solve */
    uint64_t user;         /* caller's tag, returned in the result */
    double k_half;         /* as lbm_params */
} lbm_request;

typedef struct {
    uint64_t ticket, user;
    int32_t status;        /* EINVAL/ENOMEM on a bad request, EDEVICE, else the worse
                              of the two solves (EDIVERGED > NOT_CONVERGED > STALLED > OK) */
    int32_t status_fluid, status_ad;
    int32_t nx, ny;
    int64_t iters_fluid, iters_ad;
    double residual_fluid, residual_ad;
    double flux[5];        /* as lbm_solver_fluxes, on the final states */
    int64_t active_fluid, active_ad; /* nodes each solve updates */
    double t_submit, t_admit, t_finish; /* seconds on the server clock */
    const float *u;        /* [2][N] velocity, owned by the server until released */
    const float *c;        /* [N] concentration (0 on SOLID/WALL) */
    char message[96];      /* reason of a rejection */
    int32_t lane;          /* LBM_LANE_BATCH, LBM_LANE_SOLO or LBM_LANE_ESCALATED */
    int32_t first_status;  /* escalated: overall status of the batched attempt */
    int64_t first_iters_fluid, first_iters_ad; /* escalated: its step counts */
} lbm_result;

enum { LBM_LANE_BATCH = 0, LBM_LANE_SOLO = 1, LBM_LANE_ESCALATED = 2 };

typedef struct {
    int64_t submitted, finished, rejected, active, queued, chunks;
    uint64_t pool_bytes, pool_used, pool_peak;
    double lattice_updates; /* active-node updates of the finished requests */
    double busy_seconds;    /* wall time with work on the device (either lane) */
    double clock;           /* seconds since creation */
    int64_t solo, escalated; /* finished requests solved on the solo lane, of which
                                escalated */
    int64_t chunks_wide;   /* chunks of `chunks` taken over 64 x 16 tiles */
} lbm_server_stats_t;

/* Device bytes one request of this size takes from the pool. */
size_t lbm_server_footprint(int32_t nx, int32_t ny, int32_t storage);
/* Allocates the pool and starts the worker threads on ctx's device (the
 * server has its own stream).  EINVAL on a bad configuration, ENOMEM.
 * Tuning through the environment: LBM_SERVED_TILE_Y=4 (read once per
 * process) keeps every chunk on paired 64 x 4 launches;
 * LBM_SERVED_WIDE_MIN_TILES (read by each create) sets the table size, in
 * 64 x 16 tiles, from which FP32 chunks take the wide form (256). */
lbm_status lbm_server_create(lbm_ctx *ctx, const lbm_server_cfg *cfg, lbm_server **out);
/* Queue a request (copied).  EINVAL (see lbm_server_error) for bad
 * parameters or a batch request larger than the pool; mask problems found later
 * (a geometry that cannot be built or does not percolate) come back as a
 * result with status EINVAL. */
lbm_status lbm_server_submit(lbm_server *s, const lbm_request *r, uint64_t *ticket);
/* Up to max finished results, waiting up to wait_s seconds for the first.
 * Each result's arrays stay valid until lbm_result_release. */
lbm_status lbm_server_poll(lbm_server *s, lbm_result *out, int max, int *n_out, double wait_s);
void lbm_result_release(lbm_server *s, lbm_result *r);
/* Wait until every submitted request has finished (timeout_s <= 0: no
 * limit; EBUSY when it expires). */
lbm_status lbm_server_drain(lbm_server *s, double timeout_s);
lbm_status lbm_server_stats(lbm_server *s, lbm_server_stats_t *out);
/* Text of the last submit error or of a device failure. */
const char *lbm_server_error(lbm_server *s);
/* Stops the threads (queued requests are dropped), waits for the device and
 * frees everything, including unreleased results. */
void lbm_server_destroy(lbm_server *s);

/* ------------------------------------------------------------ diagnostics */
/* Device-to-device copy of `bytes` bytes by a plain streaming kernel, reps
 * times, HIP-event timed: *gbps = 2 * bytes / time (read + write),
 * *ms_per_copy = average duration. */
lbm_status lbm_copy_bandwidth(lbm_ctx *ctx, size_t bytes, int reps, double *gbps,
                              double *ms_per_copy);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */

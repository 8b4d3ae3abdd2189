// lbm_kernels.h -- host-side launch interface of the gfx950 kernels.
//
// The kernels themselves live in kernels.hip; this header is what the
// solver runtime (solver.cpp, api.cpp) calls.  All launches are
// asynchronous on the given stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbmk {

enum { ST_F32 = 0, ST_F32S = 1, ST_F16S = 2, ST_F64 = 3, ST_F32X = 4 };
enum { MODE_PLAIN = 0, MODE_CHECK = 2 };
enum { STOP_RUN = 0, STOP_OK = 1, STOP_STALLED = 2, STOP_DIVERGED = 3, STOP_MAXITER = 4 };

// Per-solve control block in device memory.  The step kernels read `stop`
// first and return at once when it is set, so the host may enqueue steps
// ahead of the residual decision without changing the state past the stop.
struct Ctrl {
    unsigned long long res_bits;  // max residual of the current check (FP64 bits)
    unsigned long long umax_bits; // max |u| of the current check (FP64 bits)
    double tol;
    double best;                  // smallest residual so far
    double r_last;                // residual of the latest check
    long long t;                  // steps covered by completed checks
    long long t_stop;             // step at which stop was decided
    long long checks;
    int stop;                     // STOP_*
    int since_best;               // checks since the last new minimum
    int window;                   // stall window in checks (<= 0: off)
    int is_fluid;                 // apply the |u| > 0.3 divergence test
    int K;                        // steps per check
    int nparts;                   // blocks of the step grid
    double peak;                  // largest residual so far
    unsigned long long *part;     // per-block maxima [2 * nparts] of a check step
    long long t_max;              // MAXITER stop once t >= t_max
};

// Domain geometry as the kernels see it.  Tiles are 64 x 4 nodes (one
// 256-thread block, four wave64 rows) of one z-plane.
struct Geo {
    int nx, ny, nz;
    int ntx, nty;    // tiles along x and y
    int ntiles;      // ntx * nty * nz
    long long N;     // nx * ny * nz
};

Geo make_geo(int nx, int ny, int nz);

// Layout code of substrate calls whose descriptor words are the D2Q9
// substrate's own (16-bit, no fluid bits; the "dim" argument of substrate
// functions is 2, 3 or this)
enum { LAY_2D_AD9 = 4 };

// Descriptor word per node (uint16 in 2-D, uint32 in 3-D):
//   bit 0                 node is in the flow domain (FLUID and linked to
//                         the outlet column: the fluid solver updates it)
//   bits 1..QF-1          fluid pull source n - c_i is blocked (bounce back)
//   bits QF..QF+QA-2      substrate pull source n - c_i is blocked (i = 1..QA-1)
//   bit  QF+QA-1          node is FLUID or BIOFILM (substrate solver updates it)
//   bit  QF+QA            node is BIOFILM (consumption)
//   bit  QF+QA+1          node samples its column's reference (one flow-
//                         domain node per x, nearest the middle of the
//                         cross-section)
inline int desc_ad_link_bit(int qf, int i) { return qf - 1 + i; }
inline int desc_ad_active_bit(int qf, int qa) { return qf - 1 + qa; }
inline int desc_biofilm_bit(int qf, int qa) { return qf + qa; }
inline int desc_ref_bit(int qf, int qa) { return qf + qa + 1; }

// Shifted storage keeps h_i = f_i - w_i R(x): R is a per-column reference
// (density for the fluid, concentration for the substrate), one float per
// x.  FP32 shifted storage keeps R constant (1, or c_ref); FP16 storage
// moves it at every check to the value at the column's sample node, so that
// the stored values stay small where the density or concentration drifts
// along the flow.  Any R is exact: a step un-shifts each pulled value with
// the reference of its source column and shifts its results with the
// reference of the buffer it writes.  Protocol per chunk of K steps: step 0
// reads with R_cur and writes with R_next; then R_cur <- R_next (roll);
// steps 1..K-1 read and write with R_cur; the check step stores the new
// sample values into R_next.

struct FluidArgs {
    const void *src;
    void *dst;
    const void *desc;
    void *uprev;    // compute-type [dim][N] velocity saved at the previous check
    Ctrl *ctrl;
    Geo g;
    double omega;   // 1 / tau
    double u_in;
    double inv_uin; // 1 / (K |u_in|): residual scale
    int streaming_stores; // 1: non-temporal population stores (large domains)
    unsigned int step;    // step counter of this solver (stochastic rounding)
    const float *ref_src; // column reference of src (FP16 storage only)
    const float *ref_dst; // column reference of dst
    float *ref_out;       // check steps: sample values for the next reference
    int zseg;             // two-step 3-D launches: output planes per block
    int ty3;              // two-step 3-D launches: column height (8 or 16)
};

struct AdArgs {
    const void *src;
    void *dst;
    const void *desc;
    const void *u;  // compute-type [dim][N] frozen velocity
    void *cprev;    // compute-type [N] concentration saved at the previous check
    Ctrl *ctrl;
    Geo g;
    double omega;   // 1 / tau_D
    double cin_s;   // c_in - shift reference (0 reference when unshifted)
    double cout_s;  // c_out - shift reference
    double c_ref;   // shift reference (0 when unshifted)
    double k_sink;  // consumption on BIOFILM: k_sink C, or k_sink C / (C + k_half)
    double k_half;  // Monod half-saturation concentration (0: first order)
    double inv_cin; // 1 / (K |c_in|): residual scale
    int outlet;     // 0 zero-gradient, 1 Dirichlet
    int streaming_stores; // 1: non-temporal population stores (large domains)
    unsigned int step;    // step counter of this solver (stochastic rounding)
    double c_in, c_out;   // unshifted boundary values
    const float *ref_src; // column references, as in FluidArgs
    const float *ref_dst;
    float *ref_out;
    int zseg;             // two-step 3-D launches: output planes per block
    int ty3;              // two-step 3-D launches: column height (8 or 16)
};

size_t storage_bytes(int storage);  // bytes per stored population
size_t compute_bytes(int storage);  // bytes per compute-type value
bool storage_shifted(int storage);
bool storage_moving_ref(int storage); // column reference updated at checks

// ref[0..n) = v
hipError_t ref_fill(float *ref, int n, float v, hipStream_t st);
// cur[0..n) = next[0..n) unless the solve has stopped (ctrl->stop)
hipError_t ref_roll(const Ctrl *ctrl, float *cur, const float *next, int n, hipStream_t st);

hipError_t fluid_step(int dim, int storage, int mode, const FluidArgs &a, hipStream_t st);
hipError_t ad_step(int dim, int storage, int mode, const AdArgs &a, hipStream_t st);
// Two steps in one launch (2-D only): steps a.step and a.step + 1, the
// check (MODE_CHECK) on the second; src -> dst like one step.  The
// intermediate state stays in LDS in the compute type: FP64 and FP32
// results equal two single steps (up to how the compiler contracts
// multiply-adds in the two code paths); FP16 storage skips one rounding.
hipError_t fluid_step2(int storage, int mode, const FluidArgs &a, hipStream_t st);
// lay: 2 (D2Q5 substrate) or LAY_2D_AD9 (D2Q9 substrate, its own words)
hipError_t ad_step2(int lay, int storage, int mode, const AdArgs &a, hipStream_t st);
// Blocks (tiles) of a two-step launch; per-block check maxima need this many
// slots (never more than g.ntiles).  pair_tiles(g): 64 x 4 tiles;
// pair_tiles(g, ty): 64 x ty tiles.
int pair_tiles(const Geo &g);
int pair_tiles(const Geo &g, int ty);
// Tile height fluid_step2 and ad_step2 use for this storage and grid: 16
// (1024-thread blocks) on grids with at least 512 such tiles, 8 (512
// threads) on grids with at least 256 such tiles, else 4 (256 threads);
// always 4 with FP16 storage (tile means).
int pair_ty(int storage, const Geo &g);
// Tile height of the multi-step launches: 16 or 8 by the same tile counts,
// 0 on smaller grids.
int multi_ty(const Geo &g);
// Most steps per launch of either solver in 2-D: 4 (fluid_stepN / ad_stepN)
// on grids that take the wide or middle tiles, except FP64; else 2.
int fluid_launch_steps(int storage, const Geo &g);
// ns = 3 or 4 fluid steps per launch (2-D; 64 x multi_ty tiles and an
// in-place LDS region, as fluid_launch_steps allows); the check, if any, on
// the last.  FP16 storage: ns = 4, plain, equal source and destination
// references only (two paired launches fused; see kernels.hip).
hipError_t fluid_stepN(int storage, int mode, int ns, const FluidArgs &a, hipStream_t st);
// ns = 3 or 4 substrate steps per launch, under the same conditions (lay as
// ad_step2).
hipError_t ad_stepN(int lay, int storage, int mode, int ns, const AdArgs &a, hipStream_t st);

// Two steps in one launch (3-D, compute types of 4 bytes): a block marches
// along z over a.zseg output planes of a 32 x a.ty3 column, steps a.step and
// a.step + 1, src -> dst like one step; the check (MODE_CHECK) on the
// second, not for storage with tile means.  FP32 results equal two single
// steps up to rounding order; FP16 storage skips one rounding.
hipError_t fluid_step3d2(int storage, int mode, const FluidArgs &a, hipStream_t st);
hipError_t ad_step3d2(int storage, int mode, const AdArgs &a, hipStream_t st);
// column height and output planes per block the grid's two-step 3-D
// launches take by default, and the blocks (per-block check maxima) of such
// a launch
int z3_tile_y(const Geo &g);
int z3_planes_per_block(const Geo &g, int ty, int blocks_per_cu);
int z3_blocks(const Geo &g, int zseg, int ty);

// f = rest state on FLUID nodes, 0 elsewhere.
hipError_t fluid_init(int dim, int storage, void *f, const void *desc, const Geo &g,
                      hipStream_t st);
// g = equilibrium at c_init in velocity u on active nodes, 0 elsewhere.
hipError_t ad_init(int dim, int storage, void *gp, const void *desc, const void *u,
                   const Geo &g, double c_init, double c_ref, hipStream_t st);

// In the calls below `ref` is the column reference the stored state is
// shifted by (float [nx]; ignored, and may be null, for unshifted storage).

// Velocity (and density) of a stored fluid state.  out_double selects the
// output type (double, else the compute type); RHO may be null.
hipError_t fluid_export(int dim, int storage, const void *f, const void *desc, const Geo &g,
                        const float *ref, void *U, void *RHO, int out_double, hipStream_t st);
// Consumption on BIOFILM nodes per step: k C (first order, kh = 0) or the
// Monod form k C / (C + kh), C the concentration the step collides with.
struct Sink {
    double k, kh;
};

// Concentration of a stored substrate state (double, or the compute type):
// the concentration of the step that produced it (the sink inverted).
hipError_t ad_export(int dim, int storage, const void *gp, const void *desc, const Geo &g,
                     const float *ref, Sink sink, void *C, int out_double, hipStream_t st);

// Stored populations <-> unshifted double [Q][N] (0 on inactive nodes).
hipError_t pops_export(int which, int dim, int storage, const void *h, const void *desc,
                       const Geo &g, const float *ref, double *out, hipStream_t st);
hipError_t pops_import(int which, int dim, int storage, void *h, const void *desc,
                       const Geo &g, const float *ref, const double *in, hipStream_t st);

// Set the populations of the listed nodes to the unshifted values vals[i].
hipError_t pops_set_nodes(int which, int dim, int storage, void *h, const Geo &g,
                          const float *ref, const long long *idx, int count, const double *vals_q,
                          hipStream_t st);

// Deterministic FP64 fluxes: out[0..4] = fluid in, fluid out, substrate in,
// substrate out, substrate consumed.  f or gp may be null (then 0).  u: the
// compute-type velocity [dim][N] the substrate's second-order Dirichlet
// faces need (may be null otherwise).  With dim = LAY_2D_AD9 the words are
// the D2Q9 substrate's own and only the substrate terms are computed.
// partials: device double [5 * FLUX_BLOCKS].
enum { FLUX_BLOCKS = 512 };
hipError_t fluxes(int dim, int storage, const void *f, const void *gp, const void *desc,
                  const Geo &g, const float *ref_f, const float *ref_g, double u_in, double c_in,
                  Sink sink, int outlet, double c_out, const void *u, double *partials,
                  double *out5, hipStream_t st);

// part: device scratch of 2 * nparts words for the per-block check maxima
hipError_t ctrl_reset(Ctrl *c, double tol, int window, int is_fluid, int K,
                      unsigned long long *part, int nparts, hipStream_t st,
                      long long t_max = 0x7fffffffffffffffll);
hipError_t decide(Ctrl *c, hipStream_t st);

hipError_t copy_kernel(const void *src, void *dst, size_t bytes, hipStream_t st);

// ---- batched serving (2-D requests: D2Q9 fluid, D2Q5 substrate) ----------
enum { SRV_IDLE = 0, SRV_FLUID = 1, SRV_AD = 2 };
enum { SRV_MAX_SLOTS = 64 };

// One request on the device.  Its substrate buffers g[b] alias the start of
// the fluid buffers f[b] (the fluid populations are dead once the velocity
// is exported); prev holds the velocity (fluid phase) or concentration
// (substrate phase) of the previous check.
struct SrvSlot {
    const void *desc; // uint16 descriptor words [N]
    void *f[2];
    void *gp[2];      // substrate A/B (aliases of f[0], f[1])
    void *u;          // compute-type [2][N]
    void *prev;       // compute-type [2][N]
    float *ref_cur, *ref_next; // column references [nx] of the current phase
    Geo g;
    double omega_f, u_in, inv_uin;
    double omega_a, cin_s, cout_s, c_ref, k_sink, k_half, inv_cin;
    double c_in, c_out;
    int outlet;
    int phase;        // SRV_*
};

// Requests being stepped: entry e covers tiles [begin[e], begin[e+1]) of
// the launch and is request slot[e]; total_tiles = begin[n_active].
struct SrvTable {
    int n_active;
    int total_tiles;
    int begin[SRV_MAX_SLOTS + 1];
    int slot[SRV_MAX_SLOTS];
};

// Two steps of every request in tab (launch j of the current chunk: steps
// 2j and 2j + 1; MODE_CHECK stores per-tile maxima at part[v] and
// part[part_cap + v]).  One block per tile: blocks must be at least
// tab->total_tiles (the extra blocks exit).
hipError_t srv_step(int storage, int mode, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                    unsigned long long *part, int part_cap, int j, int blocks, hipStream_t st);
// Widest tile height of the served launches: 16 (64 x 16 tiles,
// 1024-thread blocks, srv_stepN) for FP32 and FP32-shifted storage, 4
// (srv_step only) for FP16 storage and FP32 storage with FP64 arithmetic.
int srv_tile_ty(int storage);
// ns steps (2 or 4) of every request in tab over 64 x 16 tiles: launch j of
// the current chunk, whose first step is t_off within the chunk.  FP32
// storage forms only; otherwise as srv_step.
hipError_t srv_stepN(int storage, int mode, int ns, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                     unsigned long long *part, int part_cap, int j, int t_off, int blocks, hipStream_t st);
// Stop rule for every request in tab after a check step.
hipError_t srv_decide(const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                      const unsigned long long *part, int part_cap, hipStream_t st);
// Reference roll (ref_cur <- ref_next) of every running request in tab.
hipError_t srv_ref_roll(const SrvSlot *slots, const SrvTable *tab, const Ctrl *ctrl, hipStream_t st);
// Device-side writes of one slot entry / the whole table, in stream order.
hipError_t srv_slot_set(SrvSlot *slots, int sid, const SrvSlot &v, hipStream_t st);
hipError_t srv_table_set(SrvTable *tab, const SrvTable &v, hipStream_t st);

} // namespace lbmk

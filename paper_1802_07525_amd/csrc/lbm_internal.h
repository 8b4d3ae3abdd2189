// lbm_internal.h -- internal types of the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.h"

struct lbm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
};

namespace lbmh {

// ---- SplitMix64 (Steele, Lea & Flood 2014) ------------------------------
struct SplitMix64 {
    uint64_t state;
    uint64_t next()
    {
        state += 0x9E3779B97F4A7C15ULL;
        uint64_t z = state;
        z ^= z >> 30;
        z *= 0xBF58476D1CE4E5B9ULL;
        z ^= z >> 27;
        z *= 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    // integer in [lo, hi] by modulo of one draw
    int64_t pick(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }
};

// ---- host geometry (geom.cpp) -------------------------------------------
struct Dirs {
    int q;
    int c[19][3];
};
// fluid (D2Q9 / D3Q19) or substrate (D2Q5 / D3Q7) directions of a grid
const Dirs &fluid_dirs(int nz);
const Dirs &ad_dirs(int nz);

bool fluid_blocked(uint8_t k);
bool ad_blocked(uint8_t k);

// mask rules: classes <= 3, chassis rows/planes not active, inlet/outlet
// columns free of SOLID/BIOFILM.  Returns empty string if fine.
std::string check_mask(const lbm_grid &g, const uint8_t *cls);
// the same rules for one node (x, y, z) of class k
std::string check_cell(const lbm_grid &g, int x, int y, int z, uint8_t k);
bool percolates(const lbm_grid &g, const uint8_t *cls);
// 1 for FLUID nodes linked to the outlet column, else 0 (one byte per node)
std::vector<uint8_t> flow_domain(const lbm_grid &g, const uint8_t *cls);
// some inlet-column node is in the domain (the mask percolates)
bool domain_reaches_inlet(const lbm_grid &g, const std::vector<uint8_t> &dom);
// per column x: the node sampling the shift reference, or -1
std::vector<int64_t> reference_nodes(const lbm_grid &g, const std::vector<uint8_t> &dom);
void links_fluid(const lbm_grid &g, const uint8_t *cls, uint32_t *out);
void links_ad(const lbm_grid &g, const uint8_t *cls, uint32_t *out);
// descriptor word (lbm_kernels.h layout) of node (x, y, z)
uint32_t desc_word(const lbm_grid &g, const uint8_t *cls, const uint8_t *dom, bool ref, int x, int y,
                   int z);
// word of node (x, y) for the D2Q9 substrate (2-D), its own layout
uint16_t ad9_desc_word(const lbm_grid &g, const uint8_t *cls, bool ref, int x, int y);
// descriptor words of every node
void build_desc(const lbm_grid &g, const uint8_t *cls, const std::vector<uint8_t> &dom,
                const std::vector<int64_t> &ref, uint32_t *desc);
void build_desc(const lbm_grid &g, const uint8_t *cls, uint32_t *desc);
int64_t growth_pick(const lbm_grid &g, const uint8_t *cls, const double *C, double xi);

// ---- solver services (solver.cpp) ---------------------------------------
// enqueue the substrate concentration of every node (FP64, the value each
// node collides with) into device memory dst [N] on the solver's stream
lbm_status export_c_device(lbm_solver *s, double *dst);
// field U, RHO or C (FP64) into device memory dst; synchronises the stream
lbm_status get_field_device(lbm_solver *s, int field, void *dst);
// the frozen velocity from device double [dim][N] (staged through the host)
lbm_status set_u_device(lbm_solver *s, const double *u);

// solver whose device buffers are carved from the device region [arena,
// arena + cap) (256-byte aligned): no device or pinned allocation and no
// events; its steady solves check the control block synchronously after
// each chunk (the same launches, stop and state).  EINVAL if the region is
// too small.  Destroy with lbm_solver_destroy (frees nothing in the region).
lbm_status solver_create_in(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const lbm_params &p, void *arena,
                            size_t cap, lbm_solver **out);
// velocity (double [dim][N], device) of the fluid state, on the stream
lbm_status export_u_device(lbm_solver *s, double *dst);
// Velocity (which 0, [dim][N]) or concentration (which 1, [N]) exported in
// FP32 -- the values the served form returns -- into host memory dst.
// Storage FP32, FP32-shifted or FP16 only; synchronises the stream.
lbm_status export_f32(lbm_solver *s, int which, float *dst);

// Default stall window in checks: 1000, or for FP16 storage the checks
// that span 10,000 steps (10 at its default cadence of 1000 steps).
inline int default_stall_checks(int storage, int check_every)
{
    if (storage != LBM_FP16_SHIFTED)
        return 1000;
    const int w = 10000 / (check_every > 0 ? check_every : 1);
    return w > 1 ? w : 1;
}

// Copy ordered on the context's stream and complete on return.  A plain
// hipMemcpy runs on the null stream, which orders nothing against work on
// a non-blocking stream (the context's own, or several solvers' in one
// process): an upload could still be landing while the stream's kernels
// read the buffer.
inline hipError_t stream_copy(lbm_ctx *ctx, void *dst, const void *src, size_t bytes, hipMemcpyKind kind)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, ctx->stream);
    return e == hipSuccess ? hipStreamSynchronize(ctx->stream) : e;
}

// ---- error helpers -------------------------------------------------------
lbm_status set_err(lbm_ctx *ctx, lbm_status st, const std::string &msg);
lbm_status hip_err(lbm_ctx *ctx, hipError_t e, const char *where);

// ---- roctx ranges (trace.cpp) --------------------------------------------
// A range named `name` (a string literal) on the calling thread for the
// object's lifetime, as a roctx push and pop; shown by rocprofv3
// --marker-trace.  A no-op unless LBM_ROCTX is set (lbm.h).
class Range {
  public:
    explicit Range(const char *name);
    ~Range();
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;

  private:
    bool on_;
};

} // namespace lbmh

struct lbm_solver {
    lbm_ctx *ctx = nullptr;
    lbm_grid grid{};
    lbm_params p{};
    int dim = 2, qf = 9, qa = 5;
    lbmk::Geo geo{};
    std::vector<uint8_t> cls;
    // host mirror of the descriptors and what they derive from: the flow
    // domain and the reference node of each column (cell updates patch
    // these and upload the words)
    std::vector<uint8_t> dom;
    std::vector<int64_t> refn;
    std::vector<uint32_t> desc_h;
    size_t desc_bytes = 2;       // per node
    // D2Q9 substrate (lbm_params.ad_lattice): its own 16-bit words
    bool ad9 = false;
    void *d_desc_ad = nullptr;
    std::vector<uint16_t> desc_ad_h;
    int64_t n_fluid = 0, n_ad = 0;
    int zseg_f = 0, zseg_a = 0;  // 3-D two-step launches: output planes per block
    int ty3 = 0;                 // 3-D two-step launches: column height
    int max_launch_steps = 0;    // cap on steps per launch (0: none)
    double c_ref = 0.0;          // substrate shift reference (0 if unshifted)

    void *d_desc = nullptr;
    void *d_f[2] = {nullptr, nullptr};
    void *d_g[2] = {nullptr, nullptr};
    void *d_u = nullptr;         // compute type [dim][N]
    void *d_uprev = nullptr;     // compute type [dim][N]
    void *d_cprev = nullptr;     // compute type [N]
    lbmk::Ctrl *d_ctrl = nullptr; // [2]: fluid, substrate
    unsigned long long *d_part = nullptr; // [2][2 * part_n] per-block check maxima
    int part_n = 0;              // blocks of the largest check launch
    float *d_ref = nullptr;      // column references [4][nx]: fluid cur, next; substrate cur, next
    double *d_partials = nullptr;
    double *d_out5 = nullptr;
    double *d_stage = nullptr;   // lazily sized double staging buffer
    size_t stage_bytes = 0;
    long long *d_idx = nullptr;  // small scratch for cell updates
    double *d_vals = nullptr;
    int fcur = 0, gcur = 0;
    bool fluid_ready = false, ad_ready = false;
    // steps taken so far by each solver (seeds the FP16 stochastic rounding;
    // saved in checkpoints so that a resumed run continues bit-exactly)
    unsigned long long fsteps = 0, gsteps = 0;

    // device memory region the buffers are carved from instead of device
    // allocations (the no-allocation solve); null: each buffer is allocated
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;

    lbmk::Ctrl *h_ctrl = nullptr; // pinned ring of control snapshots (host heap with an arena)
    hipEvent_t ev_ring[8] = {};
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
};

// bio-electrochemical state beside a solver (bio.hip; biofilm.cpp changes it)
struct lbm_bio {
    lbm_solver *s = nullptr;
    lbm_bio_params p{};
    std::vector<double> cb;      // biomass per node, mg/L (host, N)
    std::vector<double> mox;     // M_ox per node (host mirror, N)
    std::vector<int32_t> cells;  // nodes holding biomass, ascending
    bool mox_stale = false;      // the device copy is newer than `mox`
    size_t cap = 0;              // cells the device arrays hold
    int32_t *d_idx = nullptr;
    double *d_cb = nullptr, *d_mox = nullptr, *d_fs = nullptr;
    double *d_c = nullptr;       // substrate field [N]
    lbm_bio_out *d_out = nullptr;
    lbm_bio_out *h_out = nullptr; // pinned
    double sum_cb = 0.0, biomass = 0.0;
};


namespace lbmh {
// device M_ox -> host mirror; host fields -> cell list, totals, device (bio.hip)
lbm_status bio_pull_mox(lbm_bio *b);
lbm_status bio_push_cells(lbm_bio *b);
} // namespace lbmh

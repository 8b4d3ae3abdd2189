// solver.cpp -- solver objects: device state, steady-state loops, fields,
// cell updates, checkpoint/resume and the coupled biofilm loop.
//
// Steady loop.  The paper runs each LBM to equilibrium (Sec. 3).  Here a
// solve enqueues chunks of K steps; the last step of each chunk reduces the
// residual max |U(t) - U(t-K)| / (K |u_in|) on the device against the
// moments saved at the previous check, and a one-thread kernel
// applies the stop rule and raises a stop flag that every later step kernel
// honours by returning at once.  The host copies the
// control block into pinned memory after each chunk and keeps at most three
// chunks in flight, so the GPU never waits on the host for a decision and the
// state at the stop is exactly the state of the deciding check.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbmh;

#define HIPCHK(expr, where)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return hip_err(s->ctx, e_, where);                                                   \
    } while (0)

namespace {

const int RING = 8;
const int MAX_INFLIGHT = 3;
// A/B population working sets above this use streaming (non-temporal)
// stores: far beyond the 256 MB last-level cache the stored values are
// read back from HBM anyway; below it, ordinary stores keep them cached.
const double STREAMING_BYTES = 192.0 * 1024 * 1024;

inline size_t sbytes(const lbm_solver *s) { return lbmk::storage_bytes(s->p.storage); }
// column references of the fluid (which = 0) or substrate (1) state
inline float *ref_cur(const lbm_solver *s, int which) { return s->d_ref + (size_t)(2 * which) * s->grid.nx; }
inline float *ref_next(const lbm_solver *s, int which) { return s->d_ref + (size_t)(2 * which + 1) * s->grid.nx; }
inline size_t cbytes(const lbm_solver *s) { return lbmk::compute_bytes(s->p.storage); }
inline bool shifted(const lbm_solver *s) { return lbmk::storage_shifted(s->p.storage); }

lbm_status validate_params(lbm_ctx *ctx, const lbm_params &p)
{
    if (!(p.tau > 0.5) || !isfinite(p.tau))
        return set_err(ctx, LBM_EINVAL, "tau must be > 1/2");
    if (!(fabs(p.u_in) < 0.1) || p.u_in == 0.0)
        return set_err(ctx, LBM_EINVAL, "u_in must be nonzero with |u_in| < 0.1");
    if (!(p.D > 0.0) || !isfinite(p.D))
        return set_err(ctx, LBM_EINVAL, "D must be > 0");
    if (!(p.c_in != 0.0) || !isfinite(p.c_in))
        return set_err(ctx, LBM_EINVAL, "c_in must be finite and nonzero");
    if (!(p.k_sink >= 0.0 && p.k_sink < 1.0))
        return set_err(ctx, LBM_EINVAL, "k_sink must be in [0, 1)");
    if (!(p.k_half >= 0.0) || !isfinite(p.k_half))
        return set_err(ctx, LBM_EINVAL, "k_half must be finite and >= 0");
    if (p.k_half > 0.0 && !(p.k_sink < p.k_half))
        return set_err(ctx, LBM_EINVAL, "the Monod sink needs k_sink < k_half (a node never loses all it holds)");
    if (p.outlet != LBM_OUT_ZERO_GRADIENT && p.outlet != LBM_OUT_DIRICHLET)
        return set_err(ctx, LBM_EINVAL, "unknown outlet mode");
    if (!isfinite(p.c_out))
        return set_err(ctx, LBM_EINVAL, "c_out must be finite");
    if (p.storage < LBM_FP32 || p.storage > LBM_FP32_SHIFTED_F64)
        return set_err(ctx, LBM_EINVAL, "unknown storage");
    if (p.check_every < 2 || (p.check_every & 1))
        return set_err(ctx, LBM_EINVAL, "check_every must be even and >= 2");
    return LBM_OK;
}

// Descriptor words of the mirror to the device, in the device width.
lbm_status upload_desc_words(lbm_solver *s)
{
    const int64_t N = s->geo.N;
    if (s->desc_bytes == 2) {
        std::vector<uint16_t> p16((size_t)N);
        for (int64_t n = 0; n < N; ++n)
            p16[n] = (uint16_t)s->desc_h[n];
        HIPCHK(stream_copy(s->ctx, s->d_desc, p16.data(), (size_t)N * 2, hipMemcpyHostToDevice), "desc upload");
    } else {
        HIPCHK(stream_copy(s->ctx, s->d_desc, s->desc_h.data(), (size_t)N * 4, hipMemcpyHostToDevice),
               "desc upload");
    }
    return LBM_OK;
}

void count_active(lbm_solver *s)
{
    int64_t nf = 0, na = 0;
    // the shared words carry the D2Q5 / D3Q7 substrate bits whatever the
    // substrate lattice: the same active nodes
    const int aab = lbmk::desc_ad_active_bit(s->qf, s->dim == 3 ? 7 : 5);
    for (uint32_t d : s->desc_h) {
        nf += d & 1u;
        na += (d >> aab) & 1u;
    }
    s->n_fluid = nf;
    s->n_ad = na;
}

// Substrate layout code and descriptor words: the D2Q9 substrate's own, or
// the shared words
int ad_lay(const lbm_solver *s)
{
    return s->ad9 ? (int)lbmk::LAY_2D_AD9 : s->dim;
}
const void *ad_desc(const lbm_solver *s)
{
    return s->ad9 ? s->d_desc_ad : s->d_desc;
}

lbm_status upload_ad9_words(lbm_solver *s)
{
    HIPCHK(stream_copy(s->ctx, s->d_desc_ad, s->desc_ad_h.data(), s->desc_ad_h.size() * 2, hipMemcpyHostToDevice),
           "substrate desc upload");
    return LBM_OK;
}

// Full rebuild of the mirror from the mask, then upload.
lbm_status upload_desc(lbm_solver *s)
{
    s->dom = flow_domain(s->grid, s->cls.data());
    s->refn = reference_nodes(s->grid, s->dom);
    s->desc_h.resize((size_t)s->geo.N);
    build_desc(s->grid, s->cls.data(), s->dom, s->refn, s->desc_h.data());
    count_active(s);
    if (s->ad9) {
        s->desc_ad_h.resize((size_t)s->geo.N);
        for (int y = 0; y < s->grid.ny; ++y)
            for (int x = 0; x < s->grid.nx; ++x)
                s->desc_ad_h[(size_t)x + (size_t)s->grid.nx * y] =
                    ad9_desc_word(s->grid, s->cls.data(), s->refn[(size_t)x] == x + (int64_t)s->grid.nx * y, x, y);
        lbm_status st = upload_ad9_words(s);
        if (st)
            return st;
    }
    return upload_desc_words(s);
}

lbm_status dev_alloc(lbm_solver *s, void **p, size_t bytes, const char *what)
{
    if (*p)
        return LBM_OK;
    if (s->arena) {
        const size_t off = (s->arena_used + 255) & ~(size_t)255;
        if (off > s->arena_cap || bytes > s->arena_cap - off)
            return set_err(s->ctx, LBM_EINVAL,
                           std::string("the grid does not fit the scratch region (") + what + ": " +
                               std::to_string(off + bytes) + " of " + std::to_string(s->arena_cap) + " bytes)");
        *p = s->arena + off;
        s->arena_used = off + bytes;
        HIPCHK(hipMemsetAsync(*p, 0, bytes, s->ctx->stream), what);
        return LBM_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_err(s->ctx, LBM_ENOMEM, std::string("device allocation failed: ") + what);
    }
    if ((e = hipMemsetAsync(*p, 0, bytes, s->ctx->stream)) != hipSuccess) {
        // not handed out: a caller holding the pointer in a local would lose it
        (void)hipFree(*p);
        *p = nullptr;
        return hip_err(s->ctx, e, what);
    }
    return LBM_OK;
}

lbm_status ensure_fluid(lbm_solver *s)
{
    const size_t N = (size_t)s->geo.N;
    lbm_status st;
    for (int b = 0; b < 2; ++b)
        if ((st = dev_alloc(s, &s->d_f[b], (size_t)s->qf * N * sbytes(s), "fluid populations")))
            return st;
    return dev_alloc(s, &s->d_uprev, (size_t)s->dim * N * cbytes(s), "velocity history");
}

lbm_status ensure_ad(lbm_solver *s)
{
    const size_t N = (size_t)s->geo.N;
    lbm_status st;
    for (int b = 0; b < 2; ++b)
        if ((st = dev_alloc(s, &s->d_g[b], (size_t)s->qa * N * sbytes(s), "substrate populations")))
            return st;
    return dev_alloc(s, &s->d_cprev, N * cbytes(s), "concentration history");
}

lbm_status ensure_stage(lbm_solver *s, size_t bytes)
{
    if (s->stage_bytes >= bytes)
        return LBM_OK;
    if (s->d_stage && s->arena)
        return set_err(s->ctx, LBM_EINVAL, "staging buffer of a solver in a scratch region cannot grow");
    if (s->d_stage) {
        HIPCHK(hipStreamSynchronize(s->ctx->stream), "stage sync");
        HIPCHK(hipFree(s->d_stage), "stage free");
        s->d_stage = nullptr;
        s->stage_bytes = 0;
    }
    void *p = nullptr;
    lbm_status st = dev_alloc(s, &p, bytes, "staging buffer");
    if (st)
        return st;
    s->d_stage = static_cast<double *>(p);
    s->stage_bytes = bytes;
    return LBM_OK;
}

// 2-D solvers launch several steps at a time (one launch, LDS between them)
inline bool paired(const lbm_solver *s) { return s->dim == 2; }
// most steps one launch of this solver takes: in 3-D 2 (z-marching blocks,
// compute types of 4 bytes) or 1 (FP64); in 2-D 2, or 4 for the multi-step
// form
inline int launch_steps(const lbm_solver *s, int which)
{
    (void)which; // both solvers take the same form
    const int spl = !paired(s) ? (s->p.storage == LBM_FP64 ? 1 : 2)
                               : lbmk::fluid_launch_steps(s->p.storage, s->geo);
    return s->max_launch_steps > 0 && s->max_launch_steps < spl ? s->max_launch_steps : spl;
}
// steps of the next launch with `rem` steps left: the largest launch size
// that does not leave a single step behind, a one only to finish an odd
// count -- a chunk of K (even) steps thus ends on a multi-step launch, whose
// per-block check maxima are the ones the decide reads (K = 100 with four
// steps per launch: 25 launches of four)
inline int next_launch(int spl, int64_t rem)
{
    for (int k = spl; k >= 2; --k)
        if (k <= rem && rem - k != 1)
            return k;
    return 1;
}
// Steps of the next launch of a solver with `rem` steps left in the chunk;
// first: the chunk's first launch.  Storage that rounds on store (FP16)
// follows the paired launches (next_launch with two) and fuses two of them
// into one four-step launch wherever neither is the chunk's first (which
// moves the column references) and neither ends the chunk (the check, whose
// tile means the paired kernel takes): the stored states stay those of the
// paired launches bit for bit.  K = 100: 2, 24 x 4, 2.
inline int plan_next(const lbm_solver *s, int which, int64_t rem, bool first)
{
    const int spl = launch_steps(s, which);
    // 3-D storage with tile means (FP16) takes its check as a single step
    // (tile means over 64 x 4 tiles of one plane): a chunk ends on two
    // single steps (K = 100: 49 x 2, 1, 1)
    if (!paired(s) && spl == 2 && lbmk::storage_moving_ref(s->p.storage))
        return rem <= 2 ? 1 : 2;
    if (spl < 4 || !lbmk::storage_moving_ref(s->p.storage))
        return next_launch(spl, rem);
    const int k = next_launch(2, rem);
    if (first || k != 2 || rem < 6 || next_launch(2, rem - 2) != 2)
        return k;
    return 4;
}
inline int64_t chunk_launches(const lbm_solver *s, int which, int64_t n)
{
    int64_t c = 0;
    for (int64_t j = 0; j < n; j += plan_next(s, which, n - j, j == 0))
        ++c;
    return c;
}
// kernel launches that cover `steps` steps taken from a chunk boundary in
// chunks of check_every steps
inline int64_t launches_for(const lbm_solver *s, int which, int64_t steps)
{
    const int64_t K = s->p.check_every;
    return (steps / K) * chunk_launches(s, which, K) + chunk_launches(s, which, steps % K);
}
// blocks of the check-step launches (the per-block maxima the decide reads)
inline int check_blocks(const lbm_solver *s, int which)
{
    if (launch_steps(s, which) == 1)
        return s->geo.ntiles;
    if (!paired(s))
        return lbmk::storage_moving_ref(s->p.storage)
                   ? s->geo.ntiles
                   : lbmk::z3_blocks(s->geo, which == LBM_SOLVER_FLUID ? s->zseg_f : s->zseg_a, s->ty3);
    (void)which; // both solvers pick the same tile shape
    return lbmk::pair_tiles(s->geo, lbmk::pair_ty(s->p.storage, s->geo));
}

// One launch of `nsteps` (1; 2 to 4 in 2-D) steps reading buffer src.
// first: the first launch after a residual check, which moves the stored
// state to the column reference sampled at that check (see lbm_kernels.h)
hipError_t launch_step(lbm_solver *s, int which, int mode, int src, bool first = false, int nsteps = 1)
{
    if (which == LBM_SOLVER_FLUID) {
        lbmk::FluidArgs a;
        a.src = s->d_f[src];
        a.dst = s->d_f[src ^ 1];
        a.desc = s->d_desc;
        a.uprev = s->d_uprev;
        a.ctrl = s->d_ctrl;
        a.g = s->geo;
        a.omega = 1.0 / s->p.tau;
        a.u_in = s->p.u_in;
        a.inv_uin = 1.0 / ((double)s->p.check_every * fabs(s->p.u_in));
        a.streaming_stores = 2.0 * s->qf * (double)s->geo.N * sbytes(s) > STREAMING_BYTES;
        a.step = (unsigned int)s->fsteps;
        s->fsteps += nsteps;
        a.ref_src = ref_cur(s, 0);
        a.ref_dst = first ? ref_next(s, 0) : ref_cur(s, 0);
        a.ref_out = ref_next(s, 0);
        a.zseg = s->zseg_f;
        a.ty3 = s->ty3;
        if (nsteps >= 3)
            return lbmk::fluid_stepN(s->p.storage, mode, nsteps, a, s->ctx->stream);
        if (nsteps == 2)
            return paired(s) ? lbmk::fluid_step2(s->p.storage, mode, a, s->ctx->stream)
                             : lbmk::fluid_step3d2(s->p.storage, mode, a, s->ctx->stream);
        return lbmk::fluid_step(s->dim, s->p.storage, mode, a, s->ctx->stream);
    }
    const double cs2 = s->dim == 3 ? 0.25 : 1.0 / 3.0;
    lbmk::AdArgs a;
    a.src = s->d_g[src];
    a.dst = s->d_g[src ^ 1];
    a.desc = ad_desc(s);
    a.u = s->d_u;
    a.cprev = s->d_cprev;
    a.ctrl = s->d_ctrl + 1;
    a.g = s->geo;
    a.omega = 1.0 / (0.5 + s->p.D / cs2);
    a.cin_s = s->p.c_in - s->c_ref;
    a.cout_s = s->p.c_out - s->c_ref;
    a.c_ref = s->c_ref;
    a.k_sink = s->p.k_sink;
    a.k_half = s->p.k_half;
    a.inv_cin = 1.0 / ((double)s->p.check_every * fabs(s->p.c_in));
    a.outlet = s->p.outlet;
    a.streaming_stores = 2.0 * s->qa * (double)s->geo.N * sbytes(s) > STREAMING_BYTES;
    a.step = (unsigned int)s->gsteps;
    s->gsteps += nsteps;
    a.c_in = s->p.c_in;
    a.c_out = s->p.c_out;
    a.ref_src = ref_cur(s, 1);
    a.ref_dst = first ? ref_next(s, 1) : ref_cur(s, 1);
    a.ref_out = ref_next(s, 1);
    a.zseg = s->zseg_a;
    a.ty3 = s->ty3;
    if (nsteps >= 3)
        return lbmk::ad_stepN(ad_lay(s), s->p.storage, mode, nsteps, a, s->ctx->stream);
    if (nsteps == 2)
        return paired(s) ? lbmk::ad_step2(ad_lay(s), s->p.storage, mode, a, s->ctx->stream)
                         : lbmk::ad_step3d2(s->p.storage, mode, a, s->ctx->stream);
    return lbmk::ad_step(ad_lay(s), s->p.storage, mode, a, s->ctx->stream);
}

lbm_status init_solver(lbm_solver *s, int which)
{
    hipStream_t st = s->ctx->stream;
    const float r = which == LBM_SOLVER_FLUID ? 1.0f : (float)s->c_ref;
    HIPCHK(lbmk::ref_fill(ref_cur(s, which), 2 * s->grid.nx, r, st), "reference init");
    if (which == LBM_SOLVER_FLUID) {
        HIPCHK(lbmk::fluid_init(s->dim, s->p.storage, s->d_f[s->fcur], s->d_desc, s->geo, st),
               "fluid init");
        s->fluid_ready = true;
    } else {
        HIPCHK(lbmk::ad_init(ad_lay(s), s->p.storage, s->d_g[s->gcur], ad_desc(s), s->d_u, s->geo,
                             s->p.c_in, s->c_ref, st),
               "substrate init");
        s->ad_ready = true;
    }
    return LBM_OK;
}

// algorithmic bytes per active-node update: each population read once and
// written once, the 1-byte node class, and (substrate) the frozen velocity
double algo_bytes(const lbm_solver *s, int which)
{
    if (which == LBM_SOLVER_FLUID)
        return 2.0 * s->qf * (double)sbytes(s) + 1.0;
    return 2.0 * s->qa * (double)sbytes(s) + (double)(s->dim * cbytes(s)) + 1.0;
}

lbm_status fill_fluxes(lbm_solver *s, double *out5)
{
    const lbmk::Sink sink{s->p.k_sink, s->p.k_half};
    const void *f = s->fluid_ready ? s->d_f[s->fcur] : nullptr;
    const void *gp = s->ad_ready ? s->d_g[s->gcur] : nullptr;
    // the D2Q9 substrate has words of its own: fluid and substrate terms
    // in two passes, the second into out5 + 5
    HIPCHK(lbmk::fluxes(s->dim, s->p.storage, f, s->ad9 ? nullptr : gp, s->d_desc, s->geo, ref_cur(s, 0),
                        ref_cur(s, 1), s->p.u_in, s->p.c_in, sink, s->p.outlet, s->p.c_out, s->d_u,
                        s->d_partials, s->d_out5, s->ctx->stream),
           "fluxes");
    if (s->ad9)
        HIPCHK(lbmk::fluxes(lbmk::LAY_2D_AD9, s->p.storage, nullptr, gp, s->d_desc_ad, s->geo, ref_cur(s, 0),
                            ref_cur(s, 1), s->p.u_in, s->p.c_in, sink, s->p.outlet, s->p.c_out, s->d_u,
                            s->d_partials, s->d_out5 + 5, s->ctx->stream),
               "substrate fluxes");
    double o[10];
    HIPCHK(hipMemcpyAsync(o, s->d_out5, (s->ad9 ? 10 : 5) * sizeof(double), hipMemcpyDeviceToHost,
                          s->ctx->stream),
           "flux copy");
    HIPCHK(hipStreamSynchronize(s->ctx->stream), "flux sync");
    for (int k = 0; k < 5; ++k)
        out5[k] = s->ad9 && k >= 2 ? o[5 + k] : o[k];
    return LBM_OK;
}

lbm_status steady(lbm_solver *s, int which, double tol, int64_t max_iter, int warm,
                  lbm_info *info)
{
    if (!(tol >= 0.0) || max_iter < 1)
        return set_err(s->ctx, LBM_EINVAL, "tol must be >= 0 and max_iter >= 1");
    Range rg(which == LBM_SOLVER_FLUID ? "lbm.fluid.steady" : "lbm.ad.steady");
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    lbm_status stt = which == LBM_SOLVER_FLUID ? ensure_fluid(s) : ensure_ad(s);
    if (stt)
        return stt;
    const bool ready = which == LBM_SOLVER_FLUID ? s->fluid_ready : s->ad_ready;
    if (!warm || !ready)
        if ((stt = init_solver(s, which)))
            return stt;
    hipStream_t stream = s->ctx->stream;
    const int K = s->p.check_every;
    // default stall window: slow physical transients (a long porous medium
    // filling up behind a fixed inflow) can hold the residual level for
    // >10^4 steps, so it is long -- except with FP16 storage, whose
    // residual reaches its round-off floor within ordinary tolerances
    // (a long window there only repeats steps at the floor)
    const int window = s->p.stall_checks < 0
                           ? 0
                           : (s->p.stall_checks > 0 ? s->p.stall_checks : default_stall_checks(s->p.storage, K));
    lbmk::Ctrl *ctrl = s->d_ctrl + which;
    HIPCHK(lbmk::ctrl_reset(ctrl, tol, window, which == LBM_SOLVER_FLUID, K,
                            s->d_part + (size_t)which * 2 * s->part_n, check_blocks(s, which), stream),
           "ctrl reset");
    int &cur = which == LBM_SOLVER_FLUID ? s->fcur : s->gcur;
    const int cur0 = cur;
    unsigned long long &steps = which == LBM_SOLVER_FLUID ? s->fsteps : s->gsteps;
    const unsigned long long steps0 = steps;
    // moments of the starting state: the reference of the first check
    if (which == LBM_SOLVER_FLUID)
        HIPCHK(lbmk::fluid_export(s->dim, s->p.storage, s->d_f[cur0], s->d_desc, s->geo, ref_cur(s, 0),
                                  s->d_uprev,
                                  nullptr, 0, stream),
               "residual reference");
    else
        HIPCHK(lbmk::ad_export(ad_lay(s), s->p.storage, s->d_g[cur0], ad_desc(s), s->geo, ref_cur(s, 1),
                               lbmk::Sink{s->p.k_sink, s->p.k_half}, s->d_cprev, 0, stream),
               "residual reference");
    const auto t0 = std::chrono::steady_clock::now();
    // a solver in a scratch region has no events: it reads each chunk's
    // control snapshot synchronously
    const bool sync = s->arena != nullptr;
    if (!sync)
        HIPCHK(hipEventRecord(s->ev_a, stream), "event");
    int64_t launched = 0, head = 0, tail = 0;
    bool stopped = false;
    const bool roll = lbmk::storage_moving_ref(s->p.storage);
    int64_t nlaunch = 0;
    while (launched < max_iter && !stopped) {
        const int64_t rem = max_iter - launched;
        const int64_t n = rem >= K ? K : rem;
        for (int64_t j = 1; j <= n;) {
            const int k = plan_next(s, which, n - j + 1, j == 1);
            const int mode = (n == K && j + k - 1 == K) ? lbmk::MODE_CHECK : lbmk::MODE_PLAIN;
            HIPCHK(launch_step(s, which, mode, (int)((cur0 + nlaunch) & 1), j == 1, k), "step launch");
            if (j == 1 && roll)
                HIPCHK(lbmk::ref_roll(ctrl, ref_cur(s, which), ref_next(s, which), s->grid.nx, stream),
                       "reference roll");
            ++nlaunch;
            j += k;
        }
        if (n == K)
            HIPCHK(lbmk::decide(ctrl, stream), "decide");
        launched += n;
        const int slot = (int)(head % RING);
        HIPCHK(hipMemcpyAsync(&s->h_ctrl[slot], ctrl, sizeof(lbmk::Ctrl), hipMemcpyDeviceToHost, stream),
               "ctrl snapshot");
        if (sync) {
            HIPCHK(hipStreamSynchronize(stream), "ctrl snapshot sync");
            if (s->h_ctrl[slot].stop != lbmk::STOP_RUN)
                stopped = true;
            continue;
        }
        HIPCHK(hipEventRecord(s->ev_ring[slot], stream), "event");
        ++head;
        while (tail < head) {
            const int sl = (int)(tail % RING);
            if (head - tail > MAX_INFLIGHT) {
                HIPCHK(hipEventSynchronize(s->ev_ring[sl]), "event sync");
            } else {
                hipError_t q = hipEventQuery(s->ev_ring[sl]);
                if (q == hipErrorNotReady)
                    break;
                HIPCHK(q, "event query");
            }
            if (s->h_ctrl[sl].stop != lbmk::STOP_RUN)
                stopped = true;
            ++tail;
        }
    }
    if (!sync)
        HIPCHK(hipEventRecord(s->ev_b, stream), "event");
    HIPCHK(hipStreamSynchronize(stream), "solve sync");
    lbmk::Ctrl fin;
    HIPCHK(stream_copy(s->ctx, &fin, ctrl, sizeof(fin), hipMemcpyDeviceToHost), "ctrl read");
    const auto t1 = std::chrono::steady_clock::now();
    const int64_t t_final = fin.stop != lbmk::STOP_RUN ? fin.t_stop : launched;
    cur = (int)((cur0 + launches_for(s, which, t_final)) & 1);
    // launches queued behind the stop returned at once: the step counter
    // (the stochastic-rounding seed) counts the steps actually taken, so
    // that later solves do not depend on how many were in flight
    steps = steps0 + (unsigned long long)t_final;
    lbm_status result = LBM_NOT_CONVERGED;
    if (fin.stop == lbmk::STOP_OK)
        result = LBM_OK;
    else if (fin.stop == lbmk::STOP_STALLED)
        result = LBM_STALLED;
    else if (fin.stop == lbmk::STOP_DIVERGED)
        result = set_err(s->ctx, LBM_EDIVERGED, "solution diverged (NaN/Inf or |u| > 0.3)");
    if (which == LBM_SOLVER_FLUID)
        HIPCHK(lbmk::fluid_export(s->dim, s->p.storage, s->d_f[s->fcur], s->d_desc, s->geo, ref_cur(s, 0),
                                  s->d_u, nullptr, 0, stream),
               "velocity export");
    if (info) {
        float ms = 0.f; // no kernel time without events
        if (!sync)
            HIPCHK(hipEventElapsedTime(&ms, s->ev_a, s->ev_b), "event time");
        memset(info, 0, sizeof(*info));
        info->iters = t_final;
        info->residual = fin.checks > 0 ? fin.r_last : NAN;
        info->checks = fin.checks;
        info->active_nodes = which == LBM_SOLVER_FLUID ? s->n_fluid : s->n_ad;
        info->seconds = std::chrono::duration<double>(t1 - t0).count();
        info->kernel_ms = ms;
        info->launches = launches_for(s, which, t_final);
        const double upd = (double)t_final * (double)info->active_nodes;
        info->mlups = info->seconds > 0 ? upd / info->seconds / 1e6 : 0.0;
        info->gbps = ms > 0 ? upd * algo_bytes(s, which) / (ms * 1e-3) / 1e9 : 0.0;
        double f5[5];
        lbm_status fs = fill_fluxes(s, f5);
        if (fs)
            return fs;
        if (which == LBM_SOLVER_FLUID) {
            info->flux_in = f5[0];
            info->flux_out = f5[1];
        } else {
            info->flux_in = f5[2];
            info->flux_out = f5[3];
            info->sink_total = f5[4];
        }
    } else {
        HIPCHK(hipStreamSynchronize(stream), "sync");
    }
    return result;
}

// kind: where dst lives for the exported fields (U, RHO, C): host
// (DeviceToHost) or device (DeviceToDevice); the other fields are host only
lbm_status get_field(lbm_solver *s, int field, void *dst, hipMemcpyKind kind = hipMemcpyDeviceToHost)
{
    const size_t N = (size_t)s->geo.N;
    hipStream_t st = s->ctx->stream;
    lbm_status e;
    switch (field) {
    case LBM_FIELD_U:
    case LBM_FIELD_RHO: {
        if (!s->fluid_ready)
            return set_err(s->ctx, LBM_EINVAL, "fluid state not initialised");
        if ((e = ensure_stage(s, (size_t)(s->dim + 1) * N * 8)))
            return e;
        double *U = s->d_stage, *R = s->d_stage + (size_t)s->dim * N;
        HIPCHK(lbmk::fluid_export(s->dim, s->p.storage, s->d_f[s->fcur], s->d_desc, s->geo, ref_cur(s, 0),
                                  U, R, 1, st),
               "export");
        if (field == LBM_FIELD_U)
            HIPCHK(hipMemcpyAsync(dst, U, (size_t)s->dim * N * 8, kind, st), "copy");
        else
            HIPCHK(hipMemcpyAsync(dst, R, N * 8, kind, st), "copy");
        break;
    }
    case LBM_FIELD_C:
        if (!s->ad_ready)
            return set_err(s->ctx, LBM_EINVAL, "substrate state not initialised");
        if ((e = ensure_stage(s, N * 8)))
            return e;
        HIPCHK(lbmk::ad_export(ad_lay(s), s->p.storage, s->d_g[s->gcur], ad_desc(s), s->geo, ref_cur(s, 1),
                               lbmk::Sink{s->p.k_sink, s->p.k_half}, s->d_stage, 1, st),
               "export");
        HIPCHK(hipMemcpyAsync(dst, s->d_stage, N * 8, kind, st), "copy");
        break;
    case LBM_FIELD_CLASS:
        memcpy(dst, s->cls.data(), N);
        return LBM_OK;
    case LBM_FIELD_DESC:
        if (s->desc_bytes == 2) {
            std::vector<uint16_t> w(N);
            HIPCHK(stream_copy(s->ctx, w.data(), s->d_desc, N * 2, hipMemcpyDeviceToHost), "desc copy");
            for (size_t n = 0; n < N; ++n)
                static_cast<uint32_t *>(dst)[n] = w[n];
        } else {
            HIPCHK(stream_copy(s->ctx, dst, s->d_desc, N * 4, hipMemcpyDeviceToHost), "desc copy");
        }
        return LBM_OK;
    case LBM_FIELD_LINKS_F:
        return lbm_links(s->grid, s->cls.data(), LBM_SOLVER_FLUID, dst);
    case LBM_FIELD_LINKS_C:
        return lbm_links(s->grid, s->cls.data(), LBM_SOLVER_AD, dst);
    case LBM_FIELD_F:
    case LBM_FIELD_G: {
        const int which = field == LBM_FIELD_F ? 0 : 1;
        if (which == 0 ? !s->fluid_ready : !s->ad_ready)
            return set_err(s->ctx, LBM_EINVAL, "state not initialised");
        const int q = which == 0 ? s->qf : s->qa;
        if ((e = ensure_stage(s, (size_t)q * N * 8)))
            return e;
        HIPCHK(lbmk::pops_export(which, which == 0 ? s->dim : ad_lay(s), s->p.storage,
                                 which == 0 ? s->d_f[s->fcur] : s->d_g[s->gcur],
                                 which == 0 ? s->d_desc : ad_desc(s), s->geo, ref_cur(s, which), s->d_stage,
                                 st),
               "export");
        HIPCHK(hipMemcpyAsync(dst, s->d_stage, (size_t)q * N * 8, hipMemcpyDeviceToHost, st), "copy");
        break;
    }
    default:
        return set_err(s->ctx, LBM_ENOTFOUND, "unknown field");
    }
    HIPCHK(hipStreamSynchronize(st), "get sync");
    return LBM_OK;
}

struct StateHeader {
    char magic[8];
    int32_t nx, ny, nz, storage;
    int32_t qf, qa, fluid_ready, ad_ready;
    double tau, u_in, D, c_in, k_sink, c_out, k_half;
    int32_t outlet, check_every;
    int64_t N;
    uint64_t f_bytes, g_bytes, u_bytes, ref_bytes;
    uint64_t fsteps, gsteps;
};

size_t state_size(const lbm_solver *s)
{
    const size_t N = (size_t)s->geo.N;
    return sizeof(StateHeader) + N + (size_t)s->qf * N * sbytes(s) + (size_t)s->qa * N * sbytes(s) +
           (size_t)s->dim * N * cbytes(s) + (size_t)4 * s->grid.nx * sizeof(float);
}

} // namespace

lbm_status lbmh::get_field_device(lbm_solver *s, int field, void *dst)
{
    if (field != LBM_FIELD_U && field != LBM_FIELD_RHO && field != LBM_FIELD_C)
        return set_err(s->ctx, LBM_EINVAL, "only U, RHO and C export to device memory");
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    return get_field(s, field, dst, hipMemcpyDeviceToDevice);
}

lbm_status lbmh::set_u_device(lbm_solver *s, const double *u)
{
    const size_t n = (size_t)s->dim * (size_t)s->geo.N;
    std::vector<double> h(n);
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    HIPCHK(stream_copy(s->ctx, h.data(), u, n * 8, hipMemcpyDeviceToHost), "velocity copy");
    return lbm_solver_set_u(s, h.data());
}

lbm_status lbmh::export_c_device(lbm_solver *s, double *dst)
{
    if (!s->ad_ready)
        return set_err(s->ctx, LBM_EINVAL, "substrate state not initialised");
    HIPCHK(lbmk::ad_export(ad_lay(s), s->p.storage, s->d_g[s->gcur], ad_desc(s), s->geo, ref_cur(s, 1),
                           lbmk::Sink{s->p.k_sink, s->p.k_half}, dst, 1, s->ctx->stream),
           "export");
    return LBM_OK;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

lbm_status lbm_solver_create_ex(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const lbm_params *pp,
                                int require_percolation, lbm_solver **out);

lbm_status lbm_solver_create(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const lbm_params *p,
                             lbm_solver **out)
{
    return lbm_solver_create_ex(ctx, g, cls, p, 1, out);
}

} // extern "C"

// Creation shared by the allocating solver (arena null) and the solver in a
// scratch region
static lbm_status create_solver(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const lbm_params *pp,
                                int require_percolation, void *arena, size_t cap, lbm_solver **out)
{
    if (!ctx || !cls || !pp || !out)
        return set_err(ctx, LBM_EINVAL, "null argument");
    *out = nullptr;
    std::string m = check_mask(g, cls);
    if (!m.empty())
        return set_err(ctx, LBM_EINVAL, m);
    const int64_t N64 = (int64_t)g.nx * g.ny * g.nz;
    if (N64 > ((int64_t)1 << 31) / 19)
        return set_err(ctx, LBM_EINVAL, "grid too large");
    lbm_params p = *pp;
    // default check interval: 100 steps, or 1000 with FP16 storage, whose
    // residual (tile means) carries stochastic-rounding noise that falls
    // with the interval (see lbm.h)
    if (p.check_every == 0)
        p.check_every = p.storage == LBM_FP16_SHIFTED ? 1000 : 100;
    lbm_status st = validate_params(ctx, p);
    if (st)
        return st;
    if (p.ad_lattice != 0 && !(p.ad_lattice == 1 && g.nz == 1))
        return set_err(ctx, LBM_EINVAL, "ad_lattice: 0, or 1 (D2Q9 substrate) on a 2-D grid");
    if (require_percolation && !percolates(g, cls))
        return set_err(ctx, LBM_EINVAL, "the fluid domain does not connect inlet to outlet");
    hipError_t he = hipSetDevice(ctx->device);
    if (he != hipSuccess)
        return hip_err(ctx, he, "set device");
    lbm_solver *s = new lbm_solver();
    s->ctx = ctx;
    s->arena = static_cast<char *>(arena);
    s->arena_cap = arena ? cap : 0;
    s->grid = g;
    s->p = p;
    s->dim = g.nz > 1 ? 3 : 2;
    s->qf = s->dim == 3 ? 19 : 9;
    s->ad9 = p.ad_lattice == 1;
    s->qa = s->dim == 3 ? 7 : (s->ad9 ? 9 : 5);
    s->geo = lbmk::make_geo(g.nx, g.ny, g.nz);
    s->ty3 = g.nz > 1 ? lbmk::z3_tile_y(s->geo) : 0;
    // z-segments sized to the resident blocks per CU: the fluid kernel is
    // held to two waves per SIMD by its registers (one 512-thread or two
    // 256-thread blocks).  The substrate kernel fits four 32 x 16 blocks,
    // but its segments are sized for two: twice as many planes per block
    // recompute half the z-halo per output plane, which beats the fuller
    // round (256 x 128 x 128: 37.3 against 39.3 us per step in FP32 shifted
    // storage, 25.5 against 28.0 in FP16)
    s->zseg_f = g.nz > 1 ? lbmk::z3_planes_per_block(s->geo, s->ty3, s->ty3 == 16 ? 1 : 2) : 0;
    s->zseg_a = g.nz > 1 ? lbmk::z3_planes_per_block(s->geo, s->ty3, s->ty3 == 16 ? 2 : 5) : 0;
    // LBM_3D_PLANES_PER_BLOCK overrides the planes per block of the
    // two-step 3-D launches (tuning; tests run several segment lengths)
    if (const char *e = getenv("LBM_3D_PLANES_PER_BLOCK"))
        if (g.nz > 1 && atoi(e) > 0)
            s->zseg_f = s->zseg_a = atoi(e) < g.nz ? atoi(e) : g.nz;
    // LBM_MAX_LAUNCH_STEPS = 1 or 2 caps the steps per launch (tests compare
    // the launch forms, which take the same steps)
    if (const char *e = getenv("LBM_MAX_LAUNCH_STEPS"))
        if (atoi(e) == 1 || atoi(e) == 2)
            s->max_launch_steps = atoi(e);
    // per-block check maxima: one slot pair per block of the largest check
    // launch (64 x 4 tiles, or the 3-D two-step blocks where there are more)
    s->part_n = s->geo.ntiles;
    for (int zs : {s->zseg_f, s->zseg_a})
        if (g.nz > 1 && lbmk::z3_blocks(s->geo, zs, s->ty3) > s->part_n)
            s->part_n = lbmk::z3_blocks(s->geo, zs, s->ty3);
    s->cls.assign(cls, cls + N64);
    s->desc_bytes = s->dim == 3 ? 4 : 2;
    s->c_ref = lbmk::storage_shifted(p.storage) ? p.c_in : 0.0;
    const size_t N = (size_t)N64;
    auto fail = [&](lbm_status e) {
        lbm_solver_destroy(s);
        return e;
    };
    if ((st = dev_alloc(s, &s->d_desc, N * s->desc_bytes, "descriptors")))
        return fail(st);
    if (s->ad9 && (st = dev_alloc(s, &s->d_desc_ad, N * 2, "substrate descriptors")))
        return fail(st);
    if ((st = dev_alloc(s, &s->d_u, (size_t)s->dim * N * cbytes(s), "velocity")))
        return fail(st);
    void *tmp = nullptr;
    if ((st = dev_alloc(s, &tmp, 2 * sizeof(lbmk::Ctrl), "control")))
        return fail(st);
    s->d_ctrl = static_cast<lbmk::Ctrl *>(tmp);
    tmp = nullptr;
    if ((st = dev_alloc(s, &tmp, 4 * sizeof(unsigned long long) * (size_t)s->part_n, "check maxima")))
        return fail(st);
    s->d_part = static_cast<unsigned long long *>(tmp);
    tmp = nullptr;
    if ((st = dev_alloc(s, &tmp, 5 * lbmk::FLUX_BLOCKS * sizeof(double), "flux partials")))
        return fail(st);
    s->d_partials = static_cast<double *>(tmp);
    tmp = nullptr;
    if ((st = dev_alloc(s, &tmp, 4 * (size_t)g.nx * sizeof(float), "column references")))
        return fail(st);
    s->d_ref = static_cast<float *>(tmp);
    if ((he = lbmk::ref_fill(s->d_ref, 2 * g.nx, 1.0f, ctx->stream)) != hipSuccess ||
        (he = lbmk::ref_fill(s->d_ref + 2 * (size_t)g.nx, 2 * g.nx, (float)s->c_ref, ctx->stream)) !=
            hipSuccess)
        return fail(hip_err(ctx, he, "column references"));
    tmp = nullptr;
    if ((st = dev_alloc(s, &tmp, 16 * sizeof(double), "flux out")))
        return fail(st);
    s->d_out5 = static_cast<double *>(tmp);
    if ((st = upload_desc(s)))
        return fail(st);
    if (s->arena) {
        // no pinned memory and no events: control snapshots go to the host
        // heap, read after a stream synchronisation
        s->h_ctrl = new lbmk::Ctrl[RING];
    } else {
        he = hipHostMalloc((void **)&s->h_ctrl, RING * sizeof(lbmk::Ctrl), hipHostMallocDefault);
        if (he != hipSuccess) {
            s->h_ctrl = nullptr;
            return fail(hip_err(ctx, he, "pinned control ring"));
        }
        for (int k = 0; k < RING; ++k)
            if ((he = hipEventCreateWithFlags(&s->ev_ring[k], hipEventDisableTiming)) != hipSuccess)
                return fail(hip_err(ctx, he, "event"));
        if ((he = hipEventCreate(&s->ev_a)) != hipSuccess || (he = hipEventCreate(&s->ev_b)) != hipSuccess)
            return fail(hip_err(ctx, he, "event"));
    }
    if ((he = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return fail(hip_err(ctx, he, "create sync"));
    *out = s;
    return LBM_OK;
}

lbm_status lbmh::solver_create_in(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const lbm_params &p,
                                  void *arena, size_t cap, lbm_solver **out)
{
    if (!arena)
        return set_err(ctx, LBM_EINVAL, "null scratch region");
    return create_solver(ctx, g, cls, &p, 1, arena, cap, out);
}

lbm_status lbmh::export_u_device(lbm_solver *s, double *dst)
{
    if (!s->fluid_ready)
        return set_err(s->ctx, LBM_EINVAL, "fluid state not initialised");
    HIPCHK(lbmk::fluid_export(s->dim, s->p.storage, s->d_f[s->fcur], s->d_desc, s->geo, ref_cur(s, 0), dst,
                              nullptr, 1, s->ctx->stream),
           "export");
    return LBM_OK;
}

lbm_status lbmh::export_f32(lbm_solver *s, int which, float *dst)
{
    if (s->p.storage == LBM_FP64)
        return set_err(s->ctx, LBM_EINVAL, "FP32 export of an FP64 solver");
    if (!(which == 0 ? s->fluid_ready : s->ad_ready))
        return set_err(s->ctx, LBM_EINVAL, "state not initialised");
    const size_t N = (size_t)s->geo.N;
    const size_t bytes = (which == 0 ? (size_t)s->dim : 1) * N * 4;
    lbm_status e;
    if ((e = ensure_stage(s, bytes)))
        return e;
    hipStream_t st = s->ctx->stream;
    float *stage = reinterpret_cast<float *>(s->d_stage);
    if (which == 0)
        HIPCHK(lbmk::fluid_export(s->dim, s->p.storage, s->d_f[s->fcur], s->d_desc, s->geo, ref_cur(s, 0), stage,
                                  nullptr, 0, st),
               "export");
    else
        HIPCHK(lbmk::ad_export(ad_lay(s), s->p.storage, s->d_g[s->gcur], ad_desc(s), s->geo, ref_cur(s, 1),
                               lbmk::Sink{s->p.k_sink, s->p.k_half}, stage, 0, st),
               "export");
    HIPCHK(hipMemcpyAsync(dst, stage, bytes, hipMemcpyDeviceToHost, st), "copy");
    HIPCHK(hipStreamSynchronize(st), "sync");
    return LBM_OK;
}

extern "C" {

lbm_status lbm_solver_create_ex(lbm_ctx *ctx, lbm_grid g, const uint8_t *cls, const lbm_params *pp,
                                int require_percolation, lbm_solver **out)
{
    return create_solver(ctx, g, cls, pp, require_percolation, nullptr, 0, out);
}

void lbm_solver_destroy(lbm_solver *s)
{
    if (!s)
        return;
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    void *bufs[] = {s->d_desc, s->d_f[0],   s->d_f[1],   s->d_g[0], s->d_g[1],
                    s->d_u,    s->d_uprev,  s->d_cprev,  s->d_ctrl, s->d_part,
                    s->d_partials, s->d_out5, s->d_stage, s->d_idx, s->d_vals, s->d_ref,
                    s->d_desc_ad};
    if (!s->arena)
        for (void *b : bufs)
            if (b)
                (void)hipFree(b);
    if (s->h_ctrl) {
        if (s->arena)
            delete[] s->h_ctrl;
        else
            (void)hipHostFree(s->h_ctrl);
    }
    for (int k = 0; k < RING; ++k)
        if (s->ev_ring[k])
            (void)hipEventDestroy(s->ev_ring[k]);
    if (s->ev_a)
        (void)hipEventDestroy(s->ev_a);
    if (s->ev_b)
        (void)hipEventDestroy(s->ev_b);
    delete s;
}

lbm_status lbm_solver_fluid(lbm_solver *s, double tol, int64_t max_iter, int warm, lbm_info *info)
{
    if (!s)
        return LBM_EINVAL;
    if (!percolates(s->grid, s->cls.data()))
        return set_err(s->ctx, LBM_EINVAL, "the fluid domain does not connect inlet to outlet");
    return steady(s, LBM_SOLVER_FLUID, tol, max_iter, warm, info);
}

lbm_status lbm_solver_ad(lbm_solver *s, double tol, int64_t max_iter, int warm, lbm_info *info)
{
    if (!s)
        return LBM_EINVAL;
    return steady(s, LBM_SOLVER_AD, tol, max_iter, warm, info);
}

lbm_status lbm_solver_steps(lbm_solver *s, int which, int64_t nsteps, int cold, double *kernel_ms)
{
    if (!s || (which != 0 && which != 1) || nsteps < 0)
        return LBM_EINVAL;
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    lbm_status st = which == 0 ? ensure_fluid(s) : ensure_ad(s);
    if (st)
        return st;
    const bool ready = which == 0 ? s->fluid_ready : s->ad_ready;
    if (cold || !ready)
        if ((st = init_solver(s, which)))
            return st;
    hipStream_t stream = s->ctx->stream;
    HIPCHK(lbmk::ctrl_reset(s->d_ctrl + which, 0.0, 0, which == 0, s->p.check_every,
                            s->d_part + (size_t)which * 2 * s->part_n, check_blocks(s, which), stream),
           "ctrl");
    int &cur = which == 0 ? s->fcur : s->gcur;
    HIPCHK(hipEventRecord(s->ev_a, stream), "event");
    for (int64_t t = 0; t < nsteps;) {
        const int k = plan_next(s, which, nsteps - t, false);
        HIPCHK(launch_step(s, which, lbmk::MODE_PLAIN, cur, false, k), "step launch");
        cur ^= 1;
        t += k;
    }
    HIPCHK(hipEventRecord(s->ev_b, stream), "event");
    HIPCHK(hipStreamSynchronize(stream), "steps sync");
    if (kernel_ms) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, s->ev_a, s->ev_b), "event time");
        *kernel_ms = ms;
    }
    return LBM_OK;
}

lbm_status lbm_solver_time_steps(lbm_solver *s, int which, int nsteps, double *avg_ms)
{
    if (!s || (which != 0 && which != 1) || nsteps < 1 || !avg_ms)
        return LBM_EINVAL;
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    const bool ready = which == 0 ? s->fluid_ready : s->ad_ready;
    if (!ready)
        return set_err(s->ctx, LBM_EINVAL, "state not initialised");
    hipStream_t stream = s->ctx->stream;
    HIPCHK(lbmk::ctrl_reset(s->d_ctrl + which, 0.0, 0, which == 0, s->p.check_every,
                            s->d_part + (size_t)which * 2 * s->part_n, check_blocks(s, which), stream),
           "ctrl");
    const int k = launch_steps(s, which); // steps per launch
    const int nl = (nsteps + k - 1) / k;
    std::vector<hipEvent_t> ev((size_t)2 * nl);
    for (auto &e : ev)
        HIPCHK(hipEventCreate(&e), "event");
    int &cur = which == 0 ? s->fcur : s->gcur;
    hipError_t err = hipSuccess;
    for (int t = 0; t < nl && err == hipSuccess; ++t) {
        err = hipEventRecord(ev[2 * t], stream);
        if (err == hipSuccess)
            err = launch_step(s, which, lbmk::MODE_PLAIN, cur, false, k);
        if (err == hipSuccess)
            err = hipEventRecord(ev[2 * t + 1], stream);
        cur ^= 1;
    }
    if (err == hipSuccess)
        err = hipStreamSynchronize(stream);
    double sum = 0.0;
    for (int t = 0; t < nl && err == hipSuccess; ++t) {
        float ms = 0.f;
        err = hipEventElapsedTime(&ms, ev[2 * t], ev[2 * t + 1]);
        sum += ms;
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    HIPCHK(err, "per-launch timing");
    *avg_ms = sum / nl;
    return LBM_OK;
}

lbm_status lbm_solver_export_u(lbm_solver *s)
{
    if (!s)
        return LBM_EINVAL;
    if (!s->fluid_ready)
        return set_err(s->ctx, LBM_EINVAL, "fluid state not initialised");
    HIPCHK(lbmk::fluid_export(s->dim, s->p.storage, s->d_f[s->fcur], s->d_desc, s->geo, ref_cur(s, 0),
                              s->d_u, nullptr, 0, s->ctx->stream),
           "velocity export");
    HIPCHK(hipStreamSynchronize(s->ctx->stream), "sync");
    return LBM_OK;
}

lbm_status lbm_solver_set_u(lbm_solver *s, const double *u)
{
    if (!s || !u)
        return LBM_EINVAL;
    const size_t n = (size_t)s->dim * (size_t)s->geo.N;
    if (cbytes(s) == 8) {
        HIPCHK(stream_copy(s->ctx, s->d_u, u, n * 8, hipMemcpyHostToDevice), "set u");
    } else {
        std::vector<float> f(n);
        for (size_t k = 0; k < n; ++k)
            f[k] = (float)u[k];
        HIPCHK(stream_copy(s->ctx, s->d_u, f.data(), n * 4, hipMemcpyHostToDevice), "set u");
    }
    return LBM_OK;
}

lbm_status lbm_solver_get(lbm_solver *s, int field, void *dst)
{
    if (!s || !dst)
        return LBM_EINVAL;
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    return get_field(s, field, dst);
}

lbm_status lbm_solver_put(lbm_solver *s, int field, const double *src)
{
    if (!s || !src || (field != LBM_FIELD_F && field != LBM_FIELD_G))
        return LBM_EINVAL;
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    const int which = field == LBM_FIELD_F ? 0 : 1;
    lbm_status st = which == 0 ? ensure_fluid(s) : ensure_ad(s);
    if (st)
        return st;
    const size_t N = (size_t)s->geo.N;
    const int q = which == 0 ? s->qf : s->qa;
    if ((st = ensure_stage(s, (size_t)q * N * 8)))
        return st;
    hipStream_t stream = s->ctx->stream;
    HIPCHK(hipMemcpyAsync(s->d_stage, src, (size_t)q * N * 8, hipMemcpyHostToDevice, stream), "copy");
    HIPCHK(lbmk::pops_import(which, which == 0 ? s->dim : ad_lay(s), s->p.storage,
                             which == 0 ? s->d_f[s->fcur] : s->d_g[s->gcur],
                             which == 0 ? s->d_desc : ad_desc(s), s->geo, ref_cur(s, which), s->d_stage,
                             stream),
           "import");
    HIPCHK(hipStreamSynchronize(stream), "sync");
    if (which == 0)
        s->fluid_ready = true;
    else
        s->ad_ready = true;
    return LBM_OK;
}

lbm_status lbm_solver_device_ptr(lbm_solver *s, int field, void **ptr, size_t *bytes)
{
    if (!s || !ptr)
        return LBM_EINVAL;
    if (field != LBM_FIELD_U_DEVICE)
        return set_err(s->ctx, LBM_ENOTFOUND, "only LBM_FIELD_U_DEVICE has a device pointer");
    *ptr = s->d_u;
    if (bytes)
        *bytes = (size_t)s->dim * (size_t)s->geo.N * cbytes(s);
    return LBM_OK;
}

lbm_status lbm_solver_fluxes(lbm_solver *s, double *out5)
{
    if (!s || !out5)
        return LBM_EINVAL;
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    return fill_fluxes(s, out5);
}

lbm_status lbm_solver_update_cells(lbm_solver *s, const int64_t *idx, const uint8_t *new_cls, int64_t n)
{
    if (!s || n < 0 || (n > 0 && (!idx || !new_cls)))
        return LBM_EINVAL;
    Range rg("lbm.update_cells");
    const int64_t N = s->geo.N;
    const lbm_grid &g = s->grid;
    std::vector<uint8_t> trial = s->cls;
    for (int64_t k = 0; k < n; ++k) {
        if (idx[k] < 0 || idx[k] >= N || new_cls[k] > LBM_BIOFILM)
            return set_err(s->ctx, LBM_EINVAL, "bad cell index or class");
        const int x = (int)(idx[k] % g.nx), y = (int)((idx[k] / g.nx) % g.ny);
        const int z = (int)(idx[k] / ((int64_t)g.nx * g.ny));
        std::string m = check_cell(g, x, y, z, new_cls[k]);
        if (!m.empty())
            return set_err(s->ctx, LBM_EINVAL, m);
        trial[(size_t)idx[k]] = new_cls[k];
    }
    std::vector<uint8_t> dom1 = flow_domain(g, trial.data());
    if (!domain_reaches_inlet(g, dom1))
        return set_err(s->ctx, LBM_EINVAL, "update would disconnect inlet from outlet");
    std::vector<int64_t> ref1 = reference_nodes(g, dom1);
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    // populations of nodes whose activity changes: four lists.  Fluid
    // activity is membership of the flow domain, which an update can change
    // far from the updated cells (closing or opening a pore).
    std::vector<long long> f_off, f_on, g_off, g_on;
    for (int64_t j = 0; j < N; ++j) {
        if (s->dom[(size_t)j] && !dom1[(size_t)j])
            f_off.push_back(j);
        if (!s->dom[(size_t)j] && dom1[(size_t)j])
            f_on.push_back(j);
    }
    for (int64_t k = 0; k < n; ++k) {
        const int64_t j = idx[k];
        const uint8_t a = s->cls[(size_t)j], b = trial[(size_t)j];
        const bool ga = a == LBM_FLUID || a == LBM_BIOFILM, gb = b == LBM_FLUID || b == LBM_BIOFILM;
        if (ga && !gb)
            g_off.push_back(j);
        if (!ga && gb)
            g_on.push_back(j);
    }
    // descriptor words that can change: the updated cells and their lattice
    // neighbours (link bits), nodes entering or leaving the domain, and the
    // old and new reference nodes of every column whose reference moved
    std::vector<int64_t> touch(f_off.begin(), f_off.end());
    touch.insert(touch.end(), f_on.begin(), f_on.end());
    const Dirs &D = fluid_dirs(g.nz);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t j = idx[k];
        const int x = (int)(j % g.nx), y = (int)((j / g.nx) % g.ny);
        const int z = (int)(j / ((int64_t)g.nx * g.ny));
        for (int i = 0; i < D.q; ++i) {
            const int ax = x + D.c[i][0], ay = y + D.c[i][1], az = z + D.c[i][2];
            if (ax >= 0 && ay >= 0 && az >= 0 && ax < g.nx && ay < g.ny && az < g.nz)
                touch.push_back(ax + (int64_t)g.nx * (ay + (int64_t)g.ny * az));
        }
    }
    for (int x = 0; x < g.nx; ++x)
        if (s->refn[(size_t)x] != ref1[(size_t)x]) {
            if (s->refn[(size_t)x] >= 0)
                touch.push_back(s->refn[(size_t)x]);
            if (ref1[(size_t)x] >= 0)
                touch.push_back(ref1[(size_t)x]);
        }
    for (int64_t j : touch) {
        const int x = (int)(j % g.nx), y = (int)((j / g.nx) % g.ny);
        const int z = (int)(j / ((int64_t)g.nx * g.ny));
        s->desc_h[(size_t)j] = desc_word(g, trial.data(), dom1.data(), ref1[(size_t)x] == j, x, y, z);
        if (s->ad9)
            s->desc_ad_h[(size_t)j] = ad9_desc_word(g, trial.data(), ref1[(size_t)x] == j, x, y);
    }
    s->cls.swap(trial);
    s->dom.swap(dom1);
    s->refn.swap(ref1);
    count_active(s);
    lbm_status st = upload_desc_words(s);
    if (st)
        return st;
    if (s->ad9 && (st = upload_ad9_words(s)))
        return st;
    if (!s->d_idx) {
        void *p = nullptr;
        if ((st = dev_alloc(s, &p, 4096 * sizeof(long long), "index scratch")))
            return st;
        s->d_idx = static_cast<long long *>(p);
        p = nullptr;
        if ((st = dev_alloc(s, &p, 32 * sizeof(double), "value scratch")))
            return st;
        s->d_vals = static_cast<double *>(p);
    }
    hipStream_t stream = s->ctx->stream;
    static const double wf2[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static const double wf3[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static const double wa2[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    static const double wa3[7] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};
    auto apply = [&](int which, const std::vector<long long> &list, bool on) -> lbm_status {
        if (list.empty())
            return LBM_OK;
        void *buf = which == 0 ? s->d_f[s->fcur] : s->d_g[s->gcur];
        if (!buf)
            return LBM_OK; // solver never run: nothing stored yet
        const int q = which == 0 ? s->qf : s->qa;
        const double *w = which == 0 ? (s->dim == 3 ? wf3 : wf2)
                                     : (s->dim == 3 ? wa3 : (s->ad9 ? wf2 : wa2));
        // unshifted values; blocked nodes store 0 whatever the shift
        double vals[19];
        for (int i = 0; i < q; ++i) {
            if (!on)
                vals[i] = 0.0;
            else if (which == 0)
                vals[i] = w[i];                // rest state
            else
                vals[i] = w[i] * s->p.c_in;    // equilibrium at c_in, u = 0
        }
        HIPCHK(hipMemcpyAsync(s->d_vals, vals, q * sizeof(double), hipMemcpyHostToDevice, stream), "vals");
        for (size_t off = 0; off < list.size(); off += 4096) {
            const int cnt = (int)std::min<size_t>(4096, list.size() - off);
            HIPCHK(hipMemcpyAsync(s->d_idx, list.data() + off, cnt * sizeof(long long),
                                  hipMemcpyHostToDevice, stream),
                   "idx");
            HIPCHK(lbmk::pops_set_nodes(which, which == 0 ? s->dim : ad_lay(s), s->p.storage, buf, s->geo,
                                        on ? ref_cur(s, which) : nullptr, s->d_idx, cnt, s->d_vals,
                                        stream),
                   "cell reset");
            HIPCHK(hipStreamSynchronize(stream), "sync");
        }
        return LBM_OK;
    };
    if ((st = apply(0, f_off, false)) || (st = apply(0, f_on, true)) || (st = apply(1, g_off, false)) ||
        (st = apply(1, g_on, true)))
        return st;
    HIPCHK(hipStreamSynchronize(stream), "sync");
    return LBM_OK;
}

lbm_status lbm_solver_state_size(lbm_solver *s, size_t *bytes)
{
    if (!s || !bytes)
        return LBM_EINVAL;
    *bytes = state_size(s);
    return LBM_OK;
}

lbm_status lbm_solver_get_state(lbm_solver *s, void *dst, size_t bytes)
{
    if (!s || !dst || bytes < state_size(s))
        return LBM_EINVAL;
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    const size_t N = (size_t)s->geo.N;
    StateHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, "LBMSTAT4", 8);
    h.nx = s->grid.nx;
    h.ny = s->grid.ny;
    h.nz = s->grid.nz;
    h.storage = s->p.storage;
    h.qf = s->qf;
    h.qa = s->qa;
    h.fluid_ready = s->fluid_ready;
    h.ad_ready = s->ad_ready;
    h.tau = s->p.tau;
    h.u_in = s->p.u_in;
    h.D = s->p.D;
    h.c_in = s->p.c_in;
    h.k_sink = s->p.k_sink;
    h.k_half = s->p.k_half;
    h.c_out = s->p.c_out;
    h.outlet = s->p.outlet;
    h.check_every = s->p.check_every;
    h.N = (int64_t)N;
    h.f_bytes = (uint64_t)s->qf * N * sbytes(s);
    h.g_bytes = (uint64_t)s->qa * N * sbytes(s);
    h.u_bytes = (uint64_t)s->dim * N * cbytes(s);
    h.ref_bytes = (uint64_t)4 * s->grid.nx * sizeof(float);
    h.fsteps = s->fsteps;
    h.gsteps = s->gsteps;
    char *p = static_cast<char *>(dst);
    memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    memcpy(p, s->cls.data(), N);
    p += N;
    hipStream_t st = s->ctx->stream;
    if (s->fluid_ready)
        HIPCHK(hipMemcpyAsync(p, s->d_f[s->fcur], h.f_bytes, hipMemcpyDeviceToHost, st), "state f");
    else
        memset(p, 0, h.f_bytes);
    p += h.f_bytes;
    if (s->ad_ready)
        HIPCHK(hipMemcpyAsync(p, s->d_g[s->gcur], h.g_bytes, hipMemcpyDeviceToHost, st), "state g");
    else
        memset(p, 0, h.g_bytes);
    p += h.g_bytes;
    HIPCHK(hipMemcpyAsync(p, s->d_u, h.u_bytes, hipMemcpyDeviceToHost, st), "state u");
    p += h.u_bytes;
    HIPCHK(hipMemcpyAsync(p, s->d_ref, h.ref_bytes, hipMemcpyDeviceToHost, st), "state references");
    HIPCHK(hipStreamSynchronize(st), "state sync");
    return LBM_OK;
}

lbm_status lbm_solver_put_state(lbm_solver *s, const void *src, size_t bytes)
{
    if (!s || !src || bytes < sizeof(StateHeader))
        return LBM_EINVAL;
    StateHeader h;
    memcpy(&h, src, sizeof(h));
    if (memcmp(h.magic, "LBMSTAT4", 8) != 0 || h.nx != s->grid.nx || h.ny != s->grid.ny ||
        h.nz != s->grid.nz || h.storage != s->p.storage || h.qa != s->qa || bytes < state_size(s))
        return set_err(s->ctx, LBM_EINVAL, "checkpoint does not match this solver");
    const size_t N = (size_t)s->geo.N;
    const char *p = static_cast<const char *>(src) + sizeof(h);
    std::string m = check_mask(s->grid, reinterpret_cast<const uint8_t *>(p));
    if (!m.empty())
        return set_err(s->ctx, LBM_EINVAL, "checkpoint mask: " + m);
    HIPCHK(hipSetDevice(s->ctx->device), "set device");
    lbm_status st;
    if ((st = ensure_fluid(s)) || (st = ensure_ad(s)))
        return st;
    s->cls.assign(reinterpret_cast<const uint8_t *>(p), reinterpret_cast<const uint8_t *>(p) + N);
    if ((st = upload_desc(s)))
        return st;
    p += N;
    s->fcur = 0;
    s->gcur = 0;
    HIPCHK(stream_copy(s->ctx, s->d_f[0], p, h.f_bytes, hipMemcpyHostToDevice), "state f");
    p += h.f_bytes;
    HIPCHK(stream_copy(s->ctx, s->d_g[0], p, h.g_bytes, hipMemcpyHostToDevice), "state g");
    p += h.g_bytes;
    HIPCHK(stream_copy(s->ctx, s->d_u, p, h.u_bytes, hipMemcpyHostToDevice), "state u");
    p += h.u_bytes;
    HIPCHK(stream_copy(s->ctx, s->d_ref, p, h.ref_bytes, hipMemcpyHostToDevice), "state references");
    s->fluid_ready = h.fluid_ready != 0;
    s->ad_ready = h.ad_ready != 0;
    s->fsteps = h.fsteps;
    s->gsteps = h.gsteps;
    return LBM_OK;
}

lbm_status lbm_coupled_run(lbm_solver *s, int n_updates, const double *xi, double tol, int64_t max_iter,
                           int64_t *picked, double *J, double *J_accum, int64_t *iters_fluid,
                           int64_t *iters_ad)
{
    if (!s || n_updates < 0 || (n_updates > 0 && !xi) || !J_accum)
        return LBM_EINVAL;
    for (int m = 0; m < n_updates; ++m)
        if (!(xi[m] >= 0.0 && xi[m] < 1.0))
            return set_err(s->ctx, LBM_EINVAL, "xi must lie in [0, 1)");
    const size_t N = (size_t)s->geo.N;
    std::vector<double> C(N);
    double acc = 0.0;
    lbm_info fi, ai;
    for (int m = 0; m <= n_updates; ++m) {
        Range rg(m > 0 ? "lbm.coupled.update" : "lbm.coupled.initial");
        if (m > 0) {
            lbm_status st = get_field(s, LBM_FIELD_C, C.data());
            if (st)
                return st;
            const int64_t p = growth_pick(s->grid, s->cls.data(), C.data(), xi[m - 1]);
            if (picked)
                picked[m - 1] = p;
            if (p < 0)
                return set_err(s->ctx, LBM_EINVAL, "no biofilm growth candidate left");
            const uint8_t bio = LBM_BIOFILM;
            if ((st = lbm_solver_update_cells(s, &p, &bio, 1)))
                return st;
        }
        lbm_status sf = lbm_solver_fluid(s, tol, max_iter, m > 0, &fi);
        if (iters_fluid)
            iters_fluid[m] = fi.iters;
        if (sf < 0)
            return sf;
        lbm_status sa = lbm_solver_ad(s, tol, max_iter, m > 0, &ai);
        if (iters_ad)
            iters_ad[m] = ai.iters;
        if (sa < 0)
            return sa;
        if (J)
            J[m] = ai.sink_total;
        if (m > 0)
            acc += ai.sink_total;
    }
    *J_accum = acc;
    return LBM_OK;
}

} // extern "C"

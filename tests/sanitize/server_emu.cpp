// CPU emulation of the serving loop (server.cpp) and of the single-domain
// solver's host code (solver.cpp, api.cpp) for the sanitizer builds
// (ThreadSanitizer; AddressSanitizer with UndefinedBehaviorSanitizer).
//
// server.cpp, solver.cpp, api.cpp, biofilm.cpp and geom.cpp are linked
// against this file instead of the HIP runtime, the gfx950 kernels and the
// device side of the bio-electrochemical state:
//
//  * HIP runtime: a stream is a host thread that runs its queued operations
//    in order (copies, fills, kernels, event markers), with small random
//    delays; an event completes when its stream has run everything queued
//    before it was recorded; capture records a stream's operations into a
//    graph, and a graph launch queues them again.  Completion is published
//    under the stream's mutex, so the sanitizer sees exactly the ordering a
//    caller gets from events and synchronisation, and host memory a copy
//    reads or writes is touched by the stream thread, as the GPU would.
//  * Kernels: a stub stepper with no lattice arithmetic.  A request's state
//    is a header {phase, steps taken, owner} at the start of its population
//    buffer, and its residual history is a made-up function of the request
//    parameters and the step count (it halves every 100 steps and reaches
//    tol at a step set by u_in or D; tau and k_sink select a floor at 10 tol,
//    in every storage or in FP16 storage only, or a divergence).  The stop
//    rule is applied to that history at each check.  The batched kernels and
//    the single-domain solver's step, check, decide, export and flux kernels
//    are emulated; the solo lanes run the real single-domain solver on them.
//
// The stub kernels check what the real ones rely on and abort on a
// violation: the grid covers the slot table, each table entry spans exactly
// its request's tiles, a launch finds in its source buffer the state of the
// step it is to take (so no chunk is lost, repeated or misnumbered and every
// chunk has an even number of launches), a state belongs to the slot or
// solver that steps it, and exports read a state of the right phase.
//
// The driver (main) submits seeded request streams from several threads
// while a poller takes results and another thread reads the statistics, then
// drains.  Every result is compared with the sequential expectation: status,
// lane, step counts, the first attempt of an escalated request, and the
// exported fields and fluxes, which carry the step count of the state they
// were exported from; so are the server's statistics.  Two streams inject a
// device failure, servers are destroyed with work in flight, three
// coupled biofilm loops (growth picks, cell updates, warm re-solves) run at
// once on contexts of their own, and the hourly model loop runs the
// agent-based biofilm (biofilm.cpp) on the real solver.  Prints "ok" and
// exits 0 when all of it holds.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "lbm_internal.h"

// ------------------------------------------------------------ failures
static void emu_fail(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "emulation check failed: ");
    vfprintf(stderr, fmt, ap);
    fprintf(stderr, "\n");
    va_end(ap);
    fflush(stderr);
    abort();
}
#define EMU_CHECK(c, ...)                                                        \
    do {                                                                         \
        if (!(c))                                                                \
            emu_fail(__VA_ARGS__);                                               \
    } while (0)

// ------------------------------------------------------- HIP runtime
static std::atomic<unsigned> g_stream_seed{12345};
// device failure injection: once g_fail_at operations have been queued,
// every further operation fails, as after a device fault
static std::atomic<long long> g_ops{0}, g_fail_at{-1};
// launches of the batched step per tile form (64 x 4, 64 x 16)
static std::atomic<long long> g_launch_pair{0}, g_launch_wide{0};

struct ihipGraph {
    std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
    std::vector<std::function<void()>> ops;
};

struct ihipStream_t {
    std::mutex m;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    uint64_t enq = 0, done = 0;
    bool quit = false;
    ihipGraph *cap = nullptr;
    std::thread th;
    unsigned seed = 0;

    void run()
    {
        std::mt19937 rng(seed);
        for (;;) {
            std::function<void()> f;
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [&] { return quit || !q.empty(); });
                if (q.empty())
                    return;
                f = std::move(q.front());
                q.pop_front();
            }
            if (rng() % 8 == 0)
                std::this_thread::sleep_for(std::chrono::microseconds(rng() % 50));
            f();
            {
                std::lock_guard<std::mutex> lk(m);
                ++done;
            }
            cv.notify_all();
        }
    }
};

struct ihipEvent_t {
    std::mutex m;
    ihipStream_t *s = nullptr;
    uint64_t seq = 0;
};

static hipError_t enqueue(hipStream_t s, std::function<void()> fn)
{
    EMU_CHECK(s != nullptr, "work queued on the null stream");
    if (g_fail_at.load() >= 0 && ++g_ops >= g_fail_at.load())
        return hipErrorLaunchFailure;
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (s->cap) {
            s->cap->ops.push_back(std::move(fn));
            return hipSuccess;
        }
        s->q.push_back(std::move(fn));
        ++s->enq;
    }
    s->cv.notify_all();
    return hipSuccess;
}

static void *emu_alloc(size_t bytes)
{
    const size_t b = (bytes + 255) & ~(size_t)255;
    void *p = aligned_alloc(256, b ? b : 256);
    if (p)
        memset(p, 0xCD, b ? b : 256); // device memory starts as garbage
    return p;
}

extern "C" {

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t e)
{
    switch (e) {
    case hipSuccess:
        return "hipSuccess";
    case hipErrorInvalidValue:
        return "hipErrorInvalidValue";
    case hipErrorOutOfMemory:
        return "hipErrorOutOfMemory";
    case hipErrorNotReady:
        return "hipErrorNotReady";
    default:
        return "emulated HIP error";
    }
}

hipError_t hipMalloc(void **p, size_t bytes)
{
    *p = emu_alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned int)
{
    *p = emu_alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void *p)
{
    free(p);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    ihipStream_t *x = new ihipStream_t();
    x->seed = g_stream_seed.fetch_add(7919);
    x->th = std::thread([x] { x->run(); });
    *s = x;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::unique_lock<std::mutex> lk(s->m);
    s->cv.wait(lk, [&] { return s->done == s->enq; });
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->quit = true;
    }
    s->cv.notify_all();
    s->th.join();
    delete s;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    std::lock_guard<std::mutex> lk(s->m);
    EMU_CHECK(!s->cap, "nested capture");
    s->cap = new ihipGraph();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g)
{
    std::lock_guard<std::mutex> lk(s->m);
    EMU_CHECK(s->cap, "capture ended that never began");
    *g = s->cap;
    s->cap = nullptr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    *x = new hipGraphExec{g->ops};
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s)
{
    return enqueue(s, [x] {
        for (auto &f : x->ops)
            f();
    });
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    delete x;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g)
{
    delete g;
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned)
{
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(s->m);
    EMU_CHECK(!s->cap, "event recorded into a capture");
    std::lock_guard<std::mutex> le(e->m);
    e->s = s;
    e->seq = s->enq;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    ihipStream_t *s;
    uint64_t seq;
    {
        std::lock_guard<std::mutex> le(e->m);
        s = e->s;
        seq = e->seq;
    }
    if (!s)
        return hipSuccess;
    std::lock_guard<std::mutex> lk(s->m);
    return s->done >= seq ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e)
{
    ihipStream_t *s;
    uint64_t seq;
    {
        std::lock_guard<std::mutex> le(e->m);
        s = e->s;
        seq = e->seq;
    }
    if (!s)
        return hipSuccess;
    std::unique_lock<std::mutex> lk(s->m);
    s->cv.wait(lk, [&] { return s->done >= seq; });
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s)
{
    return enqueue(s, [=] { memcpy(dst, src, bytes); });
}
hipError_t hipMemsetAsync(void *dst, int v, size_t bytes, hipStream_t s)
{
    return enqueue(s, [=] { memset(dst, v, bytes); });
}

} // extern "C"

// ---------------------------------------------- made-up residual history
namespace emu {

// Which history a solve follows.  Fluid: tau in [0.6, 0.7) converges,
// [0.7, 0.8) has a floor in FP16 storage only, [0.8, 0.9) a floor in every
// storage, [0.9, 1) diverges (|u| = 0.5) at step S = |u_in| 1e5.  Substrate:
// S = D 1e4; k_sink < 0.5 converges, [0.5, 0.7) floor in FP16 only, >= 0.7
// diverges (NaN).
struct History {
    long long S;
    bool floor, diverge;
};

History history(bool fluid, int storage, double tau, double u_in, double D, double k_sink)
{
    History h{};
    const bool f16 = storage == LBM_FP16_SHIFTED;
    if (fluid) {
        h.S = llround(fabs(u_in) * 1e5);
        h.floor = (tau >= 0.7 && tau < 0.8 && f16) || (tau >= 0.8 && tau < 0.9);
        h.diverge = tau >= 0.9;
    } else {
        h.S = llround(D * 1e4);
        h.floor = k_sink >= 0.5 && k_sink < 0.7 && f16;
        h.diverge = k_sink >= 0.7;
    }
    return h;
}

double residual(const History &h, bool fluid, double tol, long long t)
{
    if (!fluid && h.diverge && t >= h.S)
        return NAN;
    double r = tol * exp2((double)(h.S - t) / 100.0);
    if (h.floor && r < 10.0 * tol)
        r = 10.0 * tol;
    return r;
}

double umax(const History &h, bool fluid, long long t) { return fluid && h.diverge && t >= h.S ? 0.5 : 0.01; }

unsigned long long bits(double x)
{
    unsigned long long b;
    memcpy(&b, &x, 8);
    return b;
}
double from_bits(unsigned long long b)
{
    double x;
    memcpy(&x, &b, 8);
    return x;
}

// The stop rule after one check (residual r, max |u| um): DIVERGED on
// NaN/Inf or |u| > 0.3 (fluid), OK at r <= tol, STALLED after `window`
// checks without a new maximum or a new minimum since the last maximum,
// MAXITER once t_max steps are covered.
void apply_rule(lbmk::Ctrl *c, double r, double um)
{
    c->t += c->K;
    c->checks += 1;
    c->r_last = r;
    c->res_bits = bits(r);
    c->umax_bits = bits(um);
    int stop = lbmk::STOP_RUN;
    if (std::isnan(r) || std::isinf(r) || std::isnan(um) || (c->is_fluid && um > 0.3)) {
        stop = lbmk::STOP_DIVERGED;
    } else if (r <= c->tol) {
        stop = lbmk::STOP_OK;
    } else if (r > c->peak) {
        c->peak = c->best = r;
        c->since_best = 0;
    } else if (r < c->best) {
        c->best = r;
        c->since_best = 0;
    } else if (++c->since_best >= c->window && c->window > 0) {
        stop = lbmk::STOP_STALLED;
    }
    if (stop == lbmk::STOP_RUN && c->t >= c->t_max)
        stop = lbmk::STOP_MAXITER;
    if (stop != lbmk::STOP_RUN) {
        c->t_stop = c->t;
        c->stop = stop;
    }
}

void reset(lbmk::Ctrl *c, double tol, int window, int is_fluid, int K, long long t_max)
{
    memset(c, 0, sizeof(*c));
    c->tol = tol;
    c->best = INFINITY;
    c->peak = -INFINITY;
    c->r_last = NAN;
    c->t_stop = -1;
    c->window = window;
    c->is_fluid = is_fluid;
    c->K = K;
    c->t_max = t_max;
}

struct Outcome {
    int status; // lbm_status
    long long iters, checks;
    double r_last;
};

int status_of(int stop)
{
    switch (stop) {
    case lbmk::STOP_OK:
        return LBM_OK;
    case lbmk::STOP_STALLED:
        return LBM_STALLED;
    case lbmk::STOP_DIVERGED:
        return LBM_EDIVERGED;
    default:
        return LBM_NOT_CONVERGED;
    }
}

// A whole solve, check by check.
Outcome solve(const History &h, bool fluid, double tol, int K, int window, long long max_iter)
{
    lbmk::Ctrl c;
    reset(&c, tol, window, fluid, K, (max_iter + K - 1) / K * K);
    while (c.stop == lbmk::STOP_RUN) {
        const long long t = c.t + K;
        apply_rule(&c, residual(h, fluid, tol, t), umax(h, fluid, t));
    }
    return Outcome{status_of(c.stop), c.t_stop, c.checks, c.r_last};
}

// State header at the start of a request's population buffer.
struct Hdr {
    unsigned long long magic;
    long long steps; // the batch: steps since init; the single solver: its step counter
    long long base;  // the single solver: its step counter at init
    unsigned long long owner;
    int phase;
    int fresh;       // initialised, not stepped yet
};
const unsigned long long MAGIC = 0x5EA7ED5EA7ED0001ull;

unsigned long long owner_of(const void *desc, long long N) { return (unsigned long long)(uintptr_t)desc ^ (unsigned long long)N; }

int served_ty()
{
    static const int ty = [] {
        const char *e = getenv("EMU_SERVED_TILE_TY");
        return e && atoi(e) == 16 ? 16 : 4;
    }();
    return ty;
}

} // namespace emu

// ------------------------------------------------------------- kernels
namespace lbmk {

Geo make_geo(int nx, int ny, int nz)
{
    Geo g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.ntx = (nx + 63) / 64;
    g.nty = (ny + 3) / 4;
    g.ntiles = g.ntx * g.nty * nz;
    g.N = (long long)nx * ny * nz;
    return g;
}
int pair_tiles(const Geo &g, int ty) { return g.ntx * ((g.ny + ty - 1) / ty) * g.nz; }
int pair_tiles(const Geo &g) { return pair_tiles(g, 4); }
size_t storage_bytes(int s) { return s == ST_F64 ? 8 : (s == ST_F16S ? 2 : 4); }
bool storage_shifted(int s) { return s == ST_F32S || s == ST_F16S || s == ST_F32X; }
bool storage_moving_ref(int s) { return s == ST_F16S; }
// 64 x 16 served tiles for the FP32 forms when the environment asks for
// them, else 64 x 4 (FP16 storage always 64 x 4)
int srv_tile_ty(int storage) { return storage == ST_F16S ? 4 : emu::served_ty(); }

hipError_t ref_fill(float *ref, int n, float v, hipStream_t st)
{
    return enqueue(st, [=] {
        for (int k = 0; k < n; ++k)
            ref[k] = v;
    });
}

static void write_hdr(void *f, const void *desc, const Geo &g, int phase)
{
    emu::Hdr *h = static_cast<emu::Hdr *>(f);
    h->magic = emu::MAGIC;
    h->steps = 0;
    h->base = 0;
    h->owner = emu::owner_of(desc, g.N);
    h->phase = phase;
    h->fresh = 1;
}
static const emu::Hdr *read_hdr(const void *f, const void *desc, const Geo &g, int phase, const char *who)
{
    const emu::Hdr *h = static_cast<const emu::Hdr *>(f);
    EMU_CHECK(h->magic == emu::MAGIC, "%s: no state in the buffer", who);
    EMU_CHECK(h->owner == emu::owner_of(desc, g.N), "%s: the state belongs to another request", who);
    EMU_CHECK(h->phase == phase, "%s: state of phase %d, expected %d", who, h->phase, phase);
    return h;
}

hipError_t fluid_init(int, int, void *f, const void *desc, const Geo &g, hipStream_t st)
{
    return enqueue(st, [=] { write_hdr(f, desc, g, SRV_FLUID); });
}
hipError_t ad_init(int, int, void *gp, const void *desc, const void *, const Geo &g, double, double,
                   hipStream_t st)
{
    return enqueue(st, [=] { write_hdr(gp, desc, g, SRV_AD); });
}
hipError_t fluid_export(int, int, const void *f, const void *desc, const Geo &g, const float *, void *U,
                        void *RHO, int out_double, hipStream_t st)
{
    EMU_CHECK(!RHO, "no density export is emulated");
    return enqueue(st, [=] {
        const emu::Hdr *h = read_hdr(f, desc, g, SRV_FLUID, "fluid_export");
        const double v = (double)(h->steps - h->base);
        for (long long n = 0; n < 2 * g.N; ++n) {
            if (out_double)
                static_cast<double *>(U)[n] = v;
            else
                static_cast<float *>(U)[n] = (float)v;
        }
    });
}
hipError_t ad_export(int, int, const void *gp, const void *desc, const Geo &g, const float *, Sink, void *C,
                     int out_double, hipStream_t st)
{
    return enqueue(st, [=] {
        const emu::Hdr *h = read_hdr(gp, desc, g, SRV_AD, "ad_export");
        const double v = (double)(h->steps - h->base);
        for (long long n = 0; n < g.N; ++n) {
            if (out_double)
                static_cast<double *>(C)[n] = v;
            else
                static_cast<float *>(C)[n] = (float)v;
        }
    });
}
hipError_t fluxes(int, int, const void *f, const void *gp, const void *desc, const Geo &g, const float *,
                  const float *, double, double, Sink, int, double, const void *, double *, double *out5,
                  hipStream_t st)
{
    return enqueue(st, [=] {
        for (int k = 0; k < 5; ++k)
            out5[k] = 0.0;
        if (f) {
            const emu::Hdr *h = read_hdr(f, desc, g, SRV_FLUID, "fluxes");
            out5[0] = (double)(h->steps - h->base);
        }
        if (gp) {
            const emu::Hdr *h = read_hdr(gp, desc, g, SRV_AD, "fluxes");
            out5[2] = (double)(h->steps - h->base);
        }
    });
}
hipError_t ctrl_reset(Ctrl *c, double tol, int window, int is_fluid, int K, unsigned long long *part, int nparts,
                      hipStream_t st, long long t_max)
{
    return enqueue(st, [=] {
        emu::reset(c, tol, window, is_fluid, K, t_max);
        c->part = part;
        c->nparts = nparts;
    });
}
hipError_t srv_slot_set(SrvSlot *slots, int sid, const SrvSlot &v, hipStream_t st)
{
    EMU_CHECK(sid >= 0 && sid < SRV_MAX_SLOTS, "slot %d out of range", sid);
    return enqueue(st, [=] { slots[sid] = v; });
}
hipError_t srv_table_set(SrvTable *tab, const SrvTable &v, hipStream_t st)
{
    return enqueue(st, [=] { *tab = v; });
}

static emu::History slot_history(const SrvSlot &sl, int storage)
{
    const double tau = 1.0 / sl.omega_f;
    const double D = (1.0 / sl.omega_a - 0.5) / 3.0;
    return emu::history(sl.phase == SRV_FLUID, storage, tau, sl.u_in, D, sl.k_sink);
}

// One launch of the batched step: ns steps of every running request in the
// table, the first being step t_off of the chunk; launch j reads buffer j & 1.
static void emu_step(int storage, int mode, int ns, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                     unsigned long long *part, int part_cap, int j, int t_off, int blocks, int ty)
{
    const SrvTable t = *tab;
    EMU_CHECK(t.n_active >= 0 && t.n_active <= SRV_MAX_SLOTS, "table holds %d entries", t.n_active);
    EMU_CHECK(blocks >= t.total_tiles, "grid of %d blocks for a table of %d tiles", blocks, t.total_tiles);
    EMU_CHECK(t.total_tiles <= part_cap, "table of %d tiles beyond %d check slots", t.total_tiles, part_cap);
    EMU_CHECK(t.begin[0] == 0 && t.begin[t.n_active] == t.total_tiles, "table offsets do not span its tiles");
    for (int e = 0; e < t.n_active; ++e) {
        const int sid = t.slot[e];
        EMU_CHECK(sid >= 0 && sid < SRV_MAX_SLOTS, "entry %d names slot %d", e, sid);
        const SrvSlot &sl = slots[sid];
        Ctrl *c = ctrl + sid;
        const int b0 = t.begin[e], nt = t.begin[e + 1] - b0;
        if (sl.phase == SRV_IDLE || c->stop != STOP_RUN)
            continue;
        EMU_CHECK(nt == pair_tiles(sl.g, ty), "entry %d spans %d tiles, its request has %d", e, nt,
                  pair_tiles(sl.g, ty));
        const bool fluid = sl.phase == SRV_FLUID;
        const void *src = fluid ? sl.f[j & 1] : sl.gp[j & 1];
        void *dst = fluid ? sl.f[(j & 1) ^ 1] : sl.gp[(j & 1) ^ 1];
        const emu::Hdr *h = read_hdr(src, sl.desc, sl.g, sl.phase, "step");
        EMU_CHECK(h->steps == c->t + t_off, "slot %d: launch %d of a chunk finds step %lld, expected %lld", sid, j,
                  h->steps, c->t + t_off);
        emu::Hdr *d = static_cast<emu::Hdr *>(dst);
        *d = *h;
        d->steps += ns;
        if (mode == MODE_CHECK) {
            EMU_CHECK(d->steps == c->t + c->K, "slot %d: check at step %lld, the chunk ends at %lld", sid, d->steps,
                      c->t + c->K);
            const emu::History hist = slot_history(sl, storage);
            const unsigned long long rb = emu::bits(emu::residual(hist, fluid, c->tol, d->steps));
            const unsigned long long ub = emu::bits(emu::umax(hist, fluid, d->steps));
            const int hot = (int)(d->steps / c->K) % nt; // the tile holding the maximum
            for (int v = 0; v < nt; ++v) {
                part[b0 + v] = v == hot ? rb : emu::bits(emu::from_bits(rb) * 0.25);
                part[part_cap + b0 + v] = v == hot ? ub : emu::bits(0.0);
            }
        }
    }
}

hipError_t srv_step(int storage, int mode, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                    unsigned long long *part, int part_cap, int j, int blocks, hipStream_t st)
{
    return enqueue(st, [=] {
        g_launch_pair.fetch_add(1);
        emu_step(storage, mode, 2, slots, tab, ctrl, part, part_cap, j, 2 * j, blocks, 4);
    });
}
hipError_t srv_stepN(int storage, int mode, int ns, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                     unsigned long long *part, int part_cap, int j, int t_off, int blocks, hipStream_t st)
{
    if (srv_tile_ty(storage) != 16 || (ns != 2 && ns != 4))
        return hipErrorInvalidValue;
    return enqueue(st, [=] {
        g_launch_wide.fetch_add(1);
        emu_step(storage, mode, ns, slots, tab, ctrl, part, part_cap, j, t_off, blocks, 16);
    });
}
hipError_t srv_decide(const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl, const unsigned long long *part,
                      int part_cap, hipStream_t st)
{
    return enqueue(st, [=] {
        const SrvTable t = *tab;
        for (int e = 0; e < t.n_active; ++e) {
            const int sid = t.slot[e];
            Ctrl *c = ctrl + sid;
            if (slots[sid].phase == SRV_IDLE || c->stop != STOP_RUN)
                continue;
            unsigned long long mr = 0, mu = 0;
            for (int v = t.begin[e]; v < t.begin[e + 1]; ++v) {
                mr = std::max(mr, part[v]);
                mu = std::max(mu, part[part_cap + v]);
            }
            emu::apply_rule(c, emu::from_bits(mr), emu::from_bits(mu));
        }
    });
}
hipError_t srv_ref_roll(const SrvSlot *slots, const SrvTable *tab, const Ctrl *ctrl, hipStream_t st)
{
    return enqueue(st, [=] {
        const SrvTable t = *tab;
        for (int e = 0; e < t.n_active; ++e) {
            const SrvSlot &sl = slots[t.slot[e]];
            if (sl.phase == SRV_IDLE || ctrl[t.slot[e]].stop != STOP_RUN)
                continue;
            for (int x = 0; x < sl.g.nx; ++x)
                sl.ref_cur[x] = sl.ref_next[x];
        }
    });
}

// ---- the single-domain solver's kernels (solver.cpp runs on these) -------
// A launch of ns steps of one solver: the stop flag first, as the real
// kernels; the source buffer must hold the state at the launch's step
// counter (the first launch after an init sets the counter's base); the
// check launch, which ends a chunk, writes every per-block maximum.
static void emu_solver_step(bool fluid, int mode, int ns, const void *src, void *dst, const void *desc, Ctrl *c,
                            const Geo &g, unsigned int step, double tau, double u_in, double D, double k_sink,
                            int storage)
{
    if (c->stop != STOP_RUN)
        return;
    const emu::Hdr *h = read_hdr(src, desc, g, fluid ? SRV_FLUID : SRV_AD, "solver step");
    emu::Hdr cur = *h;
    if (cur.fresh) {
        cur.fresh = 0;
        cur.base = cur.steps = (long long)step;
    }
    EMU_CHECK(cur.steps == (long long)step, "solver step: the source holds step %lld, the launch takes %u",
              cur.steps, step);
    cur.steps += ns;
    *static_cast<emu::Hdr *>(dst) = cur;
    if (mode == MODE_CHECK) {
        const long long t = c->t + c->K; // steps since the reset at the end of this chunk
        EMU_CHECK(cur.steps - cur.base >= t, "solver check at %lld steps of %lld", t, cur.steps - cur.base);
        const emu::History hist = emu::history(fluid, storage, tau, u_in, D, k_sink);
        const unsigned long long rb = emu::bits(emu::residual(hist, fluid, c->tol, t));
        const unsigned long long ub = emu::bits(emu::umax(hist, fluid, t));
        EMU_CHECK(c->part && c->nparts > 0, "check launch without per-block slots");
        for (int b = 0; b < c->nparts; ++b) {
            c->part[b] = b == (int)(t / c->K) % c->nparts ? rb : emu::bits(emu::from_bits(rb) * 0.5);
            c->part[c->nparts + b] = b == 0 ? ub : emu::bits(0.0);
        }
    }
}
static hipError_t fluid_launch(int mode, int ns, const FluidArgs &a, hipStream_t st, int storage)
{
    const FluidArgs b = a;
    return enqueue(st, [=] {
        emu_solver_step(true, mode, ns, b.src, b.dst, b.desc, b.ctrl, b.g, b.step, 1.0 / b.omega, b.u_in, 0.0, 0.0,
                        storage);
    });
}
static hipError_t ad_launch(int mode, int ns, const AdArgs &a, hipStream_t st, int storage)
{
    const AdArgs b = a;
    const double cs2 = b.g.nz > 1 ? 0.25 : 1.0 / 3.0;
    return enqueue(st, [=] {
        emu_solver_step(false, mode, ns, b.src, b.dst, b.desc, b.ctrl, b.g, b.step, 0.0, 0.0,
                        (1.0 / b.omega - 0.5) * cs2, b.k_sink, storage);
    });
}
hipError_t fluid_step(int, int storage, int mode, const FluidArgs &a, hipStream_t st)
{
    return fluid_launch(mode, 1, a, st, storage);
}
hipError_t ad_step(int, int storage, int mode, const AdArgs &a, hipStream_t st)
{
    return ad_launch(mode, 1, a, st, storage);
}
hipError_t fluid_step2(int storage, int mode, const FluidArgs &a, hipStream_t st)
{
    return fluid_launch(mode, 2, a, st, storage);
}
hipError_t ad_step2(int, int storage, int mode, const AdArgs &a, hipStream_t st)
{
    return ad_launch(mode, 2, a, st, storage);
}
hipError_t fluid_stepN(int storage, int mode, int ns, const FluidArgs &a, hipStream_t st)
{
    EMU_CHECK(ns >= 3 && ns <= 4, "fluid_stepN of %d steps", ns);
    return fluid_launch(mode, ns, a, st, storage);
}
hipError_t ad_stepN(int, int storage, int mode, int ns, const AdArgs &a, hipStream_t st)
{
    EMU_CHECK(ns >= 3 && ns <= 4, "ad_stepN of %d steps", ns);
    return ad_launch(mode, ns, a, st, storage);
}
hipError_t fluid_step3d2(int storage, int mode, const FluidArgs &a, hipStream_t st)
{
    return fluid_launch(mode, 2, a, st, storage);
}
hipError_t ad_step3d2(int storage, int mode, const AdArgs &a, hipStream_t st)
{
    return ad_launch(mode, 2, a, st, storage);
}
hipError_t decide(Ctrl *c, hipStream_t st)
{
    return enqueue(st, [=] {
        if (c->stop != STOP_RUN)
            return;
        unsigned long long mr = 0, mu = 0;
        for (int b = 0; b < c->nparts; ++b) {
            mr = std::max(mr, c->part[b]);
            mu = std::max(mu, c->part[c->nparts + b]);
        }
        emu::apply_rule(c, emu::from_bits(mr), emu::from_bits(mu));
    });
}
hipError_t ref_roll(const Ctrl *ctrl, float *cur, const float *next, int n, hipStream_t st)
{
    return enqueue(st, [=] {
        if (ctrl->stop != STOP_RUN)
            return;
        for (int k = 0; k < n; ++k)
            cur[k] = next[k];
    });
}
hipError_t copy_kernel(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    return enqueue(st, [=] { memcpy(dst, src, bytes); });
}
hipError_t pops_export(int, int, int, const void *, const void *, const Geo &, const float *, double *, hipStream_t)
{
    emu_fail("pops_export is not emulated");
    return hipErrorInvalidValue;
}
hipError_t pops_import(int, int, int, void *, const void *, const Geo &, const float *, const double *, hipStream_t)
{
    emu_fail("pops_import is not emulated");
    return hipErrorInvalidValue;
}
// cell updates: the stub state has no populations to set; the node list
// must lie in the grid
hipError_t pops_set_nodes(int, int, int, void *, const Geo &g, const float *, const long long *idx, int count,
                          const double *, hipStream_t st)
{
    return enqueue(st, [=] {
        for (int k = 0; k < count; ++k)
            EMU_CHECK(idx[k] >= 0 && idx[k] < g.N, "cell update of node %lld outside the grid", idx[k]);
    });
}
size_t compute_bytes(int s) { return s == ST_F64 ? 8 : 4; }
// four-step launches on larger grids, two-step ones below (both forms of
// the steady loop's plans)
int fluid_launch_steps(int storage, const Geo &g) { return storage != ST_F64 && g.N >= 8192 ? 4 : 2; }
int pair_ty(int, const Geo &) { return 4; }
int z3_tile_y(const Geo &) { return 16; }
int z3_planes_per_block(const Geo &g, int, int) { return g.nz < 4 ? g.nz : 4; }
int z3_blocks(const Geo &g, int zseg, int ty)
{
    return ((g.nx + 31) / 32) * ((g.ny + ty - 1) / ty) * ((g.nz + zseg - 1) / zseg);
}

} // namespace lbmk

// ---------------------------------------------------- single-domain solver
// solver.cpp and api.cpp run as they are; the HIP calls they add
extern "C" {
hipError_t hipGetDeviceCount(int *n)
{
    *n = 1;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new ihipEvent_t();
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    EMU_CHECK(hipEventSynchronize(a) == hipSuccess && hipEventSynchronize(b) == hipSuccess, "event wait");
    *ms = 1.0f;
    return hipSuccess;
}
} // extern "C"

// ------------------------------------------- bio-electrochemical state
// bio.hip's host side, reduced to the host mirrors the agent-based biofilm
// (biofilm.cpp) reads and writes: no device arrays and no mediator balance
lbm_status lbmh::bio_pull_mox(lbm_bio *b)
{
    b->mox_stale = false;
    return LBM_OK;
}
lbm_status lbmh::bio_push_cells(lbm_bio *b)
{
    b->cells.clear();
    b->sum_cb = 0.0;
    for (size_t n = 0; n < b->cb.size(); ++n)
        if (b->cb[n] > 0.0) {
            b->cells.push_back((int32_t)n);
            b->sum_cb += b->cb[n];
        }
    b->biomass = b->sum_cb;
    return LBM_OK;
}
extern "C" lbm_status lbm_bio_step(lbm_bio *b, lbm_bio_out *out)
{
    memset(out, 0, sizeof(*out));
    out->n_cells = (int32_t)b->cells.size();
    out->biomass = b->biomass;
    return LBM_OK;
}

// ----------------------------------------------------------------- driver
namespace {

struct Expect {
    int status, lane, first_status;
    long long it_f, it_a, first_f, first_a;
    bool ad_ran, first_ad_ran;
    int64_t nf, na; // nodes each solver updates
};

struct Attempt {
    int st_f, st_a;
    long long it_f, it_a;
    bool ad_ran;
    int overall;
};

int worse(int a, int b)
{
    if (a == LBM_EDIVERGED || b == LBM_EDIVERGED)
        return LBM_EDIVERGED;
    if (a == LBM_NOT_CONVERGED || b == LBM_NOT_CONVERGED)
        return LBM_NOT_CONVERGED;
    if (a == LBM_STALLED || b == LBM_STALLED)
        return LBM_STALLED;
    return LBM_OK;
}

Attempt attempt(const lbm_request &r, int storage, int K, int window)
{
    Attempt a{};
    const long long mi = (r.max_iter + K - 1) / K * K;
    const emu::Outcome f =
        emu::solve(emu::history(true, storage, r.tau, r.u_in, r.D, r.k_sink), true, r.tol, K, window, mi);
    a.st_f = f.status;
    a.it_f = f.iters;
    a.st_a = f.status;
    if (f.status != LBM_EDIVERGED) {
        const emu::Outcome g =
            emu::solve(emu::history(false, storage, r.tau, r.u_in, r.D, r.k_sink), false, r.tol, K, window, mi);
        a.st_a = g.status;
        a.it_a = g.iters;
        a.ad_ran = true;
    }
    a.overall = worse(a.st_f, a.st_a);
    return a;
}

// Whether the server accepts the request's medium, and the nodes each
// solver updates on it
bool mask_valid(const lbm_request &r, int64_t *nf = nullptr, int64_t *na = nullptr)
{
    const lbm_grid g{r.nx, r.ny, 1};
    std::vector<uint8_t> cls((size_t)r.nx * r.ny);
    double got = 0;
    if (lbm_geom_discs(g, &r.discs, r.seed, cls.data(), &got) != LBM_OK)
        return false;
    if (r.layer)
        lbm_biofilm_layer(g, cls.data());
    if (!lbmh::check_mask(g, cls.data()).empty())
        return false;
    const std::vector<uint8_t> dom = lbmh::flow_domain(g, cls.data());
    if (nf && na) {
        *nf = *na = 0;
        for (size_t n = 0; n < cls.size(); ++n) {
            *nf += dom[n] != 0;
            *na += cls[n] == LBM_FLUID || cls[n] == LBM_BIOFILM;
        }
    }
    return lbmh::domain_reaches_inlet(g, dom);
}

struct Config {
    const char *name;
    int storage, K, stall, inflight, direct, escalate, slots, lanes, prep;
    int64_t solo_nodes;
    size_t pool;
    int n_req;
    uint64_t seed;
    int burst;          // submit without pauses
    long long fail_after; // > 0: the device fails after this many queued operations
};

Expect expect(const lbm_request &r, const Config &c)
{
    Expect e{};
    const int K = c.K;
    const int window = c.stall < 0 ? 0 : (c.stall ? c.stall : lbmh::default_stall_checks(c.storage, K));
    const int64_t N = (int64_t)r.nx * r.ny;
    e.lane = c.solo_nodes > 0 && N >= c.solo_nodes ? LBM_LANE_SOLO : LBM_LANE_BATCH;
    if (!mask_valid(r, &e.nf, &e.na)) {
        e.status = LBM_EINVAL;
        return e;
    }
    Attempt a = attempt(r, c.storage, K, window);
    const bool may = c.escalate && (c.storage == LBM_FP16_SHIFTED || c.storage == LBM_FP32);
    if (may && a.overall != LBM_OK) {
        e.lane = LBM_LANE_ESCALATED;
        e.first_status = a.overall;
        e.first_f = a.it_f;
        e.first_a = a.it_a;
        e.first_ad_ran = a.ad_ran;
        a = attempt(r, LBM_FP32_SHIFTED, 100, lbmh::default_stall_checks(LBM_FP32_SHIFTED, 100));
    }
    e.status = a.overall;
    e.it_f = a.it_f;
    e.it_a = a.it_a;
    e.ad_ran = a.ad_ran;
    return e;
}

std::vector<lbm_request> make_requests(const Config &c)
{
    std::mt19937_64 rng(c.seed);
    auto uni = [&](double lo, double hi) { return lo + (hi - lo) * (double)(rng() >> 11) * (1.0 / 9007199254740992.0); };
    std::vector<lbm_request> v;
    const double taus[] = {0.65, 0.65, 0.65, 0.75, 0.85, 0.95};
    for (int i = 0; i < c.n_req; ++i) {
        lbm_request r{};
        r.nx = 16 + (int)(rng() % 150);
        r.ny = 8 + (int)(rng() % 72);
        r.discs.r_min = 1;
        r.discs.r_max = 3;
        r.discs.solid_frac = uni(0.05, 0.45);
        r.discs.overlap = (int)(rng() & 1);
        r.seed = 1000 + rng() % 100000;
        r.layer = (int)(rng() % 3 == 0);
        r.tau = taus[rng() % 6];
        r.u_in = (double)(5 + rng() % 60) * 1e-4 * (rng() % 2 ? 1.0 : -1.0);
        r.D = (double)(2 + rng() % 40) * 1e-3;
        const double ks[] = {0.1, 0.2, 0.3, 0.55, 0.75};
        r.k_sink = ks[rng() % 5];
        r.c_in = 1.0;
        r.outlet = LBM_OUT_ZERO_GRADIENT;
        r.tol = 1e-6;
        r.max_iter = rng() % 8 == 0 ? 300 + (long long)(rng() % 400) : 1000000;
        r.user = (uint64_t)i;
        v.push_back(r);
    }
    return v;
}

void run_config(const Config &c)
{
    lbm_ctx *ctx = nullptr;
    EMU_CHECK(lbm_ctx_create(0, nullptr, &ctx) == LBM_OK, "context");
    lbm_server_cfg cfg{};
    cfg.pool_bytes = c.pool;
    cfg.max_slots = c.slots;
    cfg.storage = c.storage;
    cfg.check_every = c.K;
    cfg.stall_checks = c.stall;
    cfg.inflight = c.inflight;
    cfg.prep_threads = c.prep;
    cfg.direct_launch = c.direct;
    cfg.escalate = c.escalate;
    cfg.solo_nodes = c.solo_nodes;
    cfg.solo_lanes = c.lanes;
    lbm_server *s = nullptr;
    EMU_CHECK(lbm_server_create(ctx, &cfg, &s) == LBM_OK, "%s: server create: %s", c.name, lbm_last_error(ctx));
    const bool failing = c.fail_after > 0;
    if (failing) {
        g_ops = 0;
        g_fail_at = c.fail_after;
    }
    const std::vector<lbm_request> reqs = make_requests(c);
    std::vector<Expect> exp;
    for (const auto &r : reqs)
        exp.push_back(expect(r, c));

    std::atomic<int> submitted{0}, received{0}, bad_submit{0}, accepted{0}, target{-1}, n_device{0};
    std::atomic<bool> stop_stats{false};
    std::thread stats([&] {
        while (!stop_stats.load()) {
            lbm_server_stats_t st;
            (void)lbm_server_stats(s, &st);
            std::this_thread::sleep_for(std::chrono::microseconds(300));
        }
    });
    std::vector<std::thread> subs;
    const int NS = 3;
    for (int k = 0; k < NS; ++k)
        subs.emplace_back([&, k] {
            std::mt19937 rng(77 + k);
            for (size_t i = k; i < reqs.size(); i += NS) {
                uint64_t t = 0;
                const lbm_status st = lbm_server_submit(s, &reqs[i], &t);
                if (st == LBM_OK)
                    accepted.fetch_add(1);
                else if (!(failing && st == LBM_EDEVICE))
                    bad_submit.fetch_add(1);
                submitted.fetch_add(1);
                if (!c.burst)
                    std::this_thread::sleep_for(std::chrono::microseconds(rng() % 400));
            }
        });
    std::vector<int> seen(reqs.size(), 0);
    std::thread poller([&] {
        std::vector<lbm_result> out(8);
        while (target.load() < 0 || received.load() < target.load()) {
            int n = 0;
            EMU_CHECK(lbm_server_poll(s, out.data(), (int)out.size(), &n, 0.05) == LBM_OK, "poll");
            for (int k = 0; k < n; ++k) {
                lbm_result &r = out[k];
                EMU_CHECK(r.user < reqs.size(), "%s: unknown user tag %llu", c.name, (unsigned long long)r.user);
                const lbm_request &q = reqs[r.user];
                Expect e = exp[r.user];
                if (failing && e.lane == LBM_LANE_ESCALATED && r.lane == LBM_LANE_SOLO) {
                    // a solo-lane first attempt that ended after the failure
                    // is returned as it is: nothing is escalated any more
                    e.status = e.first_status;
                    e.lane = LBM_LANE_SOLO;
                    e.it_f = e.first_f;
                    e.it_a = e.first_a;
                    e.ad_ran = e.first_ad_ran;
                }
                EMU_CHECK(!seen[r.user]++, "%s: request %llu returned twice", c.name, (unsigned long long)r.user);
                if (failing && r.status == LBM_EDEVICE) {
                    n_device.fetch_add(1);
                    lbm_result_release(s, &r);
                    received.fetch_add(1);
                    continue;
                }
                EMU_CHECK(r.status == e.status, "%s: request %llu status %d, expected %d (%s)", c.name,
                          (unsigned long long)r.user, r.status, e.status, r.message);
                if (e.status != LBM_EINVAL) {
                    EMU_CHECK(r.lane == e.lane, "%s: request %llu lane %d, expected %d", c.name,
                              (unsigned long long)r.user, r.lane, e.lane);
                    EMU_CHECK(r.iters_fluid == e.it_f && r.iters_ad == e.it_a,
                              "%s: request %llu steps %lld + %lld, expected %lld + %lld", c.name,
                              (unsigned long long)r.user, (long long)r.iters_fluid, (long long)r.iters_ad, e.it_f,
                              e.it_a);
                    if (e.lane == LBM_LANE_ESCALATED)
                        EMU_CHECK(r.first_status == e.first_status && r.first_iters_fluid == e.first_f &&
                                      r.first_iters_ad == e.first_a,
                                  "%s: request %llu first attempt %d %lld + %lld, expected %d %lld + %lld", c.name,
                                  (unsigned long long)r.user, r.first_status, (long long)r.first_iters_fluid,
                                  (long long)r.first_iters_ad, e.first_status, e.first_f, e.first_a);
                    const int64_t N = (int64_t)q.nx * q.ny;
                    EMU_CHECK(r.u && r.c, "%s: request %llu without fields", c.name, (unsigned long long)r.user);
                    const float cu = (float)e.it_f, cc = e.ad_ran ? (float)e.it_a : 0.0f;
                    EMU_CHECK(r.u[0] == cu && r.u[2 * N - 1] == cu && r.c[0] == cc && r.c[N - 1] == cc,
                              "%s: request %llu fields from another state: u %g, c %g, expected %g, %g", c.name,
                              (unsigned long long)r.user, r.u[0], r.c[0], cu, cc);
                    EMU_CHECK(r.flux[0] == (double)e.it_f && r.flux[2] == (double)cc,
                              "%s: request %llu fluxes %g %g, expected %lld %g", c.name, (unsigned long long)r.user,
                              r.flux[0], r.flux[2], e.it_f, (double)cc);
                }
                lbm_result_release(s, &r);
                received.fetch_add(1);
            }
        }
    });
    for (auto &t : subs)
        t.join();
    EMU_CHECK(bad_submit.load() == 0, "%s: %d submissions refused", c.name, bad_submit.load());
    target = accepted.load();
    const lbm_status d = lbm_server_drain(s, 120.0);
    if (failing) {
        EMU_CHECK(d == LBM_EDEVICE, "%s: drain returned %d after a device failure", c.name, (int)d);
        EMU_CHECK(strstr(lbm_server_error(s), "HIP error") != nullptr, "%s: error text '%s'", c.name,
                  lbm_server_error(s));
    } else {
        EMU_CHECK(d == LBM_OK, "%s: drain returned %d (stall)", c.name, (int)d);
    }
    poller.join();
    g_fail_at = -1;
    stop_stats = true;
    stats.join();
    lbm_server_stats_t st;
    EMU_CHECK(lbm_server_stats(s, &st) == LBM_OK, "stats");
    if (failing) {
        EMU_CHECK(st.finished == (int64_t)accepted.load() && n_device.load() > 0,
                  "%s: after the failure: %lld finished of %d accepted, %d failed", c.name, (long long)st.finished,
                  accepted.load(), n_device.load());
        lbm_server_destroy(s);
        lbm_ctx_destroy(ctx);
        printf("%s: %d of %zu requests accepted, %d ended by the device failure\n", c.name, accepted.load(),
               reqs.size(), n_device.load());
        fflush(stdout);
        return;
    }
    EMU_CHECK(st.finished == (int64_t)reqs.size() && st.active == 0 && st.queued == 0 && st.pool_used == 0,
              "%s: after the drain: finished %lld, active %lld, queued %lld, pool %llu", c.name,
              (long long)st.finished, (long long)st.active, (long long)st.queued, (unsigned long long)st.pool_used);
    lbm_server_destroy(s);
    lbm_ctx_destroy(ctx);
    int esc = 0, solo = 0, inval = 0;
    for (const auto &e : exp) {
        esc += e.status != LBM_EINVAL && e.lane == LBM_LANE_ESCALATED;
        solo += e.status != LBM_EINVAL && e.lane == LBM_LANE_SOLO;
        inval += e.status == LBM_EINVAL;
    }
    const bool wide_possible = emu::served_ty() == 16 && c.storage != LBM_FP16_SHIFTED;
    EMU_CHECK(st.chunks_wide <= st.chunks && (wide_possible || st.chunks_wide == 0),
              "%s: %lld of %lld chunks wide", c.name, (long long)st.chunks_wide, (long long)st.chunks);
    // lattice updates of every solve, the discarded first attempts included
    double upd = 0.0;
    for (const auto &e : exp) {
        if (e.status == LBM_EINVAL)
            continue;
        upd += (double)e.it_f * e.nf + (double)e.it_a * e.na;
        if (e.lane == LBM_LANE_ESCALATED)
            upd += (double)e.first_f * e.nf + (double)e.first_a * e.na;
    }
    EMU_CHECK(st.lattice_updates == upd, "%s: lattice updates %.0f, expected %.0f", c.name, st.lattice_updates, upd);
    EMU_CHECK(st.rejected == inval && st.solo == solo + esc && st.escalated == esc,
              "%s: statistics: rejected %lld, solo %lld, escalated %lld; expected %d, %d, %d", c.name,
              (long long)st.rejected, (long long)st.solo, (long long)st.escalated, inval, solo + esc, esc);
    printf("%s: %zu requests (%d solo, %d escalated, %d rejected masks), %lld chunks (%lld wide); launches so "
           "far: %lld paired, %lld wide\n", c.name, reqs.size(), solo, esc, inval, (long long)st.chunks,
           (long long)st.chunks_wide, g_launch_pair.load(), g_launch_wide.load());
    fflush(stdout);
}

// Shutdown with work in flight: requests queued, being prepared, stepped,
// retiring, on the solo lanes and finished but not polled, some results
// polled and not released.  lbm_server_destroy must stop every thread and
// free everything (the sanitizers check the rest).
void run_destroy_in_flight(int storage, uint64_t seed, int wait_ms)
{
    lbm_ctx *ctx = nullptr;
    EMU_CHECK(lbm_ctx_create(0, nullptr, &ctx) == LBM_OK, "context");
    lbm_server_cfg cfg{};
    cfg.pool_bytes = (size_t)2 << 20;
    cfg.max_slots = 6;
    cfg.storage = storage;
    cfg.check_every = 20;
    cfg.stall_checks = 5;
    cfg.prep_threads = 3;
    cfg.escalate = storage == LBM_FP16_SHIFTED;
    cfg.solo_nodes = 6000;
    cfg.solo_lanes = 2;
    lbm_server *s = nullptr;
    EMU_CHECK(lbm_server_create(ctx, &cfg, &s) == LBM_OK, "server create: %s", lbm_last_error(ctx));
    Config c{"destroy in flight", storage, 20, 5, 2, 0, 0, 6, 2, 3, 6000, (size_t)2 << 20, 60, seed, 1, 0};
    const std::vector<lbm_request> reqs = make_requests(c);
    for (const auto &r : reqs) {
        uint64_t t = 0;
        EMU_CHECK(lbm_server_submit(s, &r, &t) == LBM_OK, "submit: %s", lbm_server_error(s));
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(wait_ms));
    lbm_result out[4];
    int n = 0;
    EMU_CHECK(lbm_server_poll(s, out, 4, &n, 0.0) == LBM_OK, "poll");
    if (n > 1)
        lbm_result_release(s, &out[0]); // the others stay unreleased
    lbm_server_destroy(s);
    lbm_ctx_destroy(ctx);
    printf("destroy in flight (storage %d, after %d ms): %d results polled before\n", storage, wait_ms, n);
    fflush(stdout);
}

// The coupled biofilm loop (lbm_coupled_run: growth pick, cell update,
// warm re-solves) on its own context, with the stub kernels: every re-solve
// takes the steps the history gives, every pick becomes BIOFILM; then a
// checkpoint and restore.
void run_coupled(uint64_t seed, int n_updates, std::atomic<int> *ran)
{
    lbm_ctx *ctx = nullptr;
    EMU_CHECK(lbm_ctx_create(0, nullptr, &ctx) == LBM_OK, "context");
    const lbm_grid g{96, 48, 1};
    lbm_disc_params dp{3, 6, 0.3, 1};
    std::vector<uint8_t> cls((size_t)g.nx * g.ny);
    double got = 0;
    EMU_CHECK(lbm_geom_discs(g, &dp, seed, cls.data(), &got) == LBM_OK, "discs");
    lbm_biofilm_layer(g, cls.data());
    if (!lbmh::domain_reaches_inlet(g, lbmh::flow_domain(g, cls.data()))) {
        lbm_ctx_destroy(ctx);
        return; // a medium that does not percolate: no loop
    }
    lbm_params p{};
    p.tau = 0.65;
    p.u_in = 0.0031;
    p.D = 0.012;
    p.c_in = 1.0;
    p.k_sink = 0.2;
    p.storage = LBM_FP32_SHIFTED;
    lbm_solver *sv = nullptr;
    EMU_CHECK(lbm_solver_create(ctx, g, cls.data(), &p, &sv) == LBM_OK, "solver: %s", lbm_last_error(ctx));
    std::vector<double> xi(n_updates), J(n_updates + 1);
    std::vector<int64_t> picked(n_updates), itf(n_updates + 1), ita(n_updates + 1);
    for (int m = 0; m < n_updates; ++m)
        xi[m] = (double)((seed * 7919 + m * 104729) % 1000) / 1000.0;
    double Jacc = -1.0;
    const lbm_status st = lbm_coupled_run(sv, n_updates, xi.data(), 1e-6, 200000, picked.data(), J.data(), &Jacc,
                                          itf.data(), ita.data());
    EMU_CHECK(st == LBM_OK, "coupled loop returned %d: %s", (int)st, lbm_last_error(ctx));
    const emu::Outcome f = emu::solve(emu::history(true, p.storage, p.tau, p.u_in, p.D, p.k_sink), true, 1e-6, 100,
                                      1000, 200000);
    const emu::Outcome a = emu::solve(emu::history(false, p.storage, p.tau, p.u_in, p.D, p.k_sink), false, 1e-6,
                                      100, 1000, 200000);
    for (int m = 0; m <= n_updates; ++m)
        EMU_CHECK(itf[m] == f.iters && ita[m] == a.iters, "coupled update %d: %lld + %lld steps, expected %lld + %lld",
                  m, (long long)itf[m], (long long)ita[m], f.iters, a.iters);
    std::vector<uint8_t> fin(cls.size());
    EMU_CHECK(lbm_solver_get(sv, LBM_FIELD_CLASS, fin.data()) == LBM_OK, "class field");
    for (int m = 0; m < n_updates; ++m)
        EMU_CHECK(picked[m] >= 0 && fin[(size_t)picked[m]] == LBM_BIOFILM, "pick %d (%lld) is not BIOFILM", m,
                  (long long)picked[m]);
    // checkpoint, two warm re-solves, restore, the same two again: the
    // restored solver continues from the saved state and step counters
    size_t bytes = 0;
    EMU_CHECK(lbm_solver_state_size(sv, &bytes) == LBM_OK && bytes > 0, "state size");
    std::vector<char> saved(bytes);
    EMU_CHECK(lbm_solver_get_state(sv, saved.data(), bytes) == LBM_OK, "get state: %s", lbm_last_error(ctx));
    lbm_info i1{}, i2{}, i3{}, i4{};
    EMU_CHECK(lbm_solver_fluid(sv, 1e-6, 200000, 1, &i1) == LBM_OK && lbm_solver_ad(sv, 1e-6, 200000, 1, &i2) ==
                  LBM_OK, "solves after the checkpoint");
    EMU_CHECK(lbm_solver_put_state(sv, saved.data(), bytes) == LBM_OK, "put state: %s", lbm_last_error(ctx));
    EMU_CHECK(lbm_solver_fluid(sv, 1e-6, 200000, 1, &i3) == LBM_OK && lbm_solver_ad(sv, 1e-6, 200000, 1, &i4) ==
                  LBM_OK, "solves after the restore");
    EMU_CHECK(i1.iters == i3.iters && i2.iters == i4.iters && i1.iters == f.iters,
              "restored solves took %lld + %lld steps against %lld + %lld", (long long)i3.iters, (long long)i4.iters,
              (long long)i1.iters, (long long)i2.iters);
    lbm_solver_destroy(sv);
    lbm_ctx_destroy(ctx);
    ran->fetch_add(1);
}

// The hourly model loop (lbm_mfc_run: solves, bio step, agent-based
// biofilm with attachment, growth and spreading by random walks) on the
// real solver with the stub kernels.  Biomass sits only on BIOFILM nodes,
// and spreading moves it without loss.
void run_mfc(uint64_t seed, int hours)
{
    lbm_ctx *ctx = nullptr;
    EMU_CHECK(lbm_ctx_create(0, nullptr, &ctx) == LBM_OK, "context");
    const lbm_grid g{96, 48, 1};
    lbm_disc_params dp{3, 6, 0.25, 1};
    std::vector<uint8_t> cls((size_t)g.nx * g.ny);
    double got = 0;
    EMU_CHECK(lbm_geom_discs(g, &dp, seed, cls.data(), &got) == LBM_OK, "discs");
    if (!lbmh::domain_reaches_inlet(g, lbmh::flow_domain(g, cls.data()))) {
        lbm_ctx_destroy(ctx);
        return;
    }
    lbm_params p{};
    p.tau = 0.65;
    p.u_in = 0.0031;
    p.D = 0.012;
    p.c_in = 1.0;
    p.k_sink = 0.2;
    p.storage = LBM_FP32_SHIFTED;
    lbm_solver *sv = nullptr;
    EMU_CHECK(lbm_solver_create(ctx, g, cls.data(), &p, &sv) == LBM_OK, "solver: %s", lbm_last_error(ctx));
    lbm_bio b;
    b.s = sv;
    b.p.q_max = 8.0;
    b.p.K_s = 20.0;
    b.p.M_total = 0.05;
    b.p.K_Mox = 0.01;
    b.p.C0_bio = 450.0;
    b.p.c_scale = 1.0; // the stub concentration is a step count: fast growth
    b.p.dt_hours = 1.0;
    b.cb.assign(cls.size(), 0.0);
    b.mox.assign(cls.size(), 0.0);
    lbm_biofilm_params fp{};
    fp.k_ata = 15;
    fp.C_max = 500.0;
    fp.fr_spr = 0.4;
    fp.max_walk = 40;
    fp.Y_bio = 1.0;
    std::vector<lbm_mfc_interval> series((size_t)hours);
    const lbm_status st = lbm_mfc_run(&b, &fp, hours, seed, 1e-6, 200000, series.data());
    EMU_CHECK(st == LBM_OK || st == LBM_EINVAL, "model loop returned %d: %s", (int)st, lbm_last_error(ctx));
    std::vector<uint8_t> fin(cls.size());
    EMU_CHECK(lbm_solver_get(sv, LBM_FIELD_CLASS, fin.data()) == LBM_OK, "class field");
    for (size_t n = 0; n < fin.size(); ++n)
        EMU_CHECK(!(b.cb[n] > 0.0) || fin[n] == LBM_BIOFILM, "biomass on node %zu of class %d", n, (int)fin[n]);
    int spread = 0, walks = 0;
    for (const auto &r : series) {
        spread += r.film.spread;
        walks += r.film.walks;
    }
    lbm_solver_destroy(sv);
    lbm_ctx_destroy(ctx);
    printf("model loop (seed %llu): %s, %d spreadings, %d random walks\n", (unsigned long long)seed,
           st == LBM_OK ? "OK" : "stopped (growth would close the flow path)", spread, walks);
    fflush(stdout);
}

} // namespace

int main(int argc, char **argv)
{
    const int scale = argc > 1 ? atoi(argv[1]) : 1;
    const size_t MB = (size_t)1 << 20;
    // name, storage, K, stall checks, inflight, direct, escalate, slots, solo lanes, prep threads,
    // solo nodes, pool, requests, seed, burst
    const Config cfgs[] = {
        {"fp32s graphs", LBM_FP32_SHIFTED, 20, 5, 2, 0, 0, 8, 2, 2, 6000, 2 * MB, 40 * scale, 1, 0, 0},
        {"fp32s direct depth 3", LBM_FP32_SHIFTED, 16, 4, 3, 1, 0, 4, 1, 1, -1, 2 * MB, 30 * scale, 2, 0, 0},
        {"fp16s escalate", LBM_FP16_SHIFTED, 20, 5, 2, 0, 1, 8, 3, 3, 6000, 2 * MB, 40 * scale, 3, 0, 0},
        {"fp32 escalate depth 1", LBM_FP32, 12, 3, 1, 0, 1, 6, 2, 2, 9000, (size_t)3 * MB / 2, 30 * scale, 4, 0, 0},
        // a burst prepared by four threads, which finish out of ticket order
        {"fp32s burst", LBM_FP32_SHIFTED, 8, 3, 2, 0, 0, 3, 1, 4, -1, 4 * MB, 60 * scale, 5, 1, 0},
        // the device fails while requests are queued, prepared, stepped,
        // retiring and on the solo lanes: every accepted request still comes
        // back once (its result, or EDEVICE) and the drain reports the failure
        {"fp32s device failure", LBM_FP32_SHIFTED, 20, 5, 2, 0, 0, 6, 2, 4, 6000, 2 * MB, 40 * scale, 6, 1, 300},
        {"fp16s escalate device failure", LBM_FP16_SHIFTED, 20, 5, 2, 1, 1, 6, 2, 4, 6000, 2 * MB, 40 * scale, 7, 1,
         900},
    };
    for (const Config &c : cfgs)
        run_config(c);
    for (int w : {0, 3, 30})
        run_destroy_in_flight(w == 3 ? LBM_FP16_SHIFTED : LBM_FP32_SHIFTED, 11 + (uint64_t)w, w);
    {
        // three coupled loops at once, each with its own context and stream
        std::atomic<int> ran{0};
        std::vector<std::thread> loops;
        for (uint64_t sd : {21, 22, 23})
            loops.emplace_back([sd, &ran] { run_coupled(sd, 12, &ran); });
        for (auto &t : loops)
            t.join();
        EMU_CHECK(ran.load() >= 2, "only %d coupled loops ran", ran.load());
        printf("coupled loops: %d x 12 updates\n", ran.load());
    }
    for (uint64_t sd : {31, 32})
        run_mfc(sd, 8);
    printf("ok\n");
    return 0;
}

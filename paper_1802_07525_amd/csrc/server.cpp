// server.cpp -- served form: continuous batching of 2-D steady solves.
//
// A request is one 2-D steady problem of the paper's model loop (Sec. 2):
// the fluid solve (Sec. 2.1.1) to its residual tolerance, then the
// substrate solve (Sec. 2.1.2) in the exported velocity.  The server keeps
// every admitted request's populations resident in one device pool and
// steps all of them together:
//
//  * Submission copies the request; host preparation threads build its
//    mask (seeded discs or the caller's classes), check it and turn it into
//    descriptor words.
//  * A worker thread admits prepared requests in ticket order while a slot
//    is free and the request's footprint fits the pool (first fit), uploads
//    the descriptors through a pinned ring, initialises the request on the
//    device and adds its tiles to the device slot table.
//  * Work proceeds in chunks of K steps: launches of the batched step
//    kernel (each advances every tile of every admitted request by two or
//    four steps, in that request's phase) and one batched decide, captured once
//    as a HIP graph
//    that reads the slot table from device memory, so admissions never
//    re-capture it.  After each chunk the control blocks are copied to
//    pinned memory; the host keeps a bounded number of chunks in flight.
//  * When a snapshot shows a request's fluid solve stopped, the worker
//    enqueues the velocity export and the substrate start for it; when the
//    substrate solve stops, the concentration export and the result copy.
//    The request leaves the table, and its slot and pool range are free for
//    the next admission at once: all device work is on one stream, so
//    whatever uses them next is ordered behind the result copy.  The result
//    is handed out when that copy has completed.
//
// A request's arithmetic is that of a single solve with the same storage:
// the same per-tile code, the same step counters, the same check steps.
// Its results are therefore the same alone and in any mix, bit for bit.
//
// A solo lane -- one more host thread with a context and stream of its own
// -- runs whole requests through the single-domain solver next to the
// batch: requests large enough to fill the GPU alone (the single solver's
// wider multi-step launches serve them faster than the batch's two-step
// tiles), and, when escalation is on, reduced-storage requests whose
// batched solves did not both end OK, solved again in FP32-shifted storage.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lbm_internal.h"

using namespace lbmh;

namespace {

const size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// Per-request device buffers, in pool order.
struct Layout {
    size_t desc, f0, f1, u, prev, ref, total;
};

Layout layout_of(int32_t nx, int64_t N, int storage)
{
    const size_t sb = lbmk::storage_bytes(storage);
    Layout L;
    size_t o = 0;
    L.desc = o;
    o += align_up((size_t)N * 2);
    L.f0 = o;
    o += align_up((size_t)N * 9 * sb);
    L.f1 = o;
    o += align_up((size_t)N * 9 * sb);
    L.u = o;
    o += align_up((size_t)N * 2 * 4);
    L.prev = o;
    o += align_up((size_t)N * 2 * 4);
    L.ref = o; // column references: current, next
    o += align_up((size_t)nx * 2 * sizeof(float));
    L.total = o;
    return L;
}

// First-fit sub-allocator over the device pool; adjacent free ranges merge.
class PoolAlloc {
public:
    void reset(size_t bytes)
    {
        free_.clear();
        if (bytes)
            free_[0] = bytes;
        cap = bytes;
        used = peak = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes)
                continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o = it->first + bytes;
            free_.erase(it);
            if (rest)
                free_[o] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
        used -= bytes;
    }
    size_t cap = 0, used = 0, peak = 0;

private:
    std::map<size_t, size_t> free_;
};

// Pinned host staging ring for asynchronous copies.  Ranges are taken in
// FIFO order; a range is reused only after the event recorded behind its
// copy has completed and its owner (if any) has been handed to `reclaim`,
// which must read the data out.  Copies complete in stream order, so the
// ring reclaims from the front.
class PinnedRing {
public:
    std::function<void(void *)> reclaim;
    ~PinnedRing() { destroy(); }
    hipError_t init(size_t bytes)
    {
        cap_ = bytes;
        return hipHostMalloc((void **)&base_, bytes, hipHostMallocDefault);
    }
    void destroy()
    {
        for (auto &u : uses_)
            (void)hipEventSynchronize(u.ev), spare_.push_back(u.ev);
        uses_.clear();
        for (hipEvent_t e : spare_)
            (void)hipEventDestroy(e);
        spare_.clear();
        if (base_)
            (void)hipHostFree(base_);
        base_ = nullptr;
    }
    bool empty() const { return uses_.empty(); }
    // Reclaim every range whose copy has completed; with wait, also the
    // oldest one still in flight.
    hipError_t reap(bool wait)
    {
        while (!uses_.empty()) {
            hipError_t q = hipEventQuery(uses_.front().ev);
            if (q == hipErrorNotReady) {
                if (!wait)
                    return hipSuccess;
                wait = false;
                if ((q = hipEventSynchronize(uses_.front().ev)) != hipSuccess)
                    return q;
            } else if (q != hipSuccess) {
                return q;
            }
            pop_front();
        }
        return hipSuccess;
    }
    // Host pointer to len bytes; waits for older copies when the ring is full.
    hipError_t acquire(size_t len, char **p, void *owner)
    {
        hipError_t e;
        if (len > cap_) {
            // grow: drain every outstanding copy, then reallocate
            while (!uses_.empty())
                if ((e = reap(true)) != hipSuccess)
                    return e;
            (void)hipHostFree(base_);
            base_ = nullptr;
            cap_ = align_up(len) * 2;
            if ((e = hipHostMalloc((void **)&base_, cap_, hipHostMallocDefault)) != hipSuccess)
                return e;
            head_ = 0;
        }
        if ((e = reap(false)) != hipSuccess)
            return e;
        for (;;) {
            if (uses_.empty())
                head_ = 0;
            const size_t x = head_ + len <= cap_ ? head_ : 0;
            bool clash = false;
            for (const auto &u : uses_)
                if (x < u.off + u.len && u.off < x + len) {
                    clash = true;
                    break;
                }
            if (!clash) {
                pend_ = {x, len, nullptr, owner};
                head_ = align_up(x + len);
                *p = base_ + x;
                return hipSuccess;
            }
            if ((e = reap(true)) != hipSuccess)
                return e;
        }
    }
    // Record the event behind the copies of the last acquired range.
    hipError_t commit(hipStream_t st)
    {
        hipError_t e;
        if (!spare_.empty()) {
            pend_.ev = spare_.back();
            spare_.pop_back();
        } else if ((e = hipEventCreateWithFlags(&pend_.ev, hipEventDisableTiming)) != hipSuccess) {
            return e;
        }
        if ((e = hipEventRecord(pend_.ev, st)) != hipSuccess)
            return e;
        uses_.push_back(pend_);
        return hipSuccess;
    }

private:
    struct Use {
        size_t off, len;
        hipEvent_t ev;
        void *owner;
    };
    void pop_front()
    {
        Use u = uses_.front();
        uses_.pop_front();
        spare_.push_back(u.ev);
        if (u.owner && reclaim)
            reclaim(u.owner);
    }
    char *base_ = nullptr;
    size_t cap_ = 0, head_ = 0;
    Use pend_{};
    std::deque<Use> uses_;
    std::vector<hipEvent_t> spare_;
};

// Tile height of the batch: the kernels' choice for the storage form, or 4
// for every form when LBM_SERVED_TILE_Y = 4 (paired 64 x 4 launches; tuning
// and comparisons, read once per process)
int served_tile_ty(int storage)
{
    static const bool pair_only = [] {
        const char *e = getenv("LBM_SERVED_TILE_Y");
        return e && atoi(e) == 4;
    }();
    return pair_only ? 4 : lbmk::srv_tile_ty(storage);
}

enum { PH_QUEUED = 0, PH_FLUID = 1, PH_AD = 2, PH_RETIRING = 3, PH_DONE = 4 };

struct Job {
    uint64_t ticket = 0;
    lbm_request req{};
    std::vector<uint8_t> cls;
    std::vector<uint16_t> desc;
    lbmk::Geo geo{};
    int tiles = 0, tiles_wide = 0; // blocks of the batch launches over it: 64 x 4, 64 x 16 tiles
    int64_t n_fluid = 0, n_ad = 0;
    Layout lay{};
    double t_submit = 0, t_admit = 0, t_finish = 0;
    int status = LBM_OK; // preparation error, if any
    std::string msg;
    int sid = -1;
    size_t off = 0;
    int phase = PH_QUEUED;
    long long valid_from = 0; // first chunk whose snapshot shows the current phase
    long long t_max = 0;
    int st_fluid = LBM_OK, st_ad = LBM_OK;
    int64_t it_fluid = 0, it_ad = 0;
    double r_fluid = NAN, r_ad = NAN;
    bool ad_ran = false;
    char *staged = nullptr; // pinned result staging
    std::vector<float> u, c;
    double flux[10] = {0};
    bool preparing = false; // a preparation thread is working on it
    int lane = LBM_LANE_BATCH;
    int first_status = LBM_OK;
    int64_t first_it_fluid = 0, first_it_ad = 0;
};

int stop_status(int stop)
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

int overall_status(int a, int b)
{
    if (a == LBM_EDIVERGED || b == LBM_EDIVERGED)
        return LBM_EDIVERGED;
    if (a == LBM_NOT_CONVERGED || b == LBM_NOT_CONVERGED)
        return LBM_NOT_CONVERGED;
    if (a == LBM_STALLED || b == LBM_STALLED)
        return LBM_STALLED;
    return LBM_OK;
}

std::string request_problem(const lbm_request &r)
{
    if (r.nx < 3 || r.ny < 3)
        return "grid must be at least 3 x 3 (2-D requests)";
    if ((int64_t)r.nx * r.ny > ((int64_t)1 << 31) / 9)
        return "grid too large";
    if (!(r.tau > 0.5) || !isfinite(r.tau))
        return "tau must be > 1/2";
    if (!(fabs(r.u_in) < 0.1) || r.u_in == 0.0)
        return "u_in must be nonzero with |u_in| < 0.1";
    if (!(r.D > 0.0) || !isfinite(r.D))
        return "D must be > 0";
    if (!(r.c_in != 0.0) || !isfinite(r.c_in))
        return "c_in must be finite and nonzero";
    if (!(r.k_sink >= 0.0 && r.k_sink < 1.0))
        return "k_sink must be in [0, 1)";
    if (!(r.k_half >= 0.0) || !isfinite(r.k_half))
        return "k_half must be finite and >= 0";
    if (r.k_half > 0.0 && !(r.k_sink < r.k_half))
        return "the Monod sink needs k_sink < k_half";
    if (r.outlet != LBM_OUT_ZERO_GRADIENT && r.outlet != LBM_OUT_DIRICHLET)
        return "unknown outlet mode";
    if (!isfinite(r.c_out))
        return "c_out must be finite";
    if (!(r.tol >= 0.0) || r.max_iter < 1)
        return "tol must be >= 0 and max_iter >= 1";
    return std::string();
}

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

} // namespace

struct lbm_server {
    int device = 0;
    lbm_server_cfg cfg{};
    int K = 100, window = 0, depth = 2;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0;

    // device state
    char *pool = nullptr;
    lbmk::SrvSlot *d_slots = nullptr;
    lbmk::SrvTable *d_tab = nullptr;
    lbmk::Ctrl *d_ctrl = nullptr;
    unsigned long long *d_part = nullptr;
    int part_cap = 0;
    double *d_partials = nullptr;
    double *d_out = nullptr; // [SRV_MAX_SLOTS][10] flux results
    // one captured chunk per grid size: blocks = MIN_GRID << k, the smallest
    // one covering the table's tiles is launched (extra blocks exit at once)
    static const int MIN_GRID = 64;
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs[2]; // [0]: 64 x 4 tiles, [1]: 64 x 16
    int table_tiles = 0;
    // Tile form of each chunk: 64 x 16 tiles (four steps a launch) for the
    // FP32 forms while the batch holds at least wide_min such tiles and no
    // solo lane is solving; otherwise paired 64 x 4 launches.  On the
    // seeded stream at 50 req/s the batch alone served 1.41x faster with
    // the wide form, but beside busy solo lanes the wide form doubled the
    // batch requests' median latency for 4% more throughput, and with few
    // tiles the paired launches finish a chunk sooner.  Both forms run the
    // same per-node code on the same buffers and step counts, so a
    // request's results do not depend on the forms its chunks took.
    std::atomic<int> solo_active{0}; // solo lanes solving a request
    bool wide_ok = false;
    int wide_min = 256, wide_grid_max = 0;
    int table_ty = 4;

    // host state owned by the worker
    PoolAlloc alloc;
    PinnedRing up_ring, res_ring;
    lbmk::Ctrl *h_snap = nullptr; // pinned [RING][SRV_MAX_SLOTS]
    static const int RING = 8;
    hipEvent_t ev_snap[RING] = {};
    long long snap_chunk[RING] = {};
    std::atomic<long long> chunks{0}, chunks_wide{0}; // also read by lbm_server_stats
    long long head = 0, tail = 0;
    Job *slot_job[lbmk::SRV_MAX_SLOTS] = {};
    int tiles_used = 0, tiles_used_wide = 0;
    bool table_dirty = false;
    int n_retiring = 0;

    // shared state (mutex)
    std::mutex mu;
    std::condition_variable cv_prep, cv_work, cv_done;
    std::deque<Job *> prep_q;
    std::map<uint64_t, Job *> ready;     // prepared, by ticket
    std::deque<Job *> finished;          // not yet polled
    std::map<uint64_t, Job *> delivered; // polled, not yet released
    std::map<uint64_t, std::unique_ptr<Job>> all;
    uint64_t next_ticket = 1;
    int64_t n_submitted = 0, n_finished = 0, n_rejected = 0, n_active = 0;
    double updates = 0.0, busy = 0.0;
    bool stopping = false, failed = false;
    std::string err;
    char err_buf[256] = {0};
    std::vector<std::thread> preps;
    std::thread worker;

    // solo lanes (mutex for the queue and counters)
    std::vector<lbm_ctx *> solo_ctx;
    std::deque<Job *> solo_q;
    std::condition_variable cv_solo;
    std::vector<std::thread> solo;
    int64_t n_solo = 0, n_escalated = 0;
    std::vector<Job *> solo_cur; // the request each solo lane is solving
    int lanes_busy = 0;
    std::chrono::steady_clock::time_point lanes_since{};

    // ------------------------------------------------------------- prep
    void prep_loop()
    {
        for (;;) {
            Job *j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_prep.wait(lk, [&] { return stopping || !prep_q.empty(); });
                if (stopping)
                    return;
                j = prep_q.front();
                prep_q.pop_front();
                j->preparing = true;
            }
            {
                Range rg("lbm.srv.prepare");
                prepare(j);
            }
            std::lock_guard<std::mutex> lk(mu);
            j->preparing = false;
            if (stopping)
                continue; // abandoned: lbm_server_destroy frees it
            if (failed) {
                // fail() leaves the requests being prepared to their
                // threads: ending one there could hand it to the caller,
                // who may release it while it is still being prepared
                end_by_device_locked(j, err);
                cv_done.notify_all();
                continue;
            }
            if (j->status != LBM_OK) {
                finish_locked(j);
            } else if (j->lane == LBM_LANE_SOLO) {
                solo_q.push_back(j);
                cv_solo.notify_all();
            } else {
                ready[j->ticket] = j;
                cv_work.notify_all();
            }
        }
    }

    void prepare(Job *j)
    {
        const lbm_request &r = j->req;
        lbm_grid g{r.nx, r.ny, 1};
        const int64_t N = (int64_t)r.nx * r.ny;
        if (j->cls.empty()) {
            j->cls.assign((size_t)N, 0);
            double got = 0.0;
            lbm_status st = lbm_geom_discs(g, &r.discs, r.seed, j->cls.data(), &got);
            if (st != LBM_OK) {
                j->status = st;
                j->msg = "geometry generation failed";
                return;
            }
            if (r.layer)
                lbm_biofilm_layer(g, j->cls.data());
        }
        std::string m = check_mask(g, j->cls.data());
        std::vector<uint8_t> dom;
        if (m.empty()) {
            dom = flow_domain(g, j->cls.data());
            if (!domain_reaches_inlet(g, dom))
                m = "the fluid domain does not connect inlet to outlet";
        }
        if (!m.empty()) {
            j->status = LBM_EINVAL;
            j->msg = m;
            return;
        }
        j->geo = lbmk::make_geo(r.nx, r.ny, 1);
        if (j->lane == LBM_LANE_SOLO)
            return; // the single solver builds its own descriptors
        std::vector<uint32_t> d((size_t)N);
        build_desc(g, j->cls.data(), dom, reference_nodes(g, dom), d.data());
        j->desc.resize((size_t)N);
        const int aab = lbmk::desc_ad_active_bit(9, 5);
        for (int64_t n = 0; n < N; ++n) {
            j->desc[n] = (uint16_t)d[n];
            j->n_fluid += d[n] & 1u;
            j->n_ad += (d[n] >> aab) & 1u;
        }
        j->tiles = lbmk::pair_tiles(j->geo, 4);
        j->tiles_wide = wide_ok ? lbmk::pair_tiles(j->geo, 16) : j->tiles;
        if (!may_escalate()) {
            j->cls.clear();
            j->cls.shrink_to_fit();
        }
    }

    bool may_escalate() const
    {
        return cfg.escalate && (cfg.storage == LBM_FP16_SHIFTED || cfg.storage == LBM_FP32);
    }

    // caller holds mu
    void finish_locked(Job *j)
    {
        j->phase = PH_DONE;
        j->t_finish = now_s(t0);
        if (j->status == LBM_OK)
            updates += (double)j->it_fluid * j->n_fluid + (double)j->it_ad * j->n_ad;
        else
            ++n_rejected;
        if (j->lane != LBM_LANE_BATCH && j->status == LBM_OK) { // solved there
            ++n_solo;
            n_escalated += j->lane == LBM_LANE_ESCALATED;
        }
        ++n_finished;
        finished.push_back(j);
        cv_done.notify_all();
    }

    // ----------------------------------------------------------- worker
    // Device slot entry of request j in the given phase.
    lbmk::SrvSlot slot_entry(const Job *j, int phase) const
    {
        char *base = pool + j->off;
        const lbm_request &r = j->req;
        const double c_ref = lbmk::storage_shifted(cfg.storage) ? r.c_in : 0.0;
        lbmk::SrvSlot s{};
        s.desc = base + j->lay.desc;
        s.f[0] = base + j->lay.f0;
        s.f[1] = base + j->lay.f1;
        s.gp[0] = s.f[0]; // the substrate takes the place of the fluid
        s.gp[1] = s.f[1];
        s.u = base + j->lay.u;
        s.prev = base + j->lay.prev;
        s.ref_cur = reinterpret_cast<float *>(base + j->lay.ref);
        s.ref_next = s.ref_cur + r.nx;
        s.g = j->geo;
        s.omega_f = 1.0 / r.tau;
        s.u_in = r.u_in;
        s.inv_uin = 1.0 / ((double)K * fabs(r.u_in));
        s.omega_a = 1.0 / (0.5 + r.D / (1.0 / 3.0)); // as the single solve: D / c_s^2
        s.cin_s = r.c_in - c_ref;
        s.cout_s = r.c_out - c_ref;
        s.c_ref = c_ref;
        s.k_sink = r.k_sink;
        s.k_half = r.k_half;
        s.inv_cin = 1.0 / ((double)K * fabs(r.c_in));
        s.c_in = r.c_in;
        s.c_out = r.c_out;
        s.outlet = r.outlet;
        s.phase = phase;
        return s;
    }

    hipError_t admit(Job *j, int sid)
    {
        hipError_t e;
        const int64_t N = j->geo.N;
        const int storage = cfg.storage;
        char *base = pool + j->off;
        void *desc = base + j->lay.desc, *f0 = base + j->lay.f0;
        void *prev = base + j->lay.prev;
        char *stage;
        if ((e = up_ring.acquire((size_t)N * 2, &stage, nullptr)) != hipSuccess)
            return e;
        memcpy(stage, j->desc.data(), (size_t)N * 2);
        if ((e = hipMemcpyAsync(desc, stage, (size_t)N * 2, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return e;
        if ((e = up_ring.commit(stream)) != hipSuccess)
            return e;
        if ((e = hipMemsetAsync(d_out + 10 * sid, 0, 10 * sizeof(double), stream)) != hipSuccess)
            return e;
        float *ref = reinterpret_cast<float *>(base + j->lay.ref);
        if ((e = lbmk::ref_fill(ref, 2 * j->req.nx, 1.0f, stream)) != hipSuccess)
            return e;
        if ((e = lbmk::fluid_init(2, storage, f0, desc, j->geo, stream)) != hipSuccess)
            return e;
        if ((e = lbmk::fluid_export(2, storage, f0, desc, j->geo, ref, prev, nullptr, 0, stream)) !=
            hipSuccess)
            return e;
        j->t_max = (j->req.max_iter + K - 1) / K * (long long)K;
        if ((e = lbmk::ctrl_reset(d_ctrl + sid, j->req.tol, window, 1, K, nullptr, 0, stream, j->t_max)) !=
            hipSuccess)
            return e;
        const lbmk::SrvSlot s = slot_entry(j, lbmk::SRV_FLUID);
        if ((e = lbmk::srv_slot_set(d_slots, sid, s, stream)) != hipSuccess)
            return e;
        j->sid = sid;
        j->phase = PH_FLUID;
        j->valid_from = chunks;
        j->t_admit = now_s(t0);
        slot_job[sid] = j;
        tiles_used += j->tiles;
        tiles_used_wide += j->tiles_wide;
        table_dirty = true;
        return hipSuccess;
    }

    // Fluid solve of j has stopped: export its velocity and start the
    // substrate solve (or retire it when the fluid diverged).
    hipError_t to_substrate(Job *j)
    {
        hipError_t e;
        const int storage = cfg.storage;
        char *base = pool + j->off;
        void *desc = base + j->lay.desc, *f0 = base + j->lay.f0;
        void *u = base + j->lay.u, *prev = base + j->lay.prev;
        const lbm_request &r = j->req;
        const double c_ref = lbmk::storage_shifted(storage) ? r.c_in : 0.0;
        float *ref = reinterpret_cast<float *>(base + j->lay.ref);
        if ((e = lbmk::fluid_export(2, storage, f0, desc, j->geo, ref, u, nullptr, 0, stream)) != hipSuccess)
            return e;
        if ((e = lbmk::fluxes(2, storage, f0, nullptr, desc, j->geo, ref, nullptr, r.u_in, r.c_in, lbmk::Sink{r.k_sink, r.k_half},
                              r.outlet, r.c_out, nullptr, d_partials, d_out + 10 * j->sid, stream)) != hipSuccess)
            return e;
        if (j->st_fluid == LBM_EDIVERGED)
            return retire(j);
        // the substrate populations take the place of the fluid ones
        if ((e = lbmk::ref_fill(ref, 2 * r.nx, (float)c_ref, stream)) != hipSuccess)
            return e;
        if ((e = lbmk::ad_init(2, storage, f0, desc, u, j->geo, r.c_in, c_ref, stream)) != hipSuccess)
            return e;
        if ((e = lbmk::ad_export(2, storage, f0, desc, j->geo, ref, lbmk::Sink{r.k_sink, r.k_half}, prev, 0, stream)) !=
            hipSuccess)
            return e;
        if ((e = lbmk::ctrl_reset(d_ctrl + j->sid, r.tol, window, 0, K, nullptr, 0, stream, j->t_max)) !=
            hipSuccess)
            return e;
        const lbmk::SrvSlot s = slot_entry(j, lbmk::SRV_AD);
        if ((e = lbmk::srv_slot_set(d_slots, j->sid, s, stream)) != hipSuccess)
            return e;
        j->phase = PH_AD;
        j->ad_ran = true;
        j->valid_from = chunks;
        return hipSuccess;
    }

    // Export the concentration, copy the results to pinned memory and take
    // the request out of the table.
    hipError_t retire(Job *j)
    {
        hipError_t e;
        const int storage = cfg.storage;
        const int64_t N = j->geo.N;
        char *base = pool + j->off;
        void *desc = base + j->lay.desc, *f0 = base + j->lay.f0;
        void *u = base + j->lay.u, *prev = base + j->lay.prev;
        const lbm_request &r = j->req;
        float *ref = reinterpret_cast<float *>(base + j->lay.ref);
        double *out = d_out + 10 * j->sid;
        if (j->ad_ran) {
            if ((e = lbmk::ad_export(2, storage, f0, desc, j->geo, ref, lbmk::Sink{r.k_sink, r.k_half}, prev, 0, stream)) !=
                hipSuccess)
                return e;
            if ((e = lbmk::fluxes(2, storage, nullptr, f0, desc, j->geo, nullptr, ref, r.u_in, r.c_in,
                                  lbmk::Sink{r.k_sink, r.k_half}, r.outlet, r.c_out, nullptr, d_partials, out + 5, stream)) != hipSuccess)
                return e;
        } else if ((e = hipMemsetAsync(prev, 0, (size_t)N * 4, stream)) != hipSuccess) {
            return e;
        }
        const size_t bytes = 80 + (size_t)N * 12;
        if ((e = res_ring.acquire(bytes, &j->staged, j)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(j->staged, out, 80, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipMemcpyAsync(j->staged + 80, u, (size_t)N * 8, hipMemcpyDeviceToHost, stream)) !=
                hipSuccess ||
            (e = hipMemcpyAsync(j->staged + 80 + (size_t)N * 8, prev, (size_t)N * 4, hipMemcpyDeviceToHost,
                                stream)) != hipSuccess)
            return e;
        if ((e = res_ring.commit(stream)) != hipSuccess)
            return e;
        // Everything that touches the slot or the pool range is on this
        // stream: a request admitted into them now is ordered behind the
        // copies above, so both are free for reuse at once.
        j->phase = PH_RETIRING;
        slot_job[j->sid] = nullptr;
        tiles_used -= j->tiles;
        tiles_used_wide -= j->tiles_wide;
        {
            std::lock_guard<std::mutex> lk(mu);
            alloc.release(j->off, j->lay.total);
        }
        table_dirty = true;
        ++n_retiring;
        return hipSuccess;
    }

    // A retired request's copies are done (called by the result ring before
    // it reuses the staging range): hand out the result.
    void complete(Job *j)
    {
        const int64_t N = j->geo.N;
        memcpy(j->flux, j->staged, 80);
        j->u.resize((size_t)N * 2);
        j->c.resize((size_t)N);
        memcpy(j->u.data(), j->staged + 80, (size_t)N * 8);
        memcpy(j->c.data(), j->staged + 80 + (size_t)N * 8, (size_t)N * 4);
        j->staged = nullptr;
        j->desc.clear();
        j->desc.shrink_to_fit();
        --n_retiring;
        std::lock_guard<std::mutex> lk(mu);
        --n_active;
        const int st = overall_status(j->st_fluid, j->ad_ran ? j->st_ad : j->st_fluid);
        if (may_escalate() && st != LBM_OK && !stopping && !failed) {
            // the batched attempt's work counts; its fields are dropped
            updates += (double)j->it_fluid * j->n_fluid + (double)j->it_ad * j->n_ad;
            j->first_status = st;
            j->first_it_fluid = j->it_fluid;
            j->first_it_ad = j->it_ad;
            j->lane = LBM_LANE_ESCALATED;
            j->u.clear();
            j->c.clear();
            solo_q.push_back(j);
            cv_solo.notify_all();
            return;
        }
        j->cls.clear();
        j->cls.shrink_to_fit();
        finish_locked(j);
    }

    hipError_t write_table(int ty)
    {
        lbmk::SrvTable t{};
        int e = 0, tiles = 0;
        for (int s = 0; s < lbmk::SRV_MAX_SLOTS; ++s) {
            Job *j = slot_job[s];
            if (!j || (j->phase != PH_FLUID && j->phase != PH_AD))
                continue;
            t.begin[e] = tiles;
            t.slot[e] = s;
            tiles += ty == 16 ? j->tiles_wide : j->tiles;
            ++e;
        }
        t.begin[e] = tiles;
        t.n_active = e;
        t.total_tiles = tiles;
        // invariants the batched kernels rely on: tile offsets ascending
        // (their binary search), the table within the per-tile check slots
        for (int k = 0; k < e; ++k)
            if (t.begin[k] > t.begin[k + 1])
                return hipErrorInvalidValue;
        if (tiles > part_cap || tiles != (ty == 16 ? tiles_used_wide : tiles_used))
            return hipErrorInvalidValue;
        table_tiles = tiles;
        table_ty = ty;
        table_dirty = false;
        return lbmk::srv_table_set(d_tab, t, stream);
    }

    bool any_running() const
    {
        for (int s = 0; s < lbmk::SRV_MAX_SLOTS; ++s)
            if (slot_job[s] && (slot_job[s]->phase == PH_FLUID || slot_job[s]->phase == PH_AD))
                return true;
        return false;
    }

    hipError_t launch_chunk()
    {
        hipError_t e;
        const std::vector<hipGraphExec_t> &ex = execs[table_ty == 16 ? 1 : 0];
        if (!ex.empty()) {
            size_t k = 0;
            while ((MIN_GRID << k) < table_tiles && k + 1 < ex.size())
                ++k;
            if ((MIN_GRID << k) < table_tiles) // the grid must cover every tile of the table
                return hipErrorInvalidValue;
            if ((e = hipGraphLaunch(ex[k], stream)) != hipSuccess)
                return e;
        } else if ((e = enqueue_chunk(std::max(table_tiles, 1), table_ty == 16)) != hipSuccess) {
            return e;
        }
        const int r = (int)(head % RING);
        if ((e = hipMemcpyAsync(h_snap + (size_t)r * lbmk::SRV_MAX_SLOTS, d_ctrl,
                                sizeof(lbmk::Ctrl) * lbmk::SRV_MAX_SLOTS, hipMemcpyDeviceToHost, stream)) !=
            hipSuccess)
            return e;
        if ((e = hipEventRecord(ev_snap[r], stream)) != hipSuccess)
            return e;
        snap_chunk[r] = chunks++;
        chunks_wide += table_ty == 16;
        ++head;
        return hipSuccess;
    }

    hipError_t enqueue_chunk(int grid, bool wide)
    {
        hipError_t e;
        // Steps per launch: FP16 storage and FP32 storage with FP64
        // arithmetic two (64 x 4 tiles); FP32 and FP32-shifted storage four
        // (64 x 16 tiles), the first two launches taking two when K / 4 is
        // odd, so that a chunk has an even number of launches.  The check
        // is taken on the last launch.
        std::vector<int> plan;
        if (wide) {
            const int m = K / 4;
            plan.assign((size_t)(m & 1 ? 2 : 0), 2);
            plan.insert(plan.end(), (size_t)(m & 1 ? m - 1 : m), 4);
        } else {
            plan.assign((size_t)(K / 2), 2);
        }
        const int nl = (int)plan.size();
        int t_off = 0;
        for (int j = 0; j < nl; ++j) {
            const int mode = j == nl - 1 ? lbmk::MODE_CHECK : lbmk::MODE_PLAIN;
            e = wide ? lbmk::srv_stepN(cfg.storage, mode, plan[(size_t)j], d_slots, d_tab, d_ctrl, d_part,
                                       part_cap, j, t_off, grid, stream)
                     : lbmk::srv_step(cfg.storage, mode, d_slots, d_tab, d_ctrl, d_part, part_cap, j, grid,
                                      stream);
            if (e != hipSuccess)
                return e;
            if (j == 0 && lbmk::storage_moving_ref(cfg.storage) &&
                (e = lbmk::srv_ref_roll(d_slots, d_tab, d_ctrl, stream)) != hipSuccess)
                return e;
            t_off += plan[(size_t)j];
        }
        return lbmk::srv_decide(d_slots, d_tab, d_ctrl, d_part, part_cap, stream);
    }

    hipError_t process_snapshot()
    {
        const int r = (int)(tail % RING);
        const long long c = snap_chunk[r];
        const lbmk::Ctrl *snap = h_snap + (size_t)r * lbmk::SRV_MAX_SLOTS;
        ++tail;
        hipError_t e;
        for (int s = 0; s < lbmk::SRV_MAX_SLOTS; ++s) {
            Job *j = slot_job[s];
            if (!j || c < j->valid_from || snap[s].stop == lbmk::STOP_RUN)
                continue;
            const lbmk::Ctrl &k = snap[s];
            if (j->phase == PH_FLUID) {
                j->st_fluid = stop_status(k.stop);
                j->it_fluid = k.t_stop;
                j->r_fluid = k.checks > 0 ? k.r_last : NAN;
                if ((e = to_substrate(j)) != hipSuccess)
                    return e;
            } else if (j->phase == PH_AD) {
                j->st_ad = stop_status(k.stop);
                j->it_ad = k.t_stop;
                j->r_ad = k.checks > 0 ? k.r_last : NAN;
                if ((e = retire(j)) != hipSuccess)
                    return e;
            }
        }
        return hipSuccess;
    }

    // Admit prepared requests in ticket order while the head one fits.  The
    // head is chosen and taken out of `ready` under one lock: preparation
    // threads finish out of ticket order, so a lower ticket can enter
    // `ready` at any moment and become its head.  (Choosing the head in one
    // critical section and erasing `ready.begin()` in a later one dropped
    // that newcomer -- it was never admitted and the drain waited for it
    // forever -- and admitted the chosen request a second time.)
    hipError_t admit_ready()
    {
        for (;;) {
            Job *j = nullptr;
            int sid = -1;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (ready.empty())
                    return hipSuccess;
                auto first = ready.begin();
                j = first->second;
                for (int s = 0; s < cfg.max_slots; ++s)
                    if (!slot_job[s]) {
                        sid = s;
                        break;
                    }
                if (sid < 0 || tiles_used + j->tiles > part_cap) // 64 x 4: the most tiles
                    return hipSuccess;
                // the pool counters are read by lbm_server_stats
                if (!alloc.alloc(j->lay.total, &j->off))
                    return hipSuccess;
                ready.erase(first);
                ++n_active;
            }
            hipError_t e = admit(j, sid);
            if (e != hipSuccess)
                return e;
        }
    }

    hipError_t step_once(bool *idle)
    {
        hipError_t e;
        *idle = false;
        // finished result copies
        if ((e = res_ring.reap(false)) != hipSuccess)
            return e;
        if ((e = admit_ready()) != hipSuccess)
            return e;
        const int ty = wide_ok && solo_active.load() == 0 && tiles_used_wide >= wide_min &&
                               tiles_used_wide <= wide_grid_max
                           ? 16
                           : 4;
        if ((table_dirty || ty != table_ty) && (e = write_table(ty)) != hipSuccess)
            return e;
        const bool running = any_running();
        if (running && head - tail < depth) {
            const auto ta = std::chrono::steady_clock::now();
            if ((e = launch_chunk()) != hipSuccess)
                return e;
            busy_mark(ta);
            return hipSuccess;
        }
        if (head > tail) {
            const int r = (int)(tail % RING);
            hipError_t q = hipEventQuery(ev_snap[r]);
            if (q == hipErrorNotReady) {
                if (!(head - tail >= depth || !running))
                    return hipSuccess;
                if ((e = hipEventSynchronize(ev_snap[r])) != hipSuccess)
                    return e;
            } else if (q != hipSuccess) {
                return q;
            }
            return process_snapshot();
        }
        if (n_retiring > 0)
            return res_ring.reap(true);
        *idle = true;
        return hipSuccess;
    }

    // Busy time is the union of the lanes' busy intervals.
    bool was_busy = false;
    void lane_enter_locked(std::chrono::steady_clock::time_point t)
    {
        if (lanes_busy++ == 0)
            lanes_since = t;
    }
    void lane_leave_locked()
    {
        if (--lanes_busy == 0)
            busy += std::chrono::duration<double>(std::chrono::steady_clock::now() - lanes_since).count();
    }
    void busy_mark(std::chrono::steady_clock::time_point t)
    {
        if (!was_busy) {
            std::lock_guard<std::mutex> lk(mu);
            lane_enter_locked(t);
            was_busy = true;
        }
    }
    void busy_end()
    {
        if (was_busy) {
            std::lock_guard<std::mutex> lk(mu);
            lane_leave_locked();
            was_busy = false;
        }
    }

    // ------------------------------------------------------- solo lane
    void solo_loop(int lane)
    {
        for (;;) {
            Job *j;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_solo.wait(lk, [&] { return stopping || !solo_q.empty(); });
                if (stopping)
                    return;
                j = solo_q.front();
                solo_q.pop_front();
                solo_cur[lane] = j;
                lane_enter_locked(std::chrono::steady_clock::now());
                if (j->t_admit == 0)
                    j->t_admit = now_s(t0);
            }
            ++solo_active;
            {
                Range rg(j->lane == LBM_LANE_ESCALATED ? "lbm.srv.escalated" : "lbm.srv.solo");
                solve_alone(j, solo_ctx[lane]);
            }
            --solo_active;
            std::lock_guard<std::mutex> lk(mu);
            lane_leave_locked();
            solo_cur[lane] = nullptr;
            const int st = overall_status(j->st_fluid, j->ad_ran ? j->st_ad : j->st_fluid);
            if (j->lane == LBM_LANE_SOLO && j->status == LBM_OK && st != LBM_OK && may_escalate() &&
                !stopping && !failed) {
                // a reduced-storage solve on the solo lane: escalated as a
                // batched one would be
                updates += (double)j->it_fluid * j->n_fluid + (double)j->it_ad * j->n_ad;
                j->first_status = st;
                j->first_it_fluid = j->it_fluid;
                j->first_it_ad = j->it_ad;
                j->lane = LBM_LANE_ESCALATED;
                j->u.clear();
                j->c.clear();
                solo_q.push_back(j);
                cv_solo.notify_all();
                continue;
            }
            finish_locked(j);
        }
    }

    // The request's two solves by the single-domain solver: the server's
    // storage and cadence on the solo lane proper, FP32-shifted storage with
    // the default cadence and stall window when escalated.
    void solve_alone(Job *j, lbm_ctx *sctx)
    {
        const lbm_request &r = j->req;
        const bool esc = j->lane == LBM_LANE_ESCALATED;
        lbm_params p{};
        p.tau = r.tau;
        p.u_in = r.u_in;
        p.D = r.D;
        p.c_in = r.c_in;
        p.k_sink = r.k_sink;
        p.k_half = r.k_half;
        p.outlet = r.outlet;
        p.c_out = r.c_out;
        p.storage = esc ? LBM_FP32_SHIFTED : cfg.storage;
        p.check_every = esc ? 0 : K;
        p.stall_checks = esc ? 0 : cfg.stall_checks;
        const int64_t Ks = esc ? 100 : K;
        const int64_t max_iter = (r.max_iter + Ks - 1) / Ks * Ks;
        const lbm_grid g{r.nx, r.ny, 1};
        const int64_t N = (int64_t)r.nx * r.ny;
        j->st_fluid = j->st_ad = LBM_OK;
        j->it_fluid = j->it_ad = 0;
        j->r_fluid = j->r_ad = NAN;
        j->ad_ran = false;
        std::fill(j->flux, j->flux + 10, 0.0);
        lbm_solver *sv = nullptr;
        lbm_status st = lbm_solver_create(sctx, g, j->cls.data(), &p, &sv);
        if (esc || !may_escalate()) {
            j->cls.clear(); // no later solve of this request needs the mask
            j->cls.shrink_to_fit();
        }
        auto fail_job = [&](lbm_status e) {
            j->status = e;
            j->msg = lbm_last_error(sctx);
            if (sv)
                lbm_solver_destroy(sv);
        };
        if (st != LBM_OK)
            return fail_job(st);
        auto solve_status = [](lbm_status e) {
            return e == LBM_OK || e == LBM_STALLED || e == LBM_NOT_CONVERGED || e == LBM_EDIVERGED;
        };
        lbm_info fi{}, ai{};
        st = lbm_solver_fluid(sv, r.tol, max_iter, 0, &fi);
        if (!solve_status(st))
            return fail_job(st);
        j->st_fluid = st;
        j->it_fluid = fi.iters;
        j->r_fluid = fi.checks > 0 ? fi.residual : NAN;
        j->n_fluid = fi.active_nodes;
        // the FP32 exports, as the batch returns them
        std::vector<double> out5(5, 0.0);
        j->u.assign((size_t)N * 2, 0.0f);
        j->c.assign((size_t)N, 0.0f);
        lbm_status e;
        if ((e = export_f32(sv, 0, j->u.data())) != LBM_OK || (e = lbm_solver_fluxes(sv, out5.data())) != LBM_OK)
            return fail_job(e);
        j->flux[0] = out5[0];
        j->flux[1] = out5[1];
        if (st != LBM_EDIVERGED) {
            st = lbm_solver_ad(sv, r.tol, max_iter, 0, &ai);
            if (!solve_status(st))
                return fail_job(st);
            j->st_ad = st;
            j->it_ad = ai.iters;
            j->r_ad = ai.checks > 0 ? ai.residual : NAN;
            j->n_ad = ai.active_nodes;
            j->ad_ran = true;
            if ((e = export_f32(sv, 1, j->c.data())) != LBM_OK || (e = lbm_solver_fluxes(sv, out5.data())) != LBM_OK)
                return fail_job(e);
            j->flux[7] = out5[2];
            j->flux[8] = out5[3];
            j->flux[9] = out5[4];
        }
        lbm_solver_destroy(sv);
    }

    void work_loop()
    {
        hipError_t e = hipSetDevice(device);
        while (e == hipSuccess) {
            bool idle = false;
            {
                Range rg("lbm.srv.step");
                e = step_once(&idle);
            }
            if (e != hipSuccess)
                break;
            if (idle) {
                busy_end();
                std::unique_lock<std::mutex> lk(mu);
                if (stopping)
                    return;
                cv_work.wait_for(lk, std::chrono::milliseconds(20),
                                 [&] { return stopping || !ready.empty(); });
                if (stopping)
                    return;
            } else {
                std::lock_guard<std::mutex> lk(mu);
                if (stopping)
                    break;
            }
        }
        if (e != hipSuccess)
            fail(std::string("HIP error in the serving loop: ") + hipGetErrorString(e));
    }

    // caller holds mu
    void end_by_device_locked(Job *j, const std::string &m)
    {
        j->status = LBM_EDEVICE;
        j->msg = m;
        j->phase = PH_DONE;
        j->t_finish = now_s(t0);
        ++n_finished;
        finished.push_back(j);
    }

    // Device failure: every request not yet finished ends with EDEVICE.
    // Those a solo lane or a preparation thread is working on are ended by
    // that thread when it is done with them.
    void fail(const std::string &m)
    {
        std::lock_guard<std::mutex> lk(mu);
        failed = true;
        err = m;
        for (auto &kv : all) {
            Job *j = kv.second.get();
            if (j->phase == PH_DONE || j->preparing ||
                std::find(solo_cur.begin(), solo_cur.end(), j) != solo_cur.end())
                continue;
            end_by_device_locked(j, m);
        }
        prep_q.clear();
        ready.clear();
        solo_q.clear();
        cv_done.notify_all();
    }

    void fill_result(Job *j, lbm_result *o)
    {
        memset(o, 0, sizeof(*o));
        o->ticket = j->ticket;
        o->user = j->req.user;
        o->nx = j->req.nx;
        o->ny = j->req.ny;
        if (j->status != LBM_OK) {
            o->status = j->status;
            snprintf(o->message, sizeof(o->message), "%s", j->msg.c_str());
        } else {
            o->status_fluid = j->st_fluid;
            o->status_ad = j->ad_ran ? j->st_ad : j->st_fluid;
            o->status = overall_status(j->st_fluid, o->status_ad);
        }
        o->iters_fluid = j->it_fluid;
        o->iters_ad = j->it_ad;
        o->residual_fluid = j->r_fluid;
        o->residual_ad = j->r_ad;
        o->flux[0] = j->flux[0];
        o->flux[1] = j->flux[1];
        o->flux[2] = j->flux[7];
        o->flux[3] = j->flux[8];
        o->flux[4] = j->flux[9];
        o->active_fluid = j->n_fluid;
        o->active_ad = j->n_ad;
        o->t_submit = j->t_submit;
        o->t_admit = j->t_admit;
        o->t_finish = j->t_finish;
        o->u = j->u.empty() ? nullptr : j->u.data();
        o->c = j->c.empty() ? nullptr : j->c.data();
        o->lane = j->lane;
        o->first_status = j->first_status;
        o->first_iters_fluid = j->first_it_fluid;
        o->first_iters_ad = j->first_it_ad;
    }
};

extern "C" {

size_t lbm_server_footprint(int32_t nx, int32_t ny, int32_t storage)
{
    if (nx < 1 || ny < 1 || storage < LBM_FP32 || storage == LBM_FP64 || storage > LBM_FP32_SHIFTED_F64)
        return 0;
    return layout_of(nx, (int64_t)nx * ny, storage).total;
}

lbm_status lbm_server_create(lbm_ctx *ctx, const lbm_server_cfg *cfg, lbm_server **out)
{
    if (!ctx || !cfg || !out)
        return set_err(ctx, LBM_EINVAL, "null argument");
    *out = nullptr;
    lbm_server_cfg c = *cfg;
    if (c.storage < LBM_FP32 || c.storage == LBM_FP64 || c.storage > LBM_FP32_SHIFTED_F64)
        return set_err(ctx, LBM_EINVAL,
                       "server storage must be FP32, FP32_SHIFTED, FP16_SHIFTED or FP32_SHIFTED_F64");
    if (c.max_slots == 0)
        c.max_slots = 32;
    if (c.max_slots < 1 || c.max_slots > lbmk::SRV_MAX_SLOTS)
        return set_err(ctx, LBM_EINVAL, "max_slots must be in 1..64");
    if (c.check_every == 0)
        c.check_every = c.storage == LBM_FP16_SHIFTED ? 1000 : 100; // as lbm_params
    if (c.check_every < 4 || (c.check_every % 4) || c.check_every > 1000)
        return set_err(ctx, LBM_EINVAL, "check_every must be a multiple of 4 in 4..1000");
    if (c.inflight == 0)
        c.inflight = 2;
    if (c.inflight < 1 || c.inflight > 6)
        return set_err(ctx, LBM_EINVAL, "inflight must be in 1..6");
    if (c.prep_threads == 0)
        c.prep_threads = 2;
    if (c.prep_threads < 1 || c.prep_threads > 16)
        return set_err(ctx, LBM_EINVAL, "prep_threads must be in 1..16");
    if (c.pool_bytes < (size_t)1 << 16)
        return set_err(ctx, LBM_EINVAL, "pool_bytes must be at least 64 KiB");
    if (c.escalate != 0 && c.escalate != 1)
        return set_err(ctx, LBM_EINVAL, "escalate must be 0 or 1");
    if (c.solo_nodes == 0)
        c.solo_nodes = (int64_t)1 << 18;
    if (c.solo_lanes == 0)
        c.solo_lanes = 2;
    if (c.solo_lanes < 1 || c.solo_lanes > 8)
        return set_err(ctx, LBM_EINVAL, "solo_lanes must be in 1..8");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return hip_err(ctx, e, "set device");
    std::unique_ptr<lbm_server> s(new lbm_server());
    s->device = ctx->device;
    s->cfg = c;
    s->K = c.check_every;
    s->window = c.stall_checks < 0 ? 0 : (c.stall_checks > 0 ? c.stall_checks : default_stall_checks(c.storage, s->K));
    s->depth = c.inflight;
    s->t0 = std::chrono::steady_clock::now();
    // tiles: each 64 x 4 tile holds 256 nodes (one per thread of a block)
    // of at least 54 pool bytes; ragged tiles at the domain edges add at
    // most ntx + nty per request.  The largest captured grid (the power of
    // two at or above part_cap) times the block size stays within 2^31
    // threads; 64 x 16 tiles (1024 threads) are a quarter as many, plus the
    // ragged ones, and their form is taken only while the table fits the
    // largest wide grid.
    const size_t pc = c.pool_bytes / ((size_t)256 * 54) + (size_t)c.max_slots * 1024 + 1024;
    s->part_cap = (int)std::min<size_t>(pc, ((size_t)1 << 31) / 256);
    s->wide_ok = served_tile_ty(c.storage) == 16;
    if (const char *ev = getenv("LBM_SERVED_WIDE_MIN_TILES")) // tuning and tests
        if (atoi(ev) > 0)
            s->wide_min = atoi(ev);
    s->wide_grid_max = 1 << 21; // direct launches: 2^31 threads of 1024
    auto cleanup = [&](lbm_status st) {
        lbm_server_destroy(s.release());
        return st;
    };
    auto dmalloc = [&](void **p, size_t bytes) -> hipError_t {
        hipError_t r = hipMalloc(p, bytes);
        if (r != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
        }
        return r;
    };
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess)
        return cleanup(hip_err(ctx, e, "server stream"));
    for (int k = 0; k < c.solo_lanes; ++k) {
        lbm_ctx *sc = nullptr;
        if (lbm_ctx_create(ctx->device, nullptr, &sc) != LBM_OK)
            return cleanup(set_err(ctx, LBM_EDEVICE, "solo lane context"));
        s->solo_ctx.push_back(sc);
    }
    s->solo_cur.assign((size_t)c.solo_lanes, nullptr);
    if (dmalloc((void **)&s->pool, c.pool_bytes) != hipSuccess)
        return cleanup(set_err(ctx, LBM_ENOMEM, "device pool allocation failed"));
    if (dmalloc((void **)&s->d_slots, sizeof(lbmk::SrvSlot) * lbmk::SRV_MAX_SLOTS) != hipSuccess ||
        dmalloc((void **)&s->d_tab, sizeof(lbmk::SrvTable)) != hipSuccess ||
        dmalloc((void **)&s->d_ctrl, sizeof(lbmk::Ctrl) * lbmk::SRV_MAX_SLOTS) != hipSuccess ||
        dmalloc((void **)&s->d_part, sizeof(unsigned long long) * 2 * (size_t)s->part_cap) != hipSuccess ||
        dmalloc((void **)&s->d_partials, sizeof(double) * 5 * lbmk::FLUX_BLOCKS) != hipSuccess ||
        dmalloc((void **)&s->d_out, sizeof(double) * 10 * lbmk::SRV_MAX_SLOTS) != hipSuccess)
        return cleanup(set_err(ctx, LBM_ENOMEM, "server device allocation failed"));
    if ((e = hipMemsetAsync(s->d_slots, 0, sizeof(lbmk::SrvSlot) * lbmk::SRV_MAX_SLOTS, s->stream)) !=
            hipSuccess ||
        (e = hipMemsetAsync(s->d_tab, 0, sizeof(lbmk::SrvTable), s->stream)) != hipSuccess ||
        (e = hipMemsetAsync(s->d_ctrl, 0, sizeof(lbmk::Ctrl) * lbmk::SRV_MAX_SLOTS, s->stream)) !=
            hipSuccess ||
        (e = hipMemsetAsync(s->d_out, 0, sizeof(double) * 10 * lbmk::SRV_MAX_SLOTS, s->stream)) != hipSuccess)
        return cleanup(hip_err(ctx, e, "server init"));
    s->alloc.reset(c.pool_bytes);
    if ((e = s->up_ring.init((size_t)32 << 20)) != hipSuccess ||
        (e = s->res_ring.init((size_t)64 << 20)) != hipSuccess)
        return cleanup(hip_err(ctx, e, "pinned staging"));
    if ((e = hipHostMalloc((void **)&s->h_snap, sizeof(lbmk::Ctrl) * lbmk::SRV_MAX_SLOTS * lbm_server::RING,
                           hipHostMallocDefault)) != hipSuccess) {
        s->h_snap = nullptr;
        return cleanup(hip_err(ctx, e, "pinned snapshots"));
    }
    for (int k = 0; k < lbm_server::RING; ++k)
        if ((e = hipEventCreateWithFlags(&s->ev_snap[k], hipEventDisableTiming)) != hipSuccess)
            return cleanup(hip_err(ctx, e, "event"));
    if (!c.direct_launch) {
        // the chunk, captured once per grid size: it reads the slot table at
        // run time, so admissions and retirements never re-capture
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess)
            return cleanup(hip_err(ctx, e, "server init"));
        for (int f = 0; f < (s->wide_ok ? 2 : 1); ++f) {
            const int64_t grid_cap = f ? ((int64_t)1 << 21) : ((int64_t)1 << 23);
            for (int64_t grid = lbm_server::MIN_GRID;; grid *= 2) {
                hipGraph_t g = nullptr;
                hipGraphExec_t x = nullptr;
                if ((e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                    return cleanup(hip_err(ctx, e, "graph capture"));
                hipError_t le = s->enqueue_chunk((int)grid, f == 1);
                e = hipStreamEndCapture(s->stream, &g);
                if (g)
                    s->graphs.push_back(g);
                if (le != hipSuccess || e != hipSuccess)
                    return cleanup(hip_err(ctx, le != hipSuccess ? le : e, "graph capture"));
                if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess)
                    return cleanup(hip_err(ctx, e, "graph instantiate"));
                s->execs[f].push_back(x);
                if (f)
                    s->wide_grid_max = (int)grid;
                if (grid >= s->part_cap || grid >= grid_cap)
                    break;
            }
        }
    }
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess)
        return cleanup(hip_err(ctx, e, "server init"));
    lbm_server *sp = s.get();
    s->res_ring.reclaim = [sp](void *o) { sp->complete(static_cast<Job *>(o)); };
    for (int k = 0; k < c.prep_threads; ++k)
        s->preps.emplace_back([sp] { sp->prep_loop(); });
    s->worker = std::thread([sp] { sp->work_loop(); });
    for (int k = 0; k < c.solo_lanes; ++k)
        s->solo.emplace_back([sp, k] { sp->solo_loop(k); });
    *out = s.release();
    return LBM_OK;
}

lbm_status lbm_server_submit(lbm_server *s, const lbm_request *r, uint64_t *ticket)
{
    if (!s || !r)
        return LBM_EINVAL;
    std::unique_ptr<Job> j(new Job());
    j->req = *r;
    j->req.cls = nullptr;
    const int64_t N = (int64_t)r->nx * r->ny;
    std::string m = request_problem(*r);
    if (m.empty()) {
        j->lay = layout_of(r->nx, N, s->cfg.storage);
        if (s->cfg.solo_nodes > 0 && N >= s->cfg.solo_nodes) // < 0: no solo lane
            j->lane = LBM_LANE_SOLO;
        else if (j->lay.total > s->cfg.pool_bytes ||
                 lbmk::pair_tiles(lbmk::make_geo(r->nx, r->ny, 1), 4) > s->part_cap)
            m = "request larger than the server pool";
        if (m.empty() && r->cls)
            j->cls.assign(r->cls, r->cls + N);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) {
        snprintf(s->err_buf, sizeof(s->err_buf), "%s", s->err.c_str());
        return LBM_EDEVICE;
    }
    if (s->stopping)
        return LBM_EBUSY;
    if (!m.empty()) {
        snprintf(s->err_buf, sizeof(s->err_buf), "%s", m.c_str());
        return LBM_EINVAL;
    }
    j->ticket = s->next_ticket++;
    j->t_submit = now_s(s->t0);
    if (ticket)
        *ticket = j->ticket;
    Job *jp = j.get();
    s->all[jp->ticket] = std::move(j);
    ++s->n_submitted;
    s->prep_q.push_back(jp);
    s->cv_prep.notify_one();
    return LBM_OK;
}

lbm_status lbm_server_poll(lbm_server *s, lbm_result *out, int max, int *n_out, double wait_s)
{
    if (!s || (!out && max > 0) || !n_out)
        return LBM_EINVAL;
    *n_out = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->finished.empty() && wait_s > 0)
        s->cv_done.wait_for(lk, std::chrono::duration<double>(wait_s), [&] { return !s->finished.empty(); });
    int n = 0;
    while (n < max && !s->finished.empty()) {
        Job *j = s->finished.front();
        s->finished.pop_front();
        s->delivered[j->ticket] = j;
        s->fill_result(j, out + n);
        ++n;
    }
    *n_out = n;
    return LBM_OK;
}

void lbm_result_release(lbm_server *s, lbm_result *r)
{
    if (!s || !r)
        return;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->delivered.find(r->ticket);
    if (it == s->delivered.end())
        return;
    s->delivered.erase(it);
    s->all.erase(r->ticket);
    r->u = nullptr;
    r->c = nullptr;
}

lbm_status lbm_server_drain(lbm_server *s, double timeout_s)
{
    if (!s)
        return LBM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto done = [&] { return s->n_finished == s->n_submitted; };
    if (timeout_s > 0) {
        if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
            return LBM_EBUSY;
    } else {
        s->cv_done.wait(lk, done);
    }
    return s->failed ? LBM_EDEVICE : LBM_OK;
}

lbm_status lbm_server_stats(lbm_server *s, lbm_server_stats_t *o)
{
    if (!s || !o)
        return LBM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(o, 0, sizeof(*o));
    o->submitted = s->n_submitted;
    o->finished = s->n_finished;
    o->rejected = s->n_rejected;
    o->active = s->n_active;
    o->queued = (int64_t)(s->prep_q.size() + s->ready.size() + s->solo_q.size());
    o->chunks = s->chunks;
    o->pool_bytes = s->cfg.pool_bytes;
    o->pool_used = s->alloc.used;
    o->pool_peak = s->alloc.peak;
    o->lattice_updates = s->updates;
    o->busy_seconds = s->busy;
    if (s->lanes_busy > 0)
        o->busy_seconds +=
            std::chrono::duration<double>(std::chrono::steady_clock::now() - s->lanes_since).count();
    o->clock = now_s(s->t0);
    o->solo = s->n_solo;
    o->escalated = s->n_escalated;
    o->chunks_wide = s->chunks_wide;
    return LBM_OK;
}

const char *lbm_server_error(lbm_server *s)
{
    if (!s)
        return "";
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed)
        snprintf(s->err_buf, sizeof(s->err_buf), "%s", s->err.c_str());
    return s->err_buf;
}

void lbm_server_destroy(lbm_server *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_prep.notify_all();
    s->cv_work.notify_all();
    s->cv_solo.notify_all();
    for (auto &t : s->preps)
        if (t.joinable())
            t.join();
    if (s->worker.joinable())
        s->worker.join();
    for (auto &t : s->solo)
        if (t.joinable())
            t.join();
    for (lbm_ctx *sc : s->solo_ctx)
        lbm_ctx_destroy(sc);
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    s->res_ring.reclaim = nullptr;
    s->up_ring.destroy();
    s->res_ring.destroy();
    for (auto &ex : s->execs)
        for (hipGraphExec_t x : ex)
            (void)hipGraphExecDestroy(x);
    for (hipGraph_t g : s->graphs)
        (void)hipGraphDestroy(g);
    for (int k = 0; k < lbm_server::RING; ++k)
        if (s->ev_snap[k])
            (void)hipEventDestroy(s->ev_snap[k]);
    if (s->h_snap)
        (void)hipHostFree(s->h_snap);
    void *bufs[] = {s->pool, s->d_slots, s->d_tab, s->d_ctrl, s->d_part, s->d_partials, s->d_out};
    for (void *p : bufs)
        if (p)
            (void)hipFree(p);
    if (s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
}

} // extern "C"

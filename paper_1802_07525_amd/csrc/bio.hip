// bio.hip -- the bio-electrochemical model of Sec. 2.2 (Eqs. 14-21), once
// per model interval, on the substrate field the solver holds in HBM.
//
// One interval is a scalar root solve over all biomass cells: the cell
// current I (Eq. 20, with the overpotentials of Eqs. 18-19) depends on the
// biomass-weighted mean mediator, and every cell's mediator (Eq. 15 with
// the double-Monod rate of Eq. 16 taken at the new state) depends on I
// through the oxidation gamma I dt / (m F B) shared by all biomass.  For a
// trial I each cell's new M_ox is the positive root of a quadratic; the
// mean decides which half of the bracket keeps the root.  The bisection is
// sequential, so the whole interval runs in one work-group: each pass over
// the cells is a strided loop plus an LDS tree sum (fixed order, so the
// result does not depend on timing), and the decision is taken by every
// thread on the same reduced value.  No host round trip between halvings.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbmh;

namespace {

constexpr int BIO_THREADS = 1024;
constexpr int ROOT_ITERS = 80;
constexpr double R_GAS = 8.314462618;    // J / (mol K)
constexpr double FARADAY = 96485.33212;  // C / mol

struct BioK {
    double q_max, K_s, M_total, K_Mox, E0, R_ext, R_int, eps, c_scale;
    double red_dt;        // Y q_max dt_day: the interval's reduction at full rate
    double beta_per_amp;  // gamma dt_s / (m F B): oxidation per unit biomass per ampere
    double act_per_amp;   // R T / (m F A_a I0): n_act = act_per_amp * I * M_ox / M_red
    double phi;           // R T / F
    double sum_cb, biomass, q_scale;  // q_scale = cell volume / 24 (mg/day -> mg/h)
};

// Eq. 15 for one cell over the interval at trial oxidation beta: the root
// M >= 0 of M^2 + (K + a - p) M - p K = 0, p = M0 + beta, in the form that
// avoids cancellation, capped at M_total (Eq. 14).
__device__ __forceinline__ double cell_mediator(double m0, double a, double beta, const BioK &k)
{
    const double p = m0 + beta, K = k.K_Mox;
    const double b = K + a - p;
    const double disc = sqrt(b * b + 4.0 * p * K);
    const double M = b >= 0.0 ? 2.0 * p * K / (b + disc) : 0.5 * (disc - b);
    return fmin(M, k.M_total);
}

// Eqs. 18-20 at mean M_ox and trial current I, floored at 0
__device__ __forceinline__ double current_eq20(double I, double mbar, const BioK &k)
{
    const double mred = k.M_total - mbar;
    if (!(mred > 0.0))
        return 0.0;
    const double n_conc = k.phi * log(k.M_total / mred);
    const double n_act = k.act_per_amp * I * (mbar / mred);
    const double v = (k.E0 - n_conc - n_act) / (k.R_int + k.R_ext) * (mred / (k.eps + mred));
    return fmax(v, 0.0);
}

// block-wide sum in a fixed tree order; every thread gets the total
__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = BIO_THREADS / 2; s > 0; s >>= 1) {
        if (t < s)
            red[t] += red[t + s];
        __syncthreads();
    }
    const double total = red[0];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(BIO_THREADS) void k_bio_interval(int ncell, const int32_t *__restrict__ idx,
                                                              const double *__restrict__ cb,
                                                              double *__restrict__ mox,
                                                              double *__restrict__ fs,
                                                              const double *__restrict__ C, BioK k,
                                                              lbm_bio_out *__restrict__ out)
{
    __shared__ double red[BIO_THREADS];
    const int t = threadIdx.x;
    // substrate factor of Eq. 16 per cell; the negative tail of the
    // lattice field is not consumed.  Cell j stays with thread j % 1024 in
    // every pass below, so no barrier is needed between them.
    for (int j = t; j < ncell; j += BIO_THREADS) {
        const double S = k.c_scale * fmax(C[idx[j]], 0.0);
        fs[j] = S / (S + k.K_s);
    }
    double lo = 0.0, hi = k.E0 / (k.R_int + k.R_ext);
    int iters = 0;
    for (int it = 0; it < ROOT_ITERS; ++it) {
        const double mid = lo + (hi - lo) * 0.5;
        if (!(lo < mid && mid < hi))
            break;
        ++iters;
        const double beta = k.beta_per_amp * mid;
        double part = 0.0;
        for (int j = t; j < ncell; j += BIO_THREADS)
            part += cb[j] * cell_mediator(mox[j], k.red_dt * fs[j], beta, k);
        const double mbar = block_sum(part, red) / k.sum_cb;
        if (mid - current_eq20(mid, mbar, k) > 0.0)
            hi = mid;
        else
            lo = mid;
    }
    // the new state at the root
    const double I = lo, beta = k.beta_per_amp * I;
    double pm = 0.0, pq = 0.0;
    for (int j = t; j < ncell; j += BIO_THREADS) {
        const double M = cell_mediator(mox[j], k.red_dt * fs[j], beta, k);
        mox[j] = M;
        pm += cb[j] * M;
        pq += cb[j] * (k.q_max * fs[j] * (M / (M + k.K_Mox)));
    }
    const double mbar = block_sum(pm, red) / k.sum_cb;
    const double qsum = block_sum(pq, red);
    if (t == 0) {
        const double mred = k.M_total - mbar;
        lbm_bio_out o;
        o.I_cell = I;
        o.V_cell = I * k.R_ext;
        o.V_total = I * (k.R_int + k.R_ext);
        o.n_conc = mred > 0.0 ? k.phi * log(k.M_total / mred) : INFINITY;
        o.n_act = mred > 0.0 ? k.act_per_amp * I * (mbar / mred) : INFINITY;
        o.M_ox = mbar;
        o.M_red = mred;
        o.biomass = k.biomass;
        o.q_total = qsum * k.q_scale;
        o.n_cells = ncell;
        o.root_iters = iters;
        *out = o;
    }
}

#define BIOCHK(expr, where)                                                                      \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return hip_err(b->s->ctx, e_, where);                                                \
    } while (0)

std::string check_params(const lbm_bio_params &p)
{
    const double v[] = {p.q_max, p.K_s, p.M_total, p.K_Mox, p.Y, p.gamma, p.m, p.I0, p.E0, p.R_ext,
                        p.R_int, p.A_a, p.V_a, p.T, p.eps, p.C0_bio, p.c_scale, p.dt_hours};
    for (double x : v)
        if (!isfinite(x))
            return "bio parameters must be finite";
    if (p.q_max < 0.0 || p.Y < 0.0 || p.eps < 0.0 || p.R_ext < 0.0 || p.R_int < 0.0)
        return "q_max, Y, eps, R_ext and R_int must be >= 0";
    if (!(p.K_s > 0.0 && p.M_total > 0.0 && p.K_Mox > 0.0 && p.gamma > 0.0 && p.m > 0.0 && p.I0 > 0.0 &&
          p.E0 > 0.0 && p.R_ext + p.R_int > 0.0 && p.A_a > 0.0 && p.V_a > 0.0 && p.T > 0.0 &&
          p.C0_bio > 0.0 && p.c_scale > 0.0 && p.dt_hours > 0.0))
        return "K_s, M_total, K_Mox, gamma, m, I0, E0, R_ext + R_int, A_a, V_a, T, C0_bio, c_scale "
               "and dt_hours must be > 0";
    return "";
}

// one node's biomass and mediator against the rules of lbm_bio_create
std::string check_node(const lbm_bio *b, int64_t n, double c, double m)
{
    if (!(c >= 0.0) || !isfinite(c))
        return "c_bio must be finite and >= 0";
    if (c > 0.0 && b->s->cls[(size_t)n] != LBM_BIOFILM)
        return "node " + std::to_string(n) + " holds biomass but is not BIOFILM";
    if (c > 0.0 && !(m >= 0.0 && m <= b->p.M_total))
        return "m_ox must lie in [0, M_total] where c_bio > 0";
    return "";
}

void free_dev(lbm_bio *b)
{
    (void)hipFree(b->d_idx);
    (void)hipFree(b->d_cb);
    (void)hipFree(b->d_mox);
    (void)hipFree(b->d_fs);
    b->d_idx = nullptr;
    b->d_cb = b->d_mox = b->d_fs = nullptr;
    b->cap = 0;
}

} // namespace

// device M_ox -> host mirror
lbm_status lbmh::bio_pull_mox(lbm_bio *b)
{
    if (!b->mox_stale)
        return LBM_OK;
    const size_t nc = b->cells.size();
    std::vector<double> m(nc);
    if (nc) {
        BIOCHK(hipMemcpyAsync(m.data(), b->d_mox, nc * 8, hipMemcpyDeviceToHost, b->s->ctx->stream),
               "bio copy");
        BIOCHK(hipStreamSynchronize(b->s->ctx->stream), "bio sync");
    }
    for (size_t j = 0; j < nc; ++j)
        b->mox[(size_t)b->cells[j]] = m[j];
    b->mox_stale = false;
    return LBM_OK;
}

// host fields -> compact cell list, totals and device arrays
lbm_status lbmh::bio_push_cells(lbm_bio *b)
{
    const size_t N = b->cb.size();
    b->cells.clear();
    for (size_t n = 0; n < N; ++n)
        if (b->cb[n] > 0.0)
            b->cells.push_back((int32_t)n);
    const size_t nc = b->cells.size();
    std::vector<double> c(nc), m(nc);
    double sum = 0.0;
    for (size_t j = 0; j < nc; ++j) {  // ascending node order
        c[j] = b->cb[(size_t)b->cells[j]];
        m[j] = b->mox[(size_t)b->cells[j]];
        sum += c[j];
    }
    b->sum_cb = sum;
    b->biomass = sum * (b->p.V_a / (double)N);
    if (nc > b->cap) {
        free_dev(b);
        const size_t cap = std::max(nc, (size_t)1024);
        hipError_t e = hipMalloc((void **)&b->d_idx, cap * 4);
        if (e == hipSuccess)
            e = hipMalloc((void **)&b->d_cb, cap * 8);
        if (e == hipSuccess)
            e = hipMalloc((void **)&b->d_mox, cap * 8);
        if (e == hipSuccess)
            e = hipMalloc((void **)&b->d_fs, cap * 8);
        if (e != hipSuccess) {
            free_dev(b);
            return set_err(b->s->ctx, LBM_ENOMEM, "bio cell arrays");
        }
        b->cap = cap;
    }
    if (nc) {
        hipStream_t st = b->s->ctx->stream;
        BIOCHK(hipMemcpyAsync(b->d_idx, b->cells.data(), nc * 4, hipMemcpyHostToDevice, st), "bio upload");
        BIOCHK(hipMemcpyAsync(b->d_cb, c.data(), nc * 8, hipMemcpyHostToDevice, st), "bio upload");
        BIOCHK(hipMemcpyAsync(b->d_mox, m.data(), nc * 8, hipMemcpyHostToDevice, st), "bio upload");
        BIOCHK(hipStreamSynchronize(st), "bio sync");  // the host vectors go out of scope
    }
    return LBM_OK;
}

extern "C" {

void lbm_bio_destroy(lbm_bio *b)
{
    if (!b)
        return;
    if (b->s)
        (void)hipStreamSynchronize(b->s->ctx->stream);
    free_dev(b);
    (void)hipFree(b->d_c);
    (void)hipFree(b->d_out);
    if (b->h_out)
        (void)hipHostFree(b->h_out);
    delete b;
}

lbm_status lbm_bio_create(lbm_solver *s, const lbm_bio_params *p, const double *c_bio,
                          const double *m_ox, lbm_bio **out)
{
    if (!s || !p || !out)
        return LBM_EINVAL;
    *out = nullptr;
    std::string msg = check_params(*p);
    if (!msg.empty())
        return set_err(s->ctx, LBM_EINVAL, msg);
    const size_t N = (size_t)s->geo.N;
    if (N > (size_t)INT32_MAX)
        return set_err(s->ctx, LBM_EINVAL, "bio model needs fewer than 2^31 nodes");
    lbm_bio *b = new lbm_bio;
    b->s = s;
    b->p = *p;
    b->cb.assign(N, 0.0);
    b->mox.assign(N, 0.0);
    for (size_t n = 0; n < N; ++n) {
        const double c = c_bio ? c_bio[n] : (s->cls[n] == LBM_BIOFILM ? p->C0_bio : 0.0);
        const double m = m_ox ? m_ox[n] : p->M_total;
        msg = check_node(b, (int64_t)n, c, m);
        if (!msg.empty()) {
            delete b;
            return set_err(s->ctx, LBM_EINVAL, msg);
        }
        b->cb[n] = c;
        b->mox[n] = c > 0.0 ? m : 0.0;
    }
    hipError_t e = hipSetDevice(s->ctx->device);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->d_c, N * 8);
    if (e == hipSuccess)
        e = hipMalloc((void **)&b->d_out, sizeof(lbm_bio_out));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&b->h_out, sizeof(lbm_bio_out), hipHostMallocDefault);
    if (e != hipSuccess) {
        lbm_bio_destroy(b);
        return set_err(s->ctx, LBM_ENOMEM, "bio state");
    }
    lbm_status st = bio_push_cells(b);
    if (st) {
        lbm_bio_destroy(b);
        return st;
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_bio_step(lbm_bio *b, lbm_bio_out *out)
{
    if (!b)
        return LBM_EINVAL;
    lbm_solver *s = b->s;
    for (int32_t n : b->cells)
        if (s->cls[(size_t)n] != LBM_BIOFILM)
            return set_err(s->ctx, LBM_EINVAL,
                           "node " + std::to_string(n) + " holds biomass but is no longer BIOFILM");
    const lbm_bio_params &p = b->p;
    const int ncell = (int)b->cells.size();
    lbm_bio_out o{};
    if (ncell == 0) {  // no biomass: no current
        if (!s->ad_ready)
            return set_err(s->ctx, LBM_EINVAL, "substrate state not initialised");
        if (out)
            *out = o;
        return LBM_OK;
    }
    lbm_status st = export_c_device(s, b->d_c);
    if (st)
        return st;
    BioK k;
    k.q_max = p.q_max;
    k.K_s = p.K_s;
    k.M_total = p.M_total;
    k.K_Mox = p.K_Mox;
    k.E0 = p.E0;
    k.R_ext = p.R_ext;
    k.R_int = p.R_int;
    k.eps = p.eps;
    k.c_scale = p.c_scale;
    k.red_dt = p.Y * p.q_max * (p.dt_hours / 24.0);
    k.beta_per_amp = p.gamma * (p.dt_hours * 3600.0) / (p.m * FARADAY * b->biomass);
    k.phi = R_GAS * p.T / FARADAY;
    k.act_per_amp = k.phi / (p.m * p.A_a * p.I0);
    k.sum_cb = b->sum_cb;
    k.biomass = b->biomass;
    k.q_scale = (p.V_a / (double)s->geo.N) / 24.0;
    hipStream_t stream = s->ctx->stream;
    hipLaunchKernelGGL(k_bio_interval, dim3(1), dim3(BIO_THREADS), 0, stream, ncell, b->d_idx, b->d_cb,
                       b->d_mox, b->d_fs, b->d_c, k, b->d_out);
    BIOCHK(hipGetLastError(), "bio launch");
    BIOCHK(hipMemcpyAsync(b->h_out, b->d_out, sizeof(lbm_bio_out), hipMemcpyDeviceToHost, stream), "bio out");
    BIOCHK(hipStreamSynchronize(stream), "bio sync");
    b->mox_stale = true;
    if (out)
        *out = *b->h_out;
    return LBM_OK;
}

lbm_status lbm_bio_get(lbm_bio *b, int field, double *dst)
{
    if (!b || !dst || (field != LBM_BIO_CBIO && field != LBM_BIO_MOX))
        return LBM_EINVAL;
    if (field == LBM_BIO_CBIO) {
        memcpy(dst, b->cb.data(), b->cb.size() * 8);
        return LBM_OK;
    }
    lbm_status st = bio_pull_mox(b);
    if (st)
        return st;
    memcpy(dst, b->mox.data(), b->mox.size() * 8);
    return LBM_OK;
}

lbm_status lbm_bio_set(lbm_bio *b, const int64_t *nodes, const double *c_bio, const double *m_ox,
                       int64_t n)
{
    if (!b || n < 0 || (n > 0 && (!nodes || !c_bio || !m_ox)))
        return LBM_EINVAL;
    const int64_t N = (int64_t)b->cb.size();
    for (int64_t i = 0; i < n; ++i) {
        if (nodes[i] < 0 || nodes[i] >= N)
            return set_err(b->s->ctx, LBM_EINVAL, "node index out of range");
        std::string msg = check_node(b, nodes[i], c_bio[i], m_ox[i]);
        if (!msg.empty())
            return set_err(b->s->ctx, LBM_EINVAL, msg);
    }
    lbm_status st = bio_pull_mox(b);
    if (st)
        return st;
    for (int64_t i = 0; i < n; ++i) {
        b->cb[(size_t)nodes[i]] = c_bio[i];
        b->mox[(size_t)nodes[i]] = c_bio[i] > 0.0 ? m_ox[i] : 0.0;
    }
    return bio_push_cells(b);
}

} // extern "C"

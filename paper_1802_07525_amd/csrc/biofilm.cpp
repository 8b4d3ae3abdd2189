// biofilm.cpp -- the agent-based biofilm of Sec. 2.3 and the model loop of
// Sec. 2 (fluid, substrate, bio-electrochemistry, biofilm; one hour each).
//
// Attachment, growth and spreading act on a few thousand biomass cells per
// interval with data-dependent random walks and chains of moves: sequential
// host work.  It reads the substrate field once (the GPU exports it), works
// on the host mirrors of the bio state, and hands the nodes that turn
// BIOFILM to lbm_solver_update_cells, which patches descriptor words and
// populations on the device incrementally.  Nothing is changed when that
// update is refused (growth would close the flow path).
#include <math.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbmh;

namespace {

// SplitMix64 draws as the stages consume them
struct Draws {
    SplitMix64 r;
    double uniform() { return (double)(r.next() >> 11) * 0x1.0p-53; }
    int64_t index(int64_t m) { return (int64_t)(uniform() * (double)m); }
};

struct Grid {
    int nx, ny, nz;
    int64_t N;
    const Dirs *dirs;
    // neighbour of n along direction i, or -1 off the grid
    int64_t nb(int64_t n, int i) const
    {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        const int x2 = x + dirs->c[i][0], y2 = y + dirs->c[i][1], z2 = z + dirs->c[i][2];
        if (x2 < 0 || x2 >= nx || y2 < 0 || y2 >= ny || z2 < 0 || z2 >= nz)
            return -1;
        return x2 + (int64_t)nx * (y2 + (int64_t)ny * z2);
    }
};

std::string check_film(const lbm_biofilm_params &p)
{
    if (p.k_ata < 0 || p.max_walk < 0)
        return "k_ata and max_walk must be >= 0";
    if (!(p.C_max > 0.0) || !isfinite(p.C_max))
        return "C_max must be finite and > 0";
    if (!(p.fr_spr > 0.0 && p.fr_spr < 1.0))
        return "fr_spr must lie in (0, 1)";
    if (!(p.Y_bio >= 0.0) || !isfinite(p.Y_bio))
        return "Y_bio must be finite and >= 0";
    return "";
}

} // namespace

extern "C" {

lbm_status lbm_biofilm_step(lbm_bio *b, const lbm_biofilm_params *fp, uint64_t seed,
                            lbm_biofilm_stats *out)
{
    if (!b || !fp)
        return LBM_EINVAL;
    lbm_solver *s = b->s;
    Range rg("lbm.biofilm.step");
    std::string msg = check_film(*fp);
    if (!msg.empty())
        return set_err(s->ctx, LBM_EINVAL, msg);
    if (!s->ad_ready)
        return set_err(s->ctx, LBM_EINVAL, "substrate state not initialised");
    const lbm_bio_params &bp = b->p;
    Grid G{s->grid.nx, s->grid.ny, s->grid.nz, s->geo.N, &fluid_dirs(s->grid.nz)};
    const int64_t N = G.N;
    std::vector<double> C((size_t)N);
    lbm_status st = lbm_solver_get(s, LBM_FIELD_C, C.data());
    if (st)
        return st;
    if ((st = bio_pull_mox(b)))
        return st;
    std::vector<uint8_t> cls = s->cls;
    std::vector<double> cb = b->cb, mo = b->mox;
    auto free_node = [&](int64_t n) {
        return n >= 0 && cls[(size_t)n] == LBM_FLUID && n % G.nx >= 1 && n % G.nx <= G.nx - 2;
    };
    Draws rnd{SplitMix64{seed}};
    std::vector<int64_t> grown;
    lbm_biofilm_stats o{};

    // 1. attachment on the fluid-electrode front
    std::vector<int64_t> front;
    for (int64_t n = 0; n < N; ++n) {
        if (!free_node(n))
            continue;
        for (int i = 1; i < G.dirs->q; ++i) {
            const int64_t m = G.nb(n, i);
            if (m >= 0 && cls[(size_t)m] == LBM_SOLID) {
                front.push_back(n);
                break;
            }
        }
    }
    const int64_t k = std::min<int64_t>(fp->k_ata, (int64_t)front.size());
    for (int64_t i = 0; i < k; ++i) {
        const int64_t j = i + rnd.index((int64_t)front.size() - i);
        std::swap(front[(size_t)i], front[(size_t)j]);
        const int64_t n = front[(size_t)i];
        cls[(size_t)n] = LBM_BIOFILM;
        cb[(size_t)n] = bp.C0_bio;
        mo[(size_t)n] = bp.M_total;
        grown.push_back(n);
    }
    o.attached = (int32_t)k;

    // 2. growth at the consumption rate of Eq. 16
    const double dt_day = bp.dt_hours / 24.0;
    for (int64_t n = 0; n < N; ++n) {
        const double c = cb[(size_t)n];
        if (!(c > 0.0))
            continue;
        const double S = bp.c_scale * std::max(C[(size_t)n], 0.0);
        const double M = mo[(size_t)n];
        const double q = bp.q_max * S / (S + bp.K_s) * M / (M + bp.K_Mox);
        cb[(size_t)n] = c + dt_day * (fp->Y_bio * q) * c;
    }

    // 3. spreading above C_max
    std::vector<int64_t> path, freeb;
    for (int64_t n = 0; n < N; ++n) {
        if (!(cb[(size_t)n] > fp->C_max))
            continue;
        freeb.clear();
        for (int i = 1; i < G.dirs->q; ++i) {
            const int64_t m = G.nb(n, i);
            if (free_node(m))
                freeb.push_back(m);
        }
        path.assign(1, n);
        if (!freeb.empty()) {
            path.push_back(freeb[(size_t)rnd.index((int64_t)freeb.size())]);
        } else {
            ++o.walks;
            int64_t cur = n;
            bool found = false;
            for (int32_t step = 0; step < fp->max_walk && !found; ++step) {
                const int64_t m = G.nb(cur, 1 + (int)rnd.index(G.dirs->q - 1));
                if (free_node(m)) {
                    path.push_back(m);
                    found = true;
                } else if (m >= 0 && cls[(size_t)m] == LBM_BIOFILM) {
                    auto it = std::find(path.begin(), path.end(), m);
                    if (it != path.end())
                        path.erase(it + 1, path.end());  // erase the loop
                    else
                        path.push_back(m);
                    cur = m;
                }
            }
            if (!found) {
                ++o.abandoned;
                continue;
            }
        }
        // move everything one node outward along the path, then split
        for (size_t i = path.size() - 1; i >= 2; --i) {
            cb[(size_t)path[i]] = cb[(size_t)path[i - 1]];
            mo[(size_t)path[i]] = mo[(size_t)path[i - 1]];
        }
        const double share = fp->fr_spr * cb[(size_t)n];
        cb[(size_t)path[1]] = share;
        mo[(size_t)path[1]] = mo[(size_t)n];
        cb[(size_t)n] = cb[(size_t)n] - share;
        cls[(size_t)path.back()] = LBM_BIOFILM;
        grown.push_back(path.back());
        ++o.spread;
    }

    // apply: classes on the solver (refused if the flow path closes), then
    // the bio fields
    if (!grown.empty()) {
        std::vector<uint8_t> bio(grown.size(), LBM_BIOFILM);
        if ((st = lbm_solver_update_cells(s, grown.data(), bio.data(), (int64_t)grown.size())))
            return st;
    }
    b->cb.swap(cb);
    b->mox.swap(mo);
    b->mox_stale = false;
    if ((st = bio_push_cells(b)))
        return st;
    o.new_biofilm = (int32_t)grown.size();
    o.cells = (int32_t)b->cells.size();
    o.biomass = b->biomass;
    if (out)
        *out = o;
    return LBM_OK;
}

lbm_status lbm_mfc_run(lbm_bio *b, const lbm_biofilm_params *fp, int n_hours, uint64_t seed,
                       double tol, int64_t max_iter, lbm_mfc_interval *series)
{
    if (!b || !fp || n_hours < 0 || (n_hours > 0 && !series))
        return LBM_EINVAL;
    lbm_solver *s = b->s;
    SplitMix64 seeds{seed};
    using clk = std::chrono::steady_clock;
    auto secs = [](clk::time_point a, clk::time_point z) { return std::chrono::duration<double>(z - a).count(); };
    for (int h = 0; h < n_hours; ++h) {
        Range rg("lbm.mfc.hour");
        lbm_mfc_interval &r = series[h];
        r = lbm_mfc_interval{};
        lbm_info fi{}, ai{};
        const auto t0 = clk::now();
        r.nodes_fluid = s->n_fluid;
        r.nodes_ad = s->n_ad;
        const lbm_status sf = lbm_solver_fluid(s, tol, max_iter, h > 0, &fi);
        r.status_fluid = sf;
        r.iters_fluid = fi.iters;
        if (sf < 0)
            return sf;
        const lbm_status sa = lbm_solver_ad(s, tol, max_iter, h > 0, &ai);
        r.status_ad = sa;
        r.iters_ad = ai.iters;
        if (sa < 0)
            return sa;
        const auto t1 = clk::now();
        r.seconds_solves = secs(t0, t1);
        lbm_status st = lbm_bio_step(b, &r.bio);
        const auto t2 = clk::now();
        r.seconds_bio = secs(t1, t2);
        if (st)
            return st;
        st = lbm_biofilm_step(b, fp, seeds.next(), &r.film);
        r.seconds_film = secs(t2, clk::now());
        if (st)
            return st;
    }
    return LBM_OK;
}

} // extern "C"

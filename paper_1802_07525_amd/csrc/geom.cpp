// geom.cpp -- host-side integer geometry: seeded electrodes, biofilm layer,
// link masks, node descriptors, percolation and the biofilm growth pick.
//
// The paper's electrode is a random porous geometry (Sec. 3) whose figure is
// not published; the generators below are seeded stand-ins specified in
// integer arithmetic so that any two implementations agree byte for byte.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace lbmh {

static Dirs make_dirs(int q, const int (*c)[3])
{
    Dirs d;
    d.q = q;
    for (int i = 0; i < q; ++i)
        for (int k = 0; k < 3; ++k)
            d.c[i][k] = c[i][k];
    return d;
}

// Same direction numbering as the kernels (lbm.h documents it).
static const int C_D2Q9[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int C_D3Q19[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                   {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                   {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                   {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

const Dirs &fluid_dirs(int nz)
{
    static const Dirs d2 = make_dirs(9, C_D2Q9), d3 = make_dirs(19, C_D3Q19);
    return nz > 1 ? d3 : d2;
}
const Dirs &ad_dirs(int nz)
{
    static const Dirs d2 = make_dirs(5, C_D2Q9), d3 = make_dirs(7, C_D3Q19);
    return nz > 1 ? d3 : d2;
}

bool fluid_blocked(uint8_t k)
{
    return k == LBM_SOLID || k == LBM_WALL || k == LBM_BIOFILM;
}
bool ad_blocked(uint8_t k)
{
    return k == LBM_SOLID || k == LBM_WALL;
}

static inline int64_t idx3(const lbm_grid &g, int64_t x, int64_t y, int64_t z)
{
    return x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
}

static void fill_chassis(const lbm_grid &g, uint8_t *cls)
{
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y) {
            const bool wall = y == 0 || y == g.ny - 1 || (g.nz > 1 && (z == 0 || z == g.nz - 1));
            memset(cls + idx3(g, 0, y, z), wall ? LBM_WALL : LBM_FLUID, (size_t)g.nx);
        }
}

std::string check_cell(const lbm_grid &g, int x, int y, int z, uint8_t k)
{
    const bool chassis = y == 0 || y == g.ny - 1 || (g.nz > 1 && (z == 0 || z == g.nz - 1));
    if (k > LBM_BIOFILM)
        return "unknown node class " + std::to_string(k);
    if (chassis && !(k == LBM_WALL || k == LBM_SOLID))
        return "chassis rows/planes must be WALL or SOLID";
    if ((x == 0 || x == g.nx - 1) && (k == LBM_SOLID || k == LBM_BIOFILM))
        return "inlet/outlet columns must hold no SOLID or BIOFILM";
    return "";
}

std::string check_mask(const lbm_grid &g, const uint8_t *cls)
{
    if (g.nx < 2 || g.ny < 3 || g.nz < 1 || g.nz == 2)
        return "grid must have nx >= 2, ny >= 3 and nz == 1 or nz >= 3";
    int64_t n = 0;
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x, ++n) {
                std::string m = check_cell(g, x, y, z, cls[n]);
                if (!m.empty())
                    return m;
            }
    return "";
}

} // namespace lbmh

using namespace lbmh;

extern "C" {

void lbm_splitmix64(uint64_t seed, int64_t count, uint64_t *out)
{
    SplitMix64 r{seed};
    for (int64_t k = 0; k < count; ++k)
        out[k] = r.next();
}

lbm_status lbm_geom_discs(lbm_grid g, const lbm_disc_params *p, uint64_t seed, uint8_t *cls,
                          double *achieved)
{
    if (!p || !cls || g.nz != 1 || g.nx < 4 || g.ny < 3 || p->r_min < 0 || p->r_max < p->r_min ||
        !(p->solid_frac >= 0.0 && p->solid_frac <= 1.0))
        return LBM_EINVAL;
    Range rg("lbm.geometry");
    fill_chassis(g, cls);
    const int64_t xa = g.nx / 4, xb = 3 * (int64_t)g.nx / 4, ya = 1, yb = g.ny - 1;
    const int64_t region = (xb - xa) * (yb - ya);
    const int64_t target = (int64_t)ceil(p->solid_frac * (double)region);
    struct Disc {
        int64_t x, y, r;
    };
    std::vector<Disc> placed;
    // Accepted discs are bucketed by centre on a grid of cell size
    // 2 r_max + 1: a disc can only clash with discs in its own or the eight
    // neighbouring cells.  "Any clash" does not depend on the order of the
    // comparisons, so the result equals that of a scan over all discs.
    const int64_t cell = 2 * (int64_t)p->r_max + 1;
    const int64_t gx = (xb - xa) / cell + 1, gy = (yb - ya) / cell + 1;
    std::vector<std::vector<int32_t>> bucket(p->overlap ? 0 : (size_t)(gx * gy));
    SplitMix64 rng{seed};
    int64_t solid = 0, attempts = 0;
    lbm_status st = LBM_OK;
    while (solid < target) {
        if (attempts == 1000000) {
            st = LBM_EINVAL;
            break;
        }
        ++attempts;
        Disc d;
        d.x = rng.pick(xa, xb - 1);
        d.y = rng.pick(ya, yb - 1);
        d.r = rng.pick(p->r_min, p->r_max);
        if (!p->overlap) {
            const int64_t cx = (d.x - xa) / cell, cy = (d.y - ya) / cell;
            bool apart = true;
            for (int64_t by = cy - 1; by <= cy + 1 && apart; ++by)
                for (int64_t bx = cx - 1; bx <= cx + 1 && apart; ++bx) {
                    if (bx < 0 || by < 0 || bx >= gx || by >= gy)
                        continue;
                    for (int32_t k : bucket[(size_t)(bx + gx * by)]) {
                        const Disc &o = placed[(size_t)k];
                        const int64_t dx = d.x - o.x, dy = d.y - o.y, rr = d.r + o.r;
                        if (dx * dx + dy * dy <= rr * rr) {
                            apart = false;
                            break;
                        }
                    }
                }
            if (!apart)
                continue;
            bucket[(size_t)(cx + gx * cy)].push_back((int32_t)placed.size());
        }
        placed.push_back(d);
        const int64_t y0 = d.y - d.r < ya ? ya : d.y - d.r, y1 = d.y + d.r >= yb ? yb - 1 : d.y + d.r;
        const int64_t x0 = d.x - d.r < xa ? xa : d.x - d.r, x1 = d.x + d.r >= xb ? xb - 1 : d.x + d.r;
        for (int64_t y = y0; y <= y1; ++y)
            for (int64_t x = x0; x <= x1; ++x) {
                const int64_t dx = x - d.x, dy = y - d.y;
                if (dx * dx + dy * dy <= d.r * d.r) {
                    uint8_t &c = cls[idx3(g, x, y, 0)];
                    if (c != LBM_SOLID) {
                        c = LBM_SOLID;
                        ++solid;
                    }
                }
            }
    }
    if (achieved)
        *achieved = (double)solid / (double)region;
    return st;
}

lbm_status lbm_geom_fibres(lbm_grid g, const lbm_fibre_params *p, uint64_t seed, uint8_t *cls,
                           double *achieved)
{
    if (!p || !cls || g.nx < 4 || g.ny < 3 || g.nz < 3 || p->r_min < 0 || p->r_max < p->r_min ||
        !(p->solid_frac >= 0.0 && p->solid_frac <= 1.0))
        return LBM_EINVAL;
    Range rg("lbm.geometry");
    fill_chassis(g, cls);
    const int64_t xa = g.nx / 4, xb = 3 * (int64_t)g.nx / 4;
    const int64_t region = (xb - xa) * (int64_t)(g.ny - 2) * (g.nz - 2);
    const int64_t target = (int64_t)ceil(p->solid_frac * (double)region);
    SplitMix64 rng{seed};
    int64_t solid = 0, attempts = 0;
    lbm_status st = LBM_OK;
    while (solid < target) {
        if (attempts == 1000000) {
            st = LBM_EINVAL;
            break;
        }
        ++attempts;
        const int64_t qx = rng.pick(xa, xb - 1), qy = rng.pick(1, g.ny - 2), qz = rng.pick(1, g.nz - 2);
        int64_t dx, dy, dz;
        do {
            dx = rng.pick(-4, 4);
            dy = rng.pick(-4, 4);
            dz = rng.pick(-4, 4);
        } while (dx == 0 && dy == 0 && dz == 0);
        const int64_t r = rng.pick(p->r_min, p->r_max);
        const int64_t lim = r * r * (dx * dx + dy * dy + dz * dz);
        for (int64_t z = 1; z < g.nz - 1; ++z)
            for (int64_t y = 1; y < g.ny - 1; ++y) {
                const int64_t py = y - qy, pz = z - qz;
                for (int64_t x = xa; x < xb; ++x) {
                    const int64_t px = x - qx;
                    const int64_t ax = py * dz - pz * dy, ay = pz * dx - px * dz, az = px * dy - py * dx;
                    if (ax * ax + ay * ay + az * az <= lim) {
                        uint8_t &c = cls[idx3(g, x, y, z)];
                        if (c != LBM_SOLID) {
                            c = LBM_SOLID;
                            ++solid;
                        }
                    }
                }
            }
    }
    if (achieved)
        *achieved = (double)solid / (double)region;
    return st;
}

lbm_status lbm_biofilm_layer(lbm_grid g, uint8_t *cls)
{
    if (!cls || g.nx < 1 || g.ny < 1 || g.nz < 1)
        return LBM_EINVAL;
    const Dirs &D = fluid_dirs(g.nz);
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    std::vector<uint8_t> before(cls, cls + N);
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                const int64_t n = idx3(g, x, y, z);
                if (before[n] != LBM_FLUID)
                    continue;
                for (int i = 1; i < D.q; ++i) {
                    const int sx = x + D.c[i][0], sy = y + D.c[i][1], sz = z + D.c[i][2];
                    if (sx < 0 || sy < 0 || sz < 0 || sx >= g.nx || sy >= g.ny || sz >= g.nz)
                        continue;
                    if (before[idx3(g, sx, sy, sz)] == LBM_SOLID) {
                        cls[n] = LBM_BIOFILM;
                        break;
                    }
                }
            }
    return LBM_OK;
}

} // extern "C"

namespace lbmh {

// Link bits of node (x, y, z): bit i set iff the pull source (x, y, z) - c_i
// is inside the grid and blocked for that solver.
template <bool FLUID>
static inline uint32_t link_bits(const lbm_grid &g, const uint8_t *cls, int x, int y, int z)
{
    const Dirs &D = FLUID ? fluid_dirs(g.nz) : ad_dirs(g.nz);
    const int64_t n = idx3(g, x, y, z);
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
    uint32_t bits = 0;
    for (int i = 1; i < D.q; ++i) {
        const int ax = x - D.c[i][0], ay = y - D.c[i][1], az = z - D.c[i][2];
        if (ax < 0 || ay < 0 || az < 0 || ax >= g.nx || ay >= g.ny || az >= g.nz)
            continue;
        const uint8_t k = cls[n - D.c[i][0] - D.c[i][1] * sy - D.c[i][2] * sz];
        if (FLUID ? fluid_blocked(k) : ad_blocked(k))
            bits |= 1u << i;
    }
    return bits;
}

template <bool FLUID>
static void links_impl(const lbm_grid &g, const uint8_t *cls, uint32_t *out)
{
    int64_t n = 0;
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x, ++n)
                out[n] = link_bits<FLUID>(g, cls, x, y, z);
}

void links_fluid(const lbm_grid &g, const uint8_t *cls, uint32_t *out)
{
    links_impl<true>(g, cls, out);
}
void links_ad(const lbm_grid &g, const uint8_t *cls, uint32_t *out)
{
    links_impl<false>(g, cls, out);
}

// Flow domain: the FLUID nodes joined to a FLUID node of the outlet column
// x = nx-1 by a chain of fluid-lattice links between FLUID nodes.  A closed
// pore (no such chain) holds no steady flow and its pressure is set by no
// boundary condition; a pocket reached from the inlet alone would gain the
// inflow forever.  Both stay out of the flow solve (Sec. 2.1.1 boundary
// conditions on the Sec. 3 pore space); the substrate solve keeps them.
//
// The search runs over maximal FLUID runs along x in each row (y, z)
// rather than over nodes.  Runs [a, b] and [c, d] of two rows are linked
// iff some of their nodes are lattice neighbours: c <= b + w and
// a <= d + w, where w = 1 for rows one apart in y or in z (the lattice
// has (+-1, +-1, 0) and (+-1, 0, +-1)) and w = 0 for rows one apart in both
// (D3Q19's (0, +-1, +-1) edges, no corners).
std::vector<uint8_t> flow_domain(const lbm_grid &g, const uint8_t *cls)
{
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int64_t rows = (int64_t)g.ny * g.nz;
    struct Run {
        int a, b;
    };
    std::vector<Run> runs;
    std::vector<int64_t> first((size_t)rows + 1);
    for (int64_t r = 0; r < rows; ++r) {
        first[(size_t)r] = (int64_t)runs.size();
        const uint8_t *c = cls + r * g.nx;
        for (int x = 0; x < g.nx;) {
            if (c[x] != LBM_FLUID) {
                ++x;
                continue;
            }
            const int a = x;
            while (x < g.nx && c[x] == LBM_FLUID)
                ++x;
            runs.push_back({a, x - 1});
        }
    }
    first[(size_t)rows] = (int64_t)runs.size();
    const int64_t R = (int64_t)runs.size();
    std::vector<int64_t> row_of((size_t)R);
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t k = first[(size_t)r]; k < first[(size_t)r + 1]; ++k)
            row_of[(size_t)k] = r;
    std::vector<uint8_t> seen((size_t)R, 0);
    std::vector<int64_t> todo;
    for (int64_t r = 0; r < rows; ++r)
        if (first[(size_t)r + 1] > first[(size_t)r] && runs[(size_t)first[(size_t)r + 1] - 1].b == g.nx - 1) {
            seen[(size_t)first[(size_t)r + 1] - 1] = 1;
            todo.push_back(first[(size_t)r + 1] - 1);
        }
    // neighbouring rows (dy, dz) and their widening
    struct Nb {
        int dy, dz, w;
    };
    static const Nb nb2[2] = {{1, 0, 1}, {-1, 0, 1}};
    static const Nb nb3[8] = {{1, 0, 1},  {-1, 0, 1},  {0, 1, 1},  {0, -1, 1},
                              {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    const Nb *nb = g.nz > 1 ? nb3 : nb2;
    const int nnb = g.nz > 1 ? 8 : 2;
    while (!todo.empty()) {
        const int64_t k = todo.back();
        todo.pop_back();
        const Run q = runs[(size_t)k];
        const int64_t r = row_of[(size_t)k];
        const int y = (int)(r % g.ny), z = (int)(r / g.ny);
        for (int t = 0; t < nnb; ++t) {
            const int ay = y + nb[t].dy, az = z + nb[t].dz;
            if (ay < 0 || az < 0 || ay >= g.ny || az >= g.nz)
                continue;
            const int64_t r2 = ay + (int64_t)g.ny * az;
            const int lo = q.a - nb[t].w, hi = q.b + nb[t].w;
            // first run of row r2 ending at or after lo
            int64_t i0 = first[(size_t)r2], i1 = first[(size_t)r2 + 1];
            while (i0 < i1) {
                const int64_t mid = (i0 + i1) / 2;
                if (runs[(size_t)mid].b < lo)
                    i0 = mid + 1;
                else
                    i1 = mid;
            }
            for (int64_t m = i0; m < first[(size_t)r2 + 1] && runs[(size_t)m].a <= hi; ++m)
                if (!seen[(size_t)m]) {
                    seen[(size_t)m] = 1;
                    todo.push_back(m);
                }
        }
    }
    std::vector<uint8_t> in((size_t)N, 0);
    for (int64_t k = 0; k < R; ++k)
        if (seen[(size_t)k]) {
            uint8_t *row = in.data() + row_of[(size_t)k] * g.nx;
            memset(row + runs[(size_t)k].a, 1, (size_t)(runs[(size_t)k].b - runs[(size_t)k].a + 1));
        }
    return in;
}

bool domain_reaches_inlet(const lbm_grid &g, const std::vector<uint8_t> &dom)
{
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            if (dom[(size_t)idx3(g, 0, y, z)])
                return true;
    return false;
}

// The flow-domain node of each column x that samples the column's shift
// reference: the one nearest the middle of the cross-section
// (|y - ny/2| + |z - nz/2|), the lowest index among equals; -1 for a column
// without flow-domain nodes.
std::vector<int64_t> reference_nodes(const lbm_grid &g, const std::vector<uint8_t> &dom)
{
    std::vector<int64_t> r((size_t)g.nx, -1);
    std::vector<int> best((size_t)g.nx, INT32_MAX);
    const int cy = g.ny / 2, cz = g.nz / 2;
    int64_t n = 0;
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y) {
            const int dist = abs(y - cy) + abs(z - cz);
            for (int x = 0; x < g.nx; ++x, ++n)
                if (dom[(size_t)n] && dist < best[x]) {
                    best[x] = dist;
                    r[x] = n;
                }
        }
    return r;
}

uint32_t desc_word(const lbm_grid &g, const uint8_t *cls, const uint8_t *dom, bool ref, int x, int y,
                   int z)
{
    const int qf = fluid_dirs(g.nz).q, qa = ad_dirs(g.nz).q;
    const int64_t n = idx3(g, x, y, z);
    const uint8_t k = cls[n];
    uint32_t d = 0;
    if (dom[n])
        d |= 1u | (link_bits<true>(g, cls, x, y, z) & ((1u << qf) - 2u));
    if (k == LBM_FLUID || k == LBM_BIOFILM) {
        const uint32_t la = link_bits<false>(g, cls, x, y, z);
        for (int i = 1; i < qa; ++i)
            if (la & (1u << i))
                d |= 1u << lbmk::desc_ad_link_bit(qf, i);
        d |= 1u << lbmk::desc_ad_active_bit(qf, qa);
    }
    if (k == LBM_BIOFILM)
        d |= 1u << lbmk::desc_biofilm_bit(qf, qa);
    if (ref)
        d |= 1u << lbmk::desc_ref_bit(qf, qa);
    return d;
}

uint16_t ad9_desc_word(const lbm_grid &g, const uint8_t *cls, bool ref, int x, int y)
{
    // the D2Q9 substrate's own word: bits 1..8 blocked pull sources (D2Q9
    // directions, substrate rule), then active, BIOFILM, reference node --
    // the substrate layout with no fluid bits below it (fluid Q taken as 1)
    const Dirs &D = fluid_dirs(1);
    const int64_t n = idx3(g, x, y, 0);
    const uint8_t k = cls[n];
    uint32_t d = 0;
    if (k == LBM_FLUID || k == LBM_BIOFILM) {
        for (int i = 1; i < D.q; ++i) {
            const int ax = x - D.c[i][0], ay = y - D.c[i][1];
            if (ax < 0 || ay < 0 || ax >= g.nx || ay >= g.ny)
                continue;
            if (ad_blocked(cls[idx3(g, ax, ay, 0)]))
                d |= 1u << lbmk::desc_ad_link_bit(1, i);
        }
        d |= 1u << lbmk::desc_ad_active_bit(1, D.q);
    }
    if (k == LBM_BIOFILM)
        d |= 1u << lbmk::desc_biofilm_bit(1, D.q);
    if (ref)
        d |= 1u << lbmk::desc_ref_bit(1, D.q);
    return (uint16_t)d;
}

void build_desc(const lbm_grid &g, const uint8_t *cls, const std::vector<uint8_t> &dom,
                const std::vector<int64_t> &ref, uint32_t *desc)
{
    int64_t n = 0;
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x, ++n)
                desc[n] = desc_word(g, cls, dom.data(), n == ref[(size_t)x], x, y, z);
}

void build_desc(const lbm_grid &g, const uint8_t *cls, uint32_t *desc)
{
    const std::vector<uint8_t> dom = flow_domain(g, cls);
    build_desc(g, cls, dom, reference_nodes(g, dom), desc);
}

// Inlet FLUID nodes are joined to the outlet column iff one of them is in
// the flow domain (joining is symmetric).
bool percolates(const lbm_grid &g, const uint8_t *cls)
{
    return domain_reaches_inlet(g, flow_domain(g, cls));
}

int64_t growth_pick(const lbm_grid &g, const uint8_t *cls, const double *C, double xi)
{
    const Dirs &D = fluid_dirs(g.nz);
    std::vector<int64_t> cand;
    // per row: near[x] = some lattice neighbour of (x, y, z) is BIOFILM, from
    // the neighbouring rows' BIOFILM flags shifted by c_x (byte loops)
    std::vector<uint8_t> near((size_t)g.nx), bio((size_t)g.nx);
    for (int z = 0; z < g.nz; ++z)
        for (int y = 0; y < g.ny; ++y) {
            std::fill(near.begin(), near.end(), 0);
            for (int i = 1; i < D.q; ++i) {
                const int ay = y + D.c[i][1], az = z + D.c[i][2], cx = D.c[i][0];
                if (ay < 0 || az < 0 || ay >= g.ny || az >= g.nz)
                    continue;
                const uint8_t *row = cls + idx3(g, 0, ay, az);
                for (int x = 0; x < g.nx; ++x)
                    bio[x] = row[x] == LBM_BIOFILM;
                // near[x] |= bio[x + cx] for x + cx inside the row
                const int lo = cx < 0 ? -cx : 0, hi = cx > 0 ? g.nx - cx : g.nx;
                for (int x = lo; x < hi; ++x)
                    near[x] |= bio[x + cx];
            }
            const int64_t n0 = idx3(g, 0, y, z);
            for (int x = 1; x < g.nx - 1; ++x)
                if (cls[n0 + x] == LBM_FLUID && near[x])
                    cand.push_back(n0 + x);
        }
    if (cand.empty())
        return -1;
    double W = 0.0;
    for (int64_t n : cand)
        W += C[n] > 0.0 ? C[n] : 0.0;
    if (W == 0.0) {
        int64_t k = (int64_t)floor(xi * (double)cand.size());
        if (k >= (int64_t)cand.size())
            k = (int64_t)cand.size() - 1;
        return cand[(size_t)k];
    }
    const double target = xi * W;
    double run = 0.0;
    int64_t last = -1;
    for (int64_t n : cand) {
        const double w = C[n] > 0.0 ? C[n] : 0.0;
        run += w;
        if (w > 0.0)
            last = n;
        if (run > target)
            return n;
    }
    return last;
}

lbm_status set_err(lbm_ctx *ctx, lbm_status st, const std::string &msg)
{
    if (ctx)
        ctx->err = msg;
    return st;
}

lbm_status hip_err(lbm_ctx *ctx, hipError_t e, const char *where)
{
    if (e == hipSuccess)
        return LBM_OK;
    if (ctx)
        ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
}

} // namespace lbmh

extern "C" {

lbm_status lbm_links(lbm_grid g, const uint8_t *cls, int which, void *out)
{
    if (!cls || !out || g.nx < 1 || g.ny < 1 || g.nz < 1 || (which != 0 && which != 1))
        return LBM_EINVAL;
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    std::vector<uint32_t> w((size_t)N);
    if (which == LBM_SOLVER_FLUID)
        links_fluid(g, cls, w.data());
    else
        links_ad(g, cls, w.data());
    for (int64_t n = 0; n < N; ++n) {
        if (which == LBM_SOLVER_AD)
            static_cast<uint8_t *>(out)[n] = (uint8_t)w[n];
        else if (g.nz > 1)
            static_cast<uint32_t *>(out)[n] = w[n];
        else
            static_cast<uint16_t *>(out)[n] = (uint16_t)w[n];
    }
    return LBM_OK;
}

int64_t lbm_link_list(lbm_grid g, const uint8_t *cls, int which, int64_t *out, int64_t cap)
{
    if (!cls || g.nx < 1 || g.ny < 1 || g.nz < 1 || (which != 0 && which != 1) || cap < 0 ||
        (cap > 0 && !out))
        return LBM_EINVAL;
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int q = which == 0 ? fluid_dirs(g.nz).q : ad_dirs(g.nz).q;
    std::vector<uint32_t> w((size_t)N);
    if (which == 0)
        links_fluid(g, cls, w.data());
    else
        links_ad(g, cls, w.data());
    int64_t count = 0;
    for (int64_t n = 0; n < N; ++n)
        for (int i = 1; i < q; ++i)
            if (w[n] & (1u << i)) {
                if (count < cap) {
                    out[2 * count] = n;
                    out[2 * count + 1] = i;
                }
                ++count;
            }
    return count;
}

int lbm_percolates(lbm_grid g, const uint8_t *cls)
{
    if (!cls || g.nx < 1 || g.ny < 1 || g.nz < 1)
        return LBM_EINVAL;
    return percolates(g, cls) ? 1 : 0;
}

lbm_status lbm_flow_domain(lbm_grid g, const uint8_t *cls, uint8_t *out)
{
    if (!cls || !out || g.nx < 1 || g.ny < 1 || g.nz < 1)
        return LBM_EINVAL;
    const std::vector<uint8_t> d = flow_domain(g, cls);
    memcpy(out, d.data(), d.size());
    return LBM_OK;
}

int64_t lbm_growth_pick(lbm_grid g, const uint8_t *cls, const double *C, double xi)
{
    if (!cls || !C || g.nx < 1 || g.ny < 1 || g.nz < 1)
        return -1;
    return growth_pick(g, cls, C, xi);
}

} // extern "C"

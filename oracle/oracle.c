/*
 * oracle.c -- plain, slow, FP64 CPU reference of the anode-compartment
 * lattice Boltzmann path of Tsompanas et al., "Modelling Microbial Fuel
 * Cells using lattice Boltzmann methods" (arXiv 1802.07525).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load this library.  It shares no
 * code, header, table or helper with the HIP library: every lattice table,
 * boundary rule, generator and reduction below is written out here on its
 * own, in double precision, in the paper's order and notation.
 *
 * What it computes (paper section / equation in brackets):
 *   - lattices D2Q9 [Sec. 2.1, Eqs. 1-3, 6-8], D2Q5, D3Q19, D3Q7 (the 3-D
 *     extension that Sec. 1 calls straightforward; D2Q5/D3Q7 for the
 *     advection-diffusion solver);
 *   - fluid BGK step: streaming, bounce-back on blocked neighbours
 *     [Sec. 2.1.1, Eq. 11], velocity inlet and pressure outlet links,
 *     moments [Eqs. 9-10], equilibrium [Eq. 5], BGK relaxation [Eq. 4];
 *   - advection-diffusion BGK step [Sec. 2.1.2, Eqs. 12-13] with the frozen
 *     fluid velocity, zero-flux solids, Dirichlet inlet, zero-gradient or
 *     Dirichlet outlet and a sink on biofilm nodes, first order or of the
 *     Monod form of the consumption rate (Eq. 16);
 *   - the flow domain: FLUID nodes linked to the outlet column (closed
 *     pores carry no steady flow; reading of Sec. 2.1.1 on the Sec. 3 pore
 *     space);
 *   - steady-state loops (each solver run to equilibrium, Sec. 3);
 *   - seeded geometry (random porous electrode, Sec. 3), biofilm layer,
 *     link masks, percolation and the simplified biofilm growth of the
 *     coupled loop (Sec. 2.3 re-solves fluid and substrate after each
 *     biofilm update, Sec. 2 model loop steps 2-6).
 *
 * Readings where the paper is silent or garbled (lattice speed c = 1,
 * half-way bounce-back, inlet/outlet link rules, linear AD equilibrium,
 * sink form, residual definition) are stated at the function that uses them.
 *
 * Build rules: C99, -O2 -ffp-contract=off, no fast-math, no intrinsics.
 * OpenMP is used only over independent rows; it changes no arithmetic.
 * Every sum runs over directions i = 0..Q-1 in ascending order, and every
 * global sum over nodes in ascending linear index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 19

/* node classes */
#define ORC_FLUID 0
#define ORC_SOLID 1
#define ORC_WALL 2
#define ORC_BIOFILM 3

/* lattice ids */
#define ORC_D2Q9 0
#define ORC_D2Q5 1
#define ORC_D3Q19 2
#define ORC_D3Q7 3

/* solve status codes (same meaning as the product's, own numbering) */
#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_STALLED 2
#define ORC_EINVAL (-1)
#define ORC_EDIVERGED (-4)

typedef struct {
    int q;
    int dim;
    int c[ORC_MAXQ][3];
    double w[ORC_MAXQ];
    int opp[ORC_MAXQ];
    double cs2;
} orc_lattice;

static void set_dir(orc_lattice *L, int i, int cx, int cy, int cz, double w)
{
    L->c[i][0] = cx;
    L->c[i][1] = cy;
    L->c[i][2] = cz;
    L->w[i] = w;
}

/* Velocity sets and weights.
 * D2Q9: Sec. 2.1, Eqs. 1-3 (c0 rest; c1,c3 = (+-1,0); c2,c4 = (0,+-1);
 * c5..c8 the diagonals) with weights 4/9, 1/9, 1/36 (Eqs. 6-8).  The paper
 * does not order c5..c8; Eq. 11 pairs 5 with 7 and 6 with 8 as opposites and
 * lets 5 and 6 move north, so 5=NE, 6=NW, 7=SW, 8=SE.
 * D2Q5 is D2Q9's first five directions with weights 1/3, 1/6 (c_s^2 = 1/3).
 * D3Q19: rest; +x,-x,+y,-y,+z,-z; then the twelve edge diagonals in
 * opposite pairs.  Weights 1/3, 1/18, 1/36 (c_s^2 = 1/3).
 * D3Q7 is D3Q19's first seven directions, weights 1/4, 1/8 (c_s^2 = 1/4). */
static int make_lattice(int id, orc_lattice *L)
{
    memset(L, 0, sizeof(*L));
    switch (id) {
    case ORC_D2Q9:
        L->q = 9;
        L->dim = 2;
        L->cs2 = 1.0 / 3.0;
        set_dir(L, 0, 0, 0, 0, 4.0 / 9.0);
        set_dir(L, 1, 1, 0, 0, 1.0 / 9.0);
        set_dir(L, 2, 0, 1, 0, 1.0 / 9.0);
        set_dir(L, 3, -1, 0, 0, 1.0 / 9.0);
        set_dir(L, 4, 0, -1, 0, 1.0 / 9.0);
        set_dir(L, 5, 1, 1, 0, 1.0 / 36.0);
        set_dir(L, 6, -1, 1, 0, 1.0 / 36.0);
        set_dir(L, 7, -1, -1, 0, 1.0 / 36.0);
        set_dir(L, 8, 1, -1, 0, 1.0 / 36.0);
        break;
    case ORC_D2Q5:
        L->q = 5;
        L->dim = 2;
        L->cs2 = 1.0 / 3.0;
        set_dir(L, 0, 0, 0, 0, 1.0 / 3.0);
        set_dir(L, 1, 1, 0, 0, 1.0 / 6.0);
        set_dir(L, 2, 0, 1, 0, 1.0 / 6.0);
        set_dir(L, 3, -1, 0, 0, 1.0 / 6.0);
        set_dir(L, 4, 0, -1, 0, 1.0 / 6.0);
        break;
    case ORC_D3Q19:
        L->q = 19;
        L->dim = 3;
        L->cs2 = 1.0 / 3.0;
        set_dir(L, 0, 0, 0, 0, 1.0 / 3.0);
        set_dir(L, 1, 1, 0, 0, 1.0 / 18.0);
        set_dir(L, 2, -1, 0, 0, 1.0 / 18.0);
        set_dir(L, 3, 0, 1, 0, 1.0 / 18.0);
        set_dir(L, 4, 0, -1, 0, 1.0 / 18.0);
        set_dir(L, 5, 0, 0, 1, 1.0 / 18.0);
        set_dir(L, 6, 0, 0, -1, 1.0 / 18.0);
        set_dir(L, 7, 1, 1, 0, 1.0 / 36.0);
        set_dir(L, 8, -1, -1, 0, 1.0 / 36.0);
        set_dir(L, 9, 1, -1, 0, 1.0 / 36.0);
        set_dir(L, 10, -1, 1, 0, 1.0 / 36.0);
        set_dir(L, 11, 1, 0, 1, 1.0 / 36.0);
        set_dir(L, 12, -1, 0, -1, 1.0 / 36.0);
        set_dir(L, 13, 1, 0, -1, 1.0 / 36.0);
        set_dir(L, 14, -1, 0, 1, 1.0 / 36.0);
        set_dir(L, 15, 0, 1, 1, 1.0 / 36.0);
        set_dir(L, 16, 0, -1, -1, 1.0 / 36.0);
        set_dir(L, 17, 0, 1, -1, 1.0 / 36.0);
        set_dir(L, 18, 0, -1, 1, 1.0 / 36.0);
        break;
    case ORC_D3Q7:
        L->q = 7;
        L->dim = 3;
        L->cs2 = 1.0 / 4.0;
        set_dir(L, 0, 0, 0, 0, 1.0 / 4.0);
        set_dir(L, 1, 1, 0, 0, 1.0 / 8.0);
        set_dir(L, 2, -1, 0, 0, 1.0 / 8.0);
        set_dir(L, 3, 0, 1, 0, 1.0 / 8.0);
        set_dir(L, 4, 0, -1, 0, 1.0 / 8.0);
        set_dir(L, 5, 0, 0, 1, 1.0 / 8.0);
        set_dir(L, 6, 0, 0, -1, 1.0 / 8.0);
        break;
    default:
        return -1;
    }
    /* opposite direction: the j with c_j = -c_i, found by search */
    for (int i = 0; i < L->q; i++) {
        L->opp[i] = -1;
        for (int j = 0; j < L->q; j++)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
                L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    }
    return 0;
}

/* Export a lattice's tables (for the identity pins). */
int orc_lattice_tables(int id, int *q, int *c /* [q][3] */, double *w,
                       int *opp, double *cs2)
{
    orc_lattice L;
    if (make_lattice(id, &L))
        return ORC_EINVAL;
    *q = L.q;
    for (int i = 0; i < L.q; i++) {
        c[3 * i + 0] = L.c[i][0];
        c[3 * i + 1] = L.c[i][1];
        c[3 * i + 2] = L.c[i][2];
        w[i] = L.w[i];
        opp[i] = L.opp[i];
    }
    *cs2 = L.cs2;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers: n = x + nx*(y + ny*z), x fastest.                           */

static int fluid_blocked(uint8_t k) /* fluid solver: biofilm is impermeable */
{
    return k == ORC_SOLID || k == ORC_WALL || k == ORC_BIOFILM;
}
static int ad_blocked(uint8_t k) /* substrate: zero flux only at electrode/chassis */
{
    return k == ORC_SOLID || k == ORC_WALL;
}
static uint8_t *flow_domain(int nx, int ny, int nz, const uint8_t *cls);

/* Substrate consumed in one step by a biofilm node at concentration C.
 * First order, k C, when k_half <= 0; otherwise the Monod form of the
 * consumption rate (Eq. 16 with the mediator factor folded into k),
 * k C / (C + k_half): k is the rate at saturation, k_half the half-
 * saturation concentration. */
static double consumed(double C, double k, double k_half)
{
    return k_half > 0.0 ? k * C / (C + k_half) : k * C;
}

/* Concentration C >= 0 before the sink, from the sum s of a biofilm node's
 * stored populations, s = C - consumed(C).  First order: C = s / (1 - k).
 * Monod: the positive root of C^2 + b C - s k_half = 0, b = k_half - k - s,
 * taken in the form that avoids cancellation for either sign of b. */
static double before_sink(double s, double k, double k_half)
{
    if (!(k_half > 0.0))
        return s / (1.0 - k);
    double b = k_half - k - s;
    double disc = sqrt(fmax(b * b + 4.0 * s * k_half, 0.0));
    return b >= 0.0 ? 2.0 * s * k_half / (b + disc) : (disc - b) / 2.0;
}

/* Equilibrium of Eq. 5 with c = dx/dt = 1 and W_i/rho0 = w_i (reading: the
 * printed c = dx/(dt*sqrt(3)) is the sound speed; with it the coefficients
 * 3, 9/2, 3/2 of Eq. 5 would be off by a factor of three, and Table 1's
 * tau_D/D pair fixes c_s^2 = 1/3). */
void orc_feq(int lat_id, double rho, const double *u, double *feq)
{
    orc_lattice L;
    make_lattice(lat_id, &L);
    double uu = 0.0;
    for (int d = 0; d < 3; d++)
        uu += u[d] * u[d];
    for (int i = 0; i < L.q; i++) {
        double cu = 0.0;
        for (int d = 0; d < 3; d++)
            cu += L.c[i][d] * u[d];
        feq[i] = L.w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Substrate equilibrium, linear in u: g_eq = w_i C (1 + c_i.u / c_s^2).
 * Reading: the paper's AD equilibrium is "as Eq. 5"; on the D2Q5/D3Q7
 * lattices the second-order terms have no isotropic closure, so the
 * standard linear form is used. */
/* Substrate equilibrium of direction i at concentration C and velocity u
 * (u[3]).  On the lattices with diagonal directions (D2Q9, D3Q19) it is
 * Eq. 5 with the concentration in place of the density -- the paper's
 * substrate LBM on D2Q9 (Sec. 2.1.2 computes G^(0) "as in Eq. 5"):
 * w_i C (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2).  On D2Q5 and D3Q7 it is the
 * linear w_i C (1 + c.u / c_s^2): their weights are not isotropic enough for
 * the second-order terms. */
static double ad_eq(const orc_lattice *L, int i, double C, const double *u)
{
    double cu = 0.0, uu = 0.0;
    for (int d = 0; d < 3; d++) {
        cu += L->c[i][d] * u[d];
        uu += u[d] * u[d];
    }
    if (L->q == 9 || L->q == 19)
        return L->w[i] * C * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    return L->w[i] * C * (1.0 + cu / L->cs2);
}

/* Even part of that equilibrium, (g_eq_i + g_eq_opp(i)) / 2, written out:
 * w_i C (1 + 9/2 (c.u)^2 - 3/2 u^2), or w_i C for the linear form.  Anti-
 * bounce-back imposes twice it at a Dirichlet face. */
static double ad_eq_even(const orc_lattice *L, int i, double C, const double *u)
{
    if (L->q == 9 || L->q == 19) {
        double cu = 0.0, uu = 0.0;
        for (int d = 0; d < 3; d++) {
            cu += L->c[i][d] * u[d];
            uu += u[d] * u[d];
        }
        return L->w[i] * C * (1.0 + 4.5 * cu * cu - 1.5 * uu);
    }
    return L->w[i] * C;
}

void orc_geq(int lat_id, double C, const double *u, double *geq)
{
    orc_lattice L;
    make_lattice(lat_id, &L);
    for (int i = 0; i < L.q; i++)
        geq[i] = ad_eq(&L, i, C, u);
}

/* ------------------------------------------------------------------------ */
/* Fluid solver.                                                             */

/* Cold start: rest state f_i = w_i (rho = 1, u = 0); blocked nodes hold 0. */
int orc_fluid_init(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                   double *f)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    int64_t N = (int64_t)nx * ny * nz;
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!dom)
        return ORC_EINVAL;
    for (int i = 0; i < L.q; i++)
        for (int64_t n = 0; n < N; n++)
            f[i * N + n] = dom[n] ? L.w[i] : 0.0;
    free(dom);
    return ORC_OK;
}

/* One time step of the fluid BGK LBM, pull form.
 *
 * f_src holds the stored post-collision populations f*(t) (layout [q][N]);
 * f_dst receives f*(t+1).  For every node n of the flow domain (FLUID
 * nodes linked to the outlet column, see flow_domain) and direction i, with
 * s = n - c_i the node the population comes from:
 *   (a) s left of column 0 (inlet): f_i = f*_opp(n) + 6 w_i c_ix u_in --
 *       bounce-back from a wall moving at the plug inflow speed; each inlet
 *       node gains exactly u_in of mass per step (sum of w_i over c_ix = +1
 *       is 1/6 on both fluid lattices);
 *   (b) s right of column nx-1 (outlet): anti-bounce-back pressure outlet
 *       f_i = -f*_opp(n) + 2 w_i rho_out (1 + 9/2 (c_i.u*)^2 - 3/2 u*^2),
 *       rho_out = 1, where u* is the velocity of this node's stored state
 *       f*(n): twice the symmetric (even) part of the Eq. 5 equilibrium at
 *       the outlet density.  (Dropping the u*^2 terms makes the outlet
 *       unstable: an empty 3-D duct at tau = 0.7 blows up within 1500
 *       steps.)
 *   (c) s blocked (electrode, chassis, biofilm) or outside in y/z:
 *       f_i = f*_opp(n) -- half-way bounce-back (Sec. 2.1.1, Eq. 11, read
 *       in its half-way form; the steady fixed point is the same as the
 *       on-node form);
 *   (d) otherwise f_i = f*_i(s) -- streaming, left side of Eq. 4.
 * The rules are tried in that order.  Test-only options: periodic[d]
 * wraps s along axis d instead of (a)/(b)/(c); force (Guo forcing) drives
 * the Poiseuille pin and is never used by the method.
 * Then rho = sum f_i (Eq. 9), j = sum c_i f_i (Eq. 10), u = (j + F/2)/rho,
 * and f*_i = f_i - (f_i - f_eq_i)/tau (Eq. 4) [+ Guo source].
 * If U is not NULL it receives u ([dim][N], 0 off the domain); if RHO is
 * not NULL it receives rho (0 off the domain).  Nodes off the domain store
 * 0.  (A domain node's FLUID neighbours are in the domain, so rule (c) on
 * the class is rule (c) on the domain.) */
static int fluid_step_dom(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                          const uint8_t *dom, double tau, double u_in, const int *periodic,
                          const double *force, const double *f_src, double *f_dst,
                          double *U, double *RHO)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    const int per[3] = {periodic ? periodic[0] : 0, periodic ? periodic[1] : 0,
                        periodic ? periodic[2] : 0};
    const double g[3] = {force ? force[0] : 0.0, force ? force[1] : 0.0,
                         force ? force[2] : 0.0};
    const double rho_out = 1.0;
    const int dims[3] = {nx, ny, nz};
    const int rows = ny * nz;

#pragma omp parallel for schedule(static)
    for (int row = 0; row < rows; row++) {
        int y = row % ny, z = row / ny;
        for (int x = 0; x < nx; x++) {
            int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
            if (!dom[n]) {
                for (int i = 0; i < L.q; i++)
                    f_dst[i * N + n] = 0.0;
                if (U)
                    for (int d = 0; d < L.dim; d++)
                        U[d * N + n] = 0.0;
                if (RHO)
                    RHO[n] = 0.0;
                continue;
            }
            double f[ORC_MAXQ];
            int pos[3] = {x, y, z};
            /* velocity of the stored state at this node (outlet rule only) */
            double us[3] = {0.0, 0.0, 0.0};
            if (x == nx - 1 && !per[0]) {
                double r = 0.0, jj[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < L.q; k++) {
                    double v = f_src[k * N + n];
                    r += v;
                    for (int d = 0; d < 3; d++)
                        jj[d] += L.c[k][d] * v;
                }
                for (int d = 0; d < 3; d++)
                    us[d] = jj[d] / r;
            }
            for (int i = 0; i < L.q; i++) {
                int s[3];
                int outside = 0; /* 0 inside, 1 inlet, 2 outlet, 3 other */
                for (int d = 0; d < 3; d++) {
                    s[d] = pos[d] - L.c[i][d];
                    if (per[d]) {
                        s[d] = (s[d] + dims[d]) % dims[d];
                    } else if (s[d] < 0 || s[d] >= dims[d]) {
                        if (d == 0)
                            outside = (s[d] < 0) ? 1 : 2;
                        else if (!outside)
                            outside = 3;
                    }
                }
                int o = L.opp[i];
                if (outside == 1) {
                    f[i] = f_src[o * N + n] + 6.0 * L.w[i] * L.c[i][0] * u_in;
                } else if (outside == 2) {
                    double cu = L.c[i][0] * us[0] + L.c[i][1] * us[1] + L.c[i][2] * us[2];
                    double uu = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
                    f[i] = -f_src[o * N + n] +
                           2.0 * L.w[i] * rho_out * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                } else if (outside == 3) {
                    f[i] = f_src[o * N + n];
                } else {
                    int64_t sn = s[0] + (int64_t)nx * (s[1] + (int64_t)ny * s[2]);
                    if (fluid_blocked(cls[sn]))
                        f[i] = f_src[o * N + n];
                    else
                        f[i] = f_src[i * N + sn];
                }
            }
            double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < L.q; i++) {
                rho += f[i];
                for (int d = 0; d < 3; d++)
                    j[d] += L.c[i][d] * f[i];
            }
            double u[3];
            for (int d = 0; d < 3; d++)
                u[d] = (j[d] + 0.5 * g[d]) / rho;
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            for (int i = 0; i < L.q; i++) {
                double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
                double feq = L.w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                double out = f[i] - (f[i] - feq) / tau;
                if (g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0) {
                    double cg = L.c[i][0] * g[0] + L.c[i][1] * g[1] + L.c[i][2] * g[2];
                    double ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
                    out += (1.0 - 0.5 / tau) * L.w[i] * (3.0 * (cg - ug) + 9.0 * cu * cg);
                }
                f_dst[i * N + n] = out;
            }
            if (U)
                for (int d = 0; d < L.dim; d++)
                    U[d * N + n] = u[d];
            if (RHO)
                RHO[n] = rho;
        }
    }
    return ORC_OK;
}

int orc_fluid_step(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                   double tau, double u_in, const int *periodic,
                   const double *force, const double *f_src, double *f_dst,
                   double *U, double *RHO)
{
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!dom)
        return ORC_EINVAL;
    int st = fluid_step_dom(lat_id, nx, ny, nz, cls, dom, tau, u_in, periodic, force,
                            f_src, f_dst, U, RHO);
    free(dom);
    return st;
}

/* Moments of a stored fluid state: rho = sum f*, u = (sum c f* + F/2)/rho.
 * BGK conserves rho and j, so these equal the pre-collision moments of the
 * step that produced the state.  Nodes off the flow domain get 0. */
static int fluid_moments_dom(int lat_id, int nx, int ny, int nz, const uint8_t *dom,
                             const double *force, const double *f, double *U,
                             double *RHO)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    const double g[3] = {force ? force[0] : 0.0, force ? force[1] : 0.0,
                         force ? force[2] : 0.0};
    for (int64_t n = 0; n < N; n++) {
        if (!dom[n]) {
            if (U)
                for (int d = 0; d < L.dim; d++)
                    U[d * N + n] = 0.0;
            if (RHO)
                RHO[n] = 0.0;
            continue;
        }
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L.q; i++) {
            rho += f[i * N + n];
            for (int d = 0; d < 3; d++)
                j[d] += L.c[i][d] * f[i * N + n];
        }
        if (U)
            for (int d = 0; d < L.dim; d++)
                U[d * N + n] = (j[d] + 0.5 * g[d]) / rho;
        if (RHO)
            RHO[n] = rho;
    }
    return ORC_OK;
}

int orc_fluid_moments(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                      const double *force, const double *f, double *U,
                      double *RHO)
{
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!dom)
        return ORC_EINVAL;
    int st = fluid_moments_dom(lat_id, nx, ny, nz, dom, force, f, U, RHO);
    free(dom);
    return st;
}

/* Mass crossing the inlet and outlet per step, evaluated on a stored state.
 * Inlet: sum over inlet links of (incoming - outgoing) populations.
 * Outlet: sum over outlet links of (outgoing - incoming).  Ascending n. */
int orc_fluid_fluxes(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                     double u_in, const double *f, double *flux_in,
                     double *flux_out)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    double fin = 0.0, fout = 0.0;
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!dom)
        return ORC_EINVAL;
    for (int64_t n = 0; n < N; n++) {
        if (!dom[n])
            continue;
        int x = (int)(n % nx);
        double us[3] = {0.0, 0.0, 0.0};
        if (x == nx - 1) {
            double r = 0.0, jj[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < L.q; k++) {
                r += f[k * N + n];
                for (int d = 0; d < 3; d++)
                    jj[d] += L.c[k][d] * f[k * N + n];
            }
            for (int d = 0; d < 3; d++)
                us[d] = jj[d] / r;
        }
        for (int i = 0; i < L.q; i++) {
            int o = L.opp[i];
            if (x == 0 && L.c[i][0] == 1) {
                double incoming = f[o * N + n] + 6.0 * L.w[i] * u_in;
                fin += incoming - f[o * N + n];
            }
            if (x == nx - 1 && L.c[i][0] == -1) {
                double cu = L.c[i][0] * us[0] + L.c[i][1] * us[1] + L.c[i][2] * us[2];
                double uu = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
                double incoming = -f[o * N + n] + 2.0 * L.w[i] * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                fout += f[o * N + n] - incoming;
            }
        }
    }
    free(dom);
    *flux_in = fin;
    *flux_out = fout;
    return ORC_OK;
}

/* Steady-state driver shared by both solvers' loops: residual bookkeeping.
 * Reading of running each solver to equilibrium (Sec. 3): at checks
 * t = K, 2K, ... the residual is the largest change per step over the check
 * interval, r(t) = max over active nodes and components of
 * |X(t) - X(t-K)| / (K * scale), X the moments of the stored state (X(0)
 * those of the starting state).  Stop at the first check with r <= tol (OK),
 * at t >= max_iter (NOT_CONVERGED), on NaN/Inf or |u| > 0.3 (DIVERGED), or
 * after stall_checks consecutive checks that set neither a new maximum of r
 * nor a new minimum since the last maximum (STALLED: the residual sits flat
 * on a round-off floor above tol; a transient that rises before it decays
 * is not a stall).  stall_checks <= 0 disables the stall test.  (A single-step difference is not used: dead-end pore nodes
 * keep an undamped momentum that bounce-back reverses every step, so in
 * reduced precision the one-step change never settles although the field
 * does.) */
typedef struct {
    double best; /* smallest r since the largest */
    int since_best;
    int window;
    double peak; /* largest r so far */
} orc_stall;

static int residual_decide(double r, double umax, double tol, orc_stall *st)
{
    if (isnan(r) || isinf(r) || isnan(umax) || umax > 0.3)
        return ORC_EDIVERGED;
    if (r <= tol)
        return ORC_OK;
    if (r > st->peak) {
        st->peak = r;
        st->best = r;
        st->since_best = 0;
    } else if (r < st->best) {
        st->best = r;
        st->since_best = 0;
    } else {
        st->since_best++;
        if (st->window > 0 && st->since_best >= st->window)
            return ORC_STALLED;
    }
    return -100; /* keep going */
}

/* The stop rule applied to a given sequence of check residuals r[0..n-1]
 * (and the largest |u| at each check, or NULL for none), as a solve applies
 * it check by check: returns the status of the check at which it stops and
 * its index in *stop_at, or NOT_CONVERGED with *stop_at = n when no check
 * stops it.  Exposed so that the rule can be checked on its own. */
int orc_stall_rule(const double *r, const double *umax, int n, double tol, int window,
                   int *stop_at)
{
    orc_stall st = {INFINITY, 0, window, -INFINITY};
    for (int k = 0; k < n; k++) {
        int dec = residual_decide(r[k], umax ? umax[k] : 0.0, tol, &st);
        if (dec != -100) {
            *stop_at = k;
            return dec;
        }
    }
    *stop_at = n;
    return ORC_NOT_CONVERGED;
}

/* Fluid steady solve from the state in f (cold or warm), in place.
 * On return f holds f*(t) at the stop, U the moments of that state. */
int orc_fluid_solve(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                    double tau, double u_in, double tol, int64_t max_iter,
                    int check_every, int stall_checks, double *f, double *U,
                    int64_t *iters, double *residual)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L) || check_every < 1 || max_iter < 1)
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    const int K = check_every;
    double *fb = malloc(sizeof(double) * L.q * N);
    double *Ucur = malloc(sizeof(double) * L.dim * N);
    double *Uprev = malloc(sizeof(double) * L.dim * N);
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!fb || !Ucur || !Uprev || !dom) {
        free(fb);
        free(Ucur);
        free(Uprev);
        free(dom);
        return ORC_EINVAL;
    }
    double *a = f, *b = fb;
    orc_stall st = {INFINITY, 0, stall_checks, -INFINITY};
    int status = ORC_NOT_CONVERGED;
    double r = INFINITY;
    int64_t t = 0;
    fluid_moments_dom(lat_id, nx, ny, nz, dom, NULL, f, Uprev, NULL);
    for (;;) {
        int need_u = (t + 1) % K == 0;
        fluid_step_dom(lat_id, nx, ny, nz, cls, dom, tau, u_in, NULL, NULL, a, b,
                       need_u ? Ucur : NULL, NULL);
        double *tmp = a;
        a = b;
        b = tmp;
        t++;
        if (t % K == 0) {
            double rmax = 0.0, umax = 0.0;
            int bad = 0;
            for (int64_t n = 0; n < N; n++) {
                if (!dom[n])
                    continue;
                for (int d = 0; d < L.dim; d++) {
                    double v = Ucur[d * N + n];
                    if (isnan(v) || isinf(v))
                        bad = 1;
                    double dv = fabs(v - Uprev[d * N + n]) / ((double)K * fabs(u_in));
                    if (dv > rmax)
                        rmax = dv;
                    if (fabs(v) > umax)
                        umax = fabs(v);
                }
            }
            memcpy(Uprev, Ucur, sizeof(double) * L.dim * N);
            r = bad ? NAN : rmax;
            int dec = residual_decide(r, umax, tol, &st);
            if (dec != -100) {
                status = dec;
                break;
            }
        }
        if (t >= max_iter) {
            status = ORC_NOT_CONVERGED;
            break;
        }
    }
    if (a != f)
        memcpy(f, a, sizeof(double) * L.q * N);
    fluid_moments_dom(lat_id, nx, ny, nz, dom, NULL, f, U, NULL);
    *iters = t;
    *residual = r;
    free(fb);
    free(Ucur);
    free(Uprev);
    free(dom);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Advection-diffusion (substrate) solver.                                    */

/* Cold start: g = g_eq(c_init, u) on AD-active nodes (FLUID or BIOFILM),
 * 0 elsewhere. */
int orc_ad_init(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                double c_init, const double *u, double *g)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t n = 0; n < N; n++) {
        int active = !ad_blocked(cls[n]);
        double un[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < L.dim; d++)
            un[d] = u[d * N + n];
        for (int i = 0; i < L.q; i++)
            g[i * N + n] = active ? ad_eq(&L, i, c_init, un) : 0.0;
    }
    return ORC_OK;
}

/* One step of the substrate BGK LBM (Sec. 2.1.2, Eq. 12), pull form.
 * u is the frozen fluid velocity [dim][N] (Sec. 2.1.2: constant during the
 * AD solve, taken from the fluid LBM).  For every active node n (FLUID or
 * BIOFILM) and direction i, s = n - c_i:
 *   (a) s left of column 0: g_i = -g*_opp(n) + 2 E_i(c_in, u(n)) -- anti-
 *       bounce-back, i.e. concentration c_in imposed half a cell before the
 *       first column (the Dirichlet input of Sec. 2.1.2); E_i is the even
 *       part of the equilibrium (w_i c_in on D2Q5/D3Q7);
 *   (b) s right of column nx-1: zero-gradient outlet g_i = g*_i(n)
 *       (outlet_mode 0; the paper gives no output value), or Dirichlet
 *       g_i = -g*_opp(n) + 2 E_i(c_out, u(n)) (outlet_mode 1);
 *   (c) s electrode/chassis or outside in y/z: g_i = g*_opp(n) -- zero-flux
 *       Neumann solids (Sec. 2.1.2); biofilm is not blocked for substrate;
 *   (d) otherwise g_i = g*_i(s).
 * Then C = sum g_i (Eq. 13), g_eq_i = ad_eq(i, C, u) (above), and
 * g*_i = g_i - (g_i - g_eq_i)/tau_D - w_i q, with q = consumed(C) on
 * BIOFILM nodes (k C, or k C / (C + k_half) for the Monod form) and 0
 * elsewhere: a biofilm node removes exactly q per step.  tau_D = 1/2 + D/c_s^2 (Table 1's tau_D and D
 * obey this with c_s^2 = 1/3).  If C_out is not NULL it receives C (0 on
 * inactive nodes). */
int orc_ad_step(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                double D, double c_in, double k_sink, double k_half, int outlet_mode,
                double c_out, const int *periodic, const double *u,
                const double *g_src, double *g_dst, double *C_out)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    const int per[3] = {periodic ? periodic[0] : 0, periodic ? periodic[1] : 0,
                        periodic ? periodic[2] : 0};
    const double tau_d = 0.5 + D / L.cs2;
    const int dims[3] = {nx, ny, nz};
    const int rows = ny * nz;

#pragma omp parallel for schedule(static)
    for (int row = 0; row < rows; row++) {
        int y = row % ny, z = row / ny;
        for (int x = 0; x < nx; x++) {
            int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
            if (ad_blocked(cls[n])) {
                for (int i = 0; i < L.q; i++)
                    g_dst[i * N + n] = 0.0;
                if (C_out)
                    C_out[n] = 0.0;
                continue;
            }
            double g[ORC_MAXQ];
            int pos[3] = {x, y, z};
            double un[3] = {0.0, 0.0, 0.0};
            for (int d = 0; d < L.dim; d++)
                un[d] = u[d * N + n];
            for (int i = 0; i < L.q; i++) {
                int s[3];
                int outside = 0;
                for (int d = 0; d < 3; d++) {
                    s[d] = pos[d] - L.c[i][d];
                    if (per[d]) {
                        s[d] = (s[d] + dims[d]) % dims[d];
                    } else if (s[d] < 0 || s[d] >= dims[d]) {
                        if (d == 0)
                            outside = (s[d] < 0) ? 1 : 2;
                        else if (!outside)
                            outside = 3;
                    }
                }
                int o = L.opp[i];
                if (outside == 1) {
                    g[i] = -g_src[o * N + n] + 2.0 * ad_eq_even(&L, i, c_in, un);
                } else if (outside == 2) {
                    if (outlet_mode == 1)
                        g[i] = -g_src[o * N + n] + 2.0 * ad_eq_even(&L, i, c_out, un);
                    else
                        g[i] = g_src[i * N + n];
                } else if (outside == 3) {
                    g[i] = g_src[o * N + n];
                } else {
                    int64_t sn = s[0] + (int64_t)nx * (s[1] + (int64_t)ny * s[2]);
                    if (ad_blocked(cls[sn]))
                        g[i] = g_src[o * N + n];
                    else
                        g[i] = g_src[i * N + sn];
                }
            }
            double C = 0.0;
            for (int i = 0; i < L.q; i++)
                C += g[i];
            double q = (cls[n] == ORC_BIOFILM) ? consumed(C, k_sink, k_half) : 0.0;
            for (int i = 0; i < L.q; i++) {
                double geq = ad_eq(&L, i, C, un);
                g_dst[i * N + n] = g[i] - (g[i] - geq) / tau_d - L.w[i] * q;
            }
            if (C_out)
                C_out[n] = C;
        }
    }
    return ORC_OK;
}

/* Concentration of a stored AD state: C = sum g* / (1 - k[biofilm]), which
 * is the pre-collision C of the step that produced the state. */
int orc_ad_moment(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                  double k_sink, double k_half, const double *g, double *C)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t n = 0; n < N; n++) {
        if (ad_blocked(cls[n])) {
            C[n] = 0.0;
            continue;
        }
        double s = 0.0;
        for (int i = 0; i < L.q; i++)
            s += g[i * N + n];
        C[n] = (cls[n] == ORC_BIOFILM) ? before_sink(s, k_sink, k_half) : s;
    }
    return ORC_OK;
}

/* Substrate crossing inlet and outlet per step and the total consumed by
 * the biofilm sink, on a stored state (ascending n). */
int orc_ad_fluxes(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                  double c_in, double k_sink, double k_half, int outlet_mode, double c_out,
                  const double *u, const double *g, double *flux_in, double *flux_out,
                  double *sink_total)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L))
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    double fin = 0.0, fout = 0.0, sink = 0.0;
    for (int64_t n = 0; n < N; n++) {
        if (ad_blocked(cls[n]))
            continue;
        int x = (int)(n % nx);
        double un[3] = {0.0, 0.0, 0.0};
        for (int d = 0; u && d < L.dim; d++)
            un[d] = u[d * N + n];
        for (int i = 0; i < L.q; i++) {
            int o = L.opp[i];
            if (x == 0 && L.c[i][0] == 1) {
                double incoming = -g[o * N + n] + 2.0 * ad_eq_even(&L, i, c_in, un);
                fin += incoming - g[o * N + n];
            }
            if (x == nx - 1 && L.c[i][0] == -1) {
                double incoming = (outlet_mode == 1)
                                      ? -g[o * N + n] + 2.0 * ad_eq_even(&L, i, c_out, un)
                                      : g[i * N + n];
                fout += g[o * N + n] - incoming;
            }
        }
        if (cls[n] == ORC_BIOFILM) {
            double s = 0.0;
            for (int i = 0; i < L.q; i++)
                s += g[i * N + n];
            sink += k_half > 0.0 ? consumed(before_sink(s, k_sink, k_half), k_sink, k_half)
                                 : k_sink * s / (1.0 - k_sink);
        }
    }
    *flux_in = fin;
    *flux_out = fout;
    *sink_total = sink;
    return ORC_OK;
}

/* AD steady solve from the state in g (cold or warm), in place; residual
 * r = max over active nodes of |C(t) - C(t-1)| / c_in. */
int orc_ad_solve(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                 const double *u, double D, double c_in, double k_sink, double k_half,
                 int outlet_mode, double c_out, double tol, int64_t max_iter,
                 int check_every, int stall_checks, double *g, double *C,
                 int64_t *iters, double *residual)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L) || check_every < 1 || max_iter < 1)
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    const int K = check_every;
    double *gb = malloc(sizeof(double) * L.q * N);
    double *Ccur = malloc(sizeof(double) * N);
    double *Cprev = malloc(sizeof(double) * N);
    if (!gb || !Ccur || !Cprev) {
        free(gb);
        free(Ccur);
        free(Cprev);
        return ORC_EINVAL;
    }
    double *a = g, *b = gb;
    orc_stall st = {INFINITY, 0, stall_checks, -INFINITY};
    int status = ORC_NOT_CONVERGED;
    double r = INFINITY;
    int64_t t = 0;
    orc_ad_moment(lat_id, nx, ny, nz, cls, k_sink, k_half, g, Cprev);
    for (;;) {
        int need_c = (t + 1) % K == 0;
        orc_ad_step(lat_id, nx, ny, nz, cls, D, c_in, k_sink, k_half, outlet_mode,
                    c_out, NULL, u, a, b, need_c ? Ccur : NULL);
        double *tmp = a;
        a = b;
        b = tmp;
        t++;
        if (t % K == 0) {
            double rmax = 0.0;
            int bad = 0;
            for (int64_t n = 0; n < N; n++) {
                if (ad_blocked(cls[n]))
                    continue;
                double v = Ccur[n];
                if (isnan(v) || isinf(v))
                    bad = 1;
                double dv = fabs(v - Cprev[n]) / ((double)K * fabs(c_in));
                if (dv > rmax)
                    rmax = dv;
            }
            memcpy(Cprev, Ccur, sizeof(double) * N);
            r = bad ? NAN : rmax;
            int dec = residual_decide(r, 0.0, tol, &st);
            if (dec != -100) {
                status = dec;
                break;
            }
        }
        if (t >= max_iter) {
            status = ORC_NOT_CONVERGED;
            break;
        }
    }
    if (a != g)
        memcpy(g, a, sizeof(double) * L.q * N);
    orc_ad_moment(lat_id, nx, ny, nz, cls, k_sink, k_half, g, C);
    *iters = t;
    *residual = r;
    free(gb);
    free(Ccur);
    free(Cprev);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Seeded geometry.  The paper's electrode is a randomly generated medium (Sec. 3)
 * whose figure is not available; these generators produce seeded stand-ins
 * with integer arithmetic only, so that two independent implementations
 * agree byte for byte.                                                      */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state advances by the
 * golden-ratio increment; output is the variant-13 finaliser of the state. */
typedef struct {
    uint64_t s;
} orc_rng;

static uint64_t rng_next(orc_rng *r)
{
    r->s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = r->s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* integer uniform on [lo, hi] by modulo (bias accepted by definition) */
static int64_t rng_int(orc_rng *r, int64_t lo, int64_t hi)
{
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)(rng_next(r) % span);
}

void orc_splitmix64(uint64_t seed, int64_t count, uint64_t *out)
{
    orc_rng r = {seed};
    for (int64_t k = 0; k < count; k++)
        out[k] = rng_next(&r);
}

/* Start from FLUID everywhere with WALL on the chassis rows y = 0, ny-1
 * (and planes z = 0, nz-1 in 3-D). */
static void chassis(int nx, int ny, int nz, uint8_t *cls)
{
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                int wall = (y == 0 || y == ny - 1);
                if (nz > 1)
                    wall = wall || z == 0 || z == nz - 1;
                cls[n] = wall ? ORC_WALL : ORC_FLUID;
            }
}

/* Disc electrode (2-D).  Region R = [nx/4, 3nx/4) x [1, ny-1).  Each attempt
 * draws cx in R's columns, then cy in R's rows, then r in [r_min, r_max].
 * Non-overlap mode rejects a disc whose centre distance to any accepted one
 * is <= r + r_j (strict separation keeps cell sets disjoint).  An accepted
 * disc marks the cells of R with (x-cx)^2 + (y-cy)^2 <= r^2 SOLID.  Stops
 * once the SOLID count in R reaches ceil(solid_frac * |R|); EINVAL after
 * 10^6 attempts. */
int orc_geom_discs(int nx, int ny, int r_min, int r_max, double solid_frac,
                   int overlap, uint64_t seed, uint8_t *cls, double *achieved)
{
    if (nx < 4 || ny < 3 || r_min < 0 || r_max < r_min || solid_frac < 0.0 ||
        solid_frac > 1.0)
        return ORC_EINVAL;
    chassis(nx, ny, 1, cls);
    int x0 = nx / 4, x1 = 3 * nx / 4, y0 = 1, y1 = ny - 1;
    int64_t area = (int64_t)(x1 - x0) * (y1 - y0);
    int64_t need = (int64_t)ceil(solid_frac * (double)area);
    int64_t cap = 1024, nd = 0, count = 0;
    int64_t *dx = malloc(sizeof(int64_t) * cap), *dy = malloc(sizeof(int64_t) * cap),
            *dr = malloc(sizeof(int64_t) * cap);
    orc_rng rng = {seed};
    int status = ORC_EINVAL;
    for (int64_t attempt = 0; attempt < 1000000; attempt++) {
        if (count >= need) {
            status = ORC_OK;
            break;
        }
        int64_t cx = rng_int(&rng, x0, x1 - 1);
        int64_t cy = rng_int(&rng, y0, y1 - 1);
        int64_t r = rng_int(&rng, r_min, r_max);
        if (!overlap) {
            int clash = 0;
            for (int64_t j = 0; j < nd && !clash; j++) {
                int64_t ddx = cx - dx[j], ddy = cy - dy[j], rr = r + dr[j];
                if (ddx * ddx + ddy * ddy <= rr * rr)
                    clash = 1;
            }
            if (clash)
                continue;
        }
        if (nd == cap) {
            cap *= 2;
            dx = realloc(dx, sizeof(int64_t) * cap);
            dy = realloc(dy, sizeof(int64_t) * cap);
            dr = realloc(dr, sizeof(int64_t) * cap);
        }
        dx[nd] = cx;
        dy[nd] = cy;
        dr[nd] = r;
        nd++;
        for (int64_t y = cy - r; y <= cy + r; y++)
            for (int64_t x = cx - r; x <= cx + r; x++) {
                if (x < x0 || x >= x1 || y < y0 || y >= y1)
                    continue;
                if ((x - cx) * (x - cx) + (y - cy) * (y - cy) > r * r)
                    continue;
                int64_t n = x + (int64_t)nx * y;
                if (cls[n] != ORC_SOLID) {
                    cls[n] = ORC_SOLID;
                    count++;
                }
            }
    }
    if (status != ORC_OK && count >= need)
        status = ORC_OK;
    free(dx);
    free(dy);
    free(dr);
    if (achieved)
        *achieved = (double)count / (double)area;
    return status;
}

/* Fibre electrode (3-D).  Region R = [nx/4, 3nx/4) x [1, ny-1) x [1, nz-1).
 * Each attempt draws a point q in R (x, y, z in that order), then a
 * direction d with components in [-4, 4] (redrawn as a whole while d = 0),
 * then r in [r_min, r_max].  Voxel p of R becomes SOLID iff
 * |(p - q) x d|^2 <= r^2 |d|^2 (an infinite cylinder, int64 arithmetic).
 * Overlap allowed; stops at SOLID count >= ceil(solid_frac * |R|). */
int orc_geom_fibres(int nx, int ny, int nz, int r_min, int r_max,
                    double solid_frac, uint64_t seed, uint8_t *cls,
                    double *achieved)
{
    if (nx < 4 || ny < 3 || nz < 3 || r_min < 0 || r_max < r_min ||
        solid_frac < 0.0 || solid_frac > 1.0)
        return ORC_EINVAL;
    chassis(nx, ny, nz, cls);
    int x0 = nx / 4, x1 = 3 * nx / 4;
    int64_t vol = (int64_t)(x1 - x0) * (ny - 2) * (nz - 2);
    int64_t need = (int64_t)ceil(solid_frac * (double)vol);
    int64_t count = 0;
    orc_rng rng = {seed};
    int status = ORC_EINVAL;
    for (int64_t attempt = 0; attempt < 1000000; attempt++) {
        if (count >= need) {
            status = ORC_OK;
            break;
        }
        int64_t qx = rng_int(&rng, x0, x1 - 1);
        int64_t qy = rng_int(&rng, 1, ny - 2);
        int64_t qz = rng_int(&rng, 1, nz - 2);
        int64_t ddx, ddy, ddz;
        do {
            ddx = rng_int(&rng, -4, 4);
            ddy = rng_int(&rng, -4, 4);
            ddz = rng_int(&rng, -4, 4);
        } while (ddx == 0 && ddy == 0 && ddz == 0);
        int64_t r = rng_int(&rng, r_min, r_max);
        int64_t dd = ddx * ddx + ddy * ddy + ddz * ddz;
        for (int64_t z = 1; z < nz - 1; z++)
            for (int64_t y = 1; y < ny - 1; y++)
                for (int64_t x = x0; x < x1; x++) {
                    int64_t px = x - qx, py = y - qy, pz = z - qz;
                    int64_t cx = py * ddz - pz * ddy;
                    int64_t cy = pz * ddx - px * ddz;
                    int64_t cz = px * ddy - py * ddx;
                    if (cx * cx + cy * cy + cz * cz > r * r * dd)
                        continue;
                    int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
                    if (cls[n] != ORC_SOLID) {
                        cls[n] = ORC_SOLID;
                        count++;
                    }
                }
    }
    if (status != ORC_OK && count >= need)
        status = ORC_OK;
    if (achieved)
        *achieved = (double)count / (double)vol;
    return status;
}

/* neighbour offsets of the fluid lattice (D2Q9 in 2-D, D3Q19 in 3-D) */
static const orc_lattice *nbr_lattice(int nz, orc_lattice *buf)
{
    make_lattice(nz > 1 ? ORC_D3Q19 : ORC_D2Q9, buf);
    return buf;
}

/* Biofilm layer: in one pass over the input mask, every FLUID node with a
 * SOLID lattice neighbour becomes BIOFILM (chassis walls do not seed it). */
int orc_biofilm_layer(int nx, int ny, int nz, uint8_t *cls)
{
    orc_lattice Lb;
    const orc_lattice *L = nbr_lattice(nz, &Lb);
    const int64_t N = (int64_t)nx * ny * nz;
    uint8_t *orig = malloc(N);
    memcpy(orig, cls, N);
    for (int64_t n = 0; n < N; n++) {
        if (orig[n] != ORC_FLUID)
            continue;
        int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        for (int i = 1; i < L->q; i++) {
            int sx = x + L->c[i][0], sy = y + L->c[i][1], sz = z + L->c[i][2];
            if (sx < 0 || sx >= nx || sy < 0 || sy >= ny || sz < 0 || sz >= nz)
                continue;
            if (orig[sx + (int64_t)nx * (sy + (int64_t)ny * sz)] == ORC_SOLID) {
                cls[n] = ORC_BIOFILM;
                break;
            }
        }
    }
    free(orig);
    return ORC_OK;
}

/* Link masks.  which = 0: fluid solver (D2Q9 / D3Q19, blocked = SOLID, WALL,
 * BIOFILM), written as uint16 (2-D) or uint32 (3-D) words.  which = 1:
 * substrate solver (D2Q5 / D3Q7, blocked = SOLID, WALL), uint8 words.  Bit i
 * is set iff the pull source n - c_i lies in the domain and is blocked. */
int orc_links(int nx, int ny, int nz, const uint8_t *cls, int which, void *out)
{
    orc_lattice L;
    int id = which == 0 ? (nz > 1 ? ORC_D3Q19 : ORC_D2Q9) : (nz > 1 ? ORC_D3Q7 : ORC_D2Q5);
    make_lattice(id, &L);
    const int64_t N = (int64_t)nx * ny * nz;
    for (int64_t n = 0; n < N; n++) {
        int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        uint32_t bits = 0;
        for (int i = 1; i < L.q; i++) {
            int sx = x - L.c[i][0], sy = y - L.c[i][1], sz = z - L.c[i][2];
            if (sx < 0 || sx >= nx || sy < 0 || sy >= ny || sz < 0 || sz >= nz)
                continue;
            uint8_t k = cls[sx + (int64_t)nx * (sy + (int64_t)ny * sz)];
            int blocked = which == 0 ? fluid_blocked(k) : ad_blocked(k);
            if (blocked)
                bits |= 1u << i;
        }
        if (which == 1)
            ((uint8_t *)out)[n] = (uint8_t)bits;
        else if (nz > 1)
            ((uint32_t *)out)[n] = bits;
        else
            ((uint16_t *)out)[n] = (uint16_t)bits;
    }
    return ORC_OK;
}

/* Percolation: breadth-first search over FLUID nodes along fluid-lattice
 * links; returns 1 iff some node of column 0 reaches column nx-1. */
int orc_percolates(int nx, int ny, int nz, const uint8_t *cls)
{
    orc_lattice Lb;
    const orc_lattice *L = nbr_lattice(nz, &Lb);
    const int64_t N = (int64_t)nx * ny * nz;
    uint8_t *seen = calloc(N, 1);
    int64_t *queue = malloc(sizeof(int64_t) * N);
    int64_t head = 0, tail = 0;
    for (int64_t n = 0; n < N; n++)
        if (n % nx == 0 && cls[n] == ORC_FLUID) {
            seen[n] = 1;
            queue[tail++] = n;
        }
    int found = 0;
    while (head < tail && !found) {
        int64_t n = queue[head++];
        int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        if (x == nx - 1) {
            found = 1;
            break;
        }
        for (int i = 1; i < L->q; i++) {
            int sx = x + L->c[i][0], sy = y + L->c[i][1], sz = z + L->c[i][2];
            if (sx < 0 || sx >= nx || sy < 0 || sy >= ny || sz < 0 || sz >= nz)
                continue;
            int64_t m = sx + (int64_t)nx * (sy + (int64_t)ny * sz);
            if (!seen[m] && cls[m] == ORC_FLUID) {
                seen[m] = 1;
                queue[tail++] = m;
            }
        }
    }
    free(seen);
    free(queue);
    return found;
}

/* Flow domain (reading: the boundary conditions of Sec. 2.1.1 set the flow
 * in the part of the Sec. 3 pore space that reaches the outlet).  dom[n] = 1
 * iff n is FLUID and a chain of fluid-lattice links between FLUID nodes
 * joins it to a FLUID node of column nx-1; breadth-first from that column.
 * A closed pore has no steady flow and no boundary fixes its pressure; a
 * pocket open only to the inlet would take in u_in per inlet link forever.
 * Such nodes hold no fluid populations (u = 0, rho reported 0); the
 * substrate solver still treats them as fluid.  Returns a malloc'd mask of
 * N bytes (NULL when out of memory). */
static uint8_t *flow_domain(int nx, int ny, int nz, const uint8_t *cls)
{
    orc_lattice Lb;
    const orc_lattice *L = nbr_lattice(nz, &Lb);
    const int64_t N = (int64_t)nx * ny * nz;
    uint8_t *dom = calloc(N, 1);
    int64_t *queue = malloc(sizeof(int64_t) * N);
    if (!dom || !queue) {
        free(dom);
        free(queue);
        return NULL;
    }
    int64_t head = 0, tail = 0;
    for (int64_t n = 0; n < N; n++)
        if (n % nx == nx - 1 && cls[n] == ORC_FLUID) {
            dom[n] = 1;
            queue[tail++] = n;
        }
    while (head < tail) {
        int64_t n = queue[head++];
        int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
        for (int i = 1; i < L->q; i++) {
            int sx = x + L->c[i][0], sy = y + L->c[i][1], sz = z + L->c[i][2];
            if (sx < 0 || sx >= nx || sy < 0 || sy >= ny || sz < 0 || sz >= nz)
                continue;
            int64_t m = sx + (int64_t)nx * (sy + (int64_t)ny * sz);
            if (!dom[m] && cls[m] == ORC_FLUID) {
                dom[m] = 1;
                queue[tail++] = m;
            }
        }
    }
    free(queue);
    return dom;
}

int orc_flow_domain(int nx, int ny, int nz, const uint8_t *cls, uint8_t *out)
{
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!dom)
        return ORC_EINVAL;
    memcpy(out, dom, (size_t)nx * ny * nz);
    free(dom);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Simplified biofilm growth (the coupled loop's stand-in for Sec. 2.3).    */

/* Candidates: FLUID nodes with 1 <= x <= nx-2 that have a BIOFILM lattice
 * neighbour, in ascending n.  Weight max(C, 0); W = running sum in that
 * order; the pick is the first candidate whose cumulative weight exceeds
 * xi * W (xi in [0, 1) is an input).  If W = 0 the pick is candidate
 * floor(xi * count).  If rounding leaves no candidate above xi * W, the last
 * candidate with positive weight is taken.  Returns -1 if none exist. */
int64_t orc_growth_pick(int nx, int ny, int nz, const uint8_t *cls,
                        const double *C, double xi)
{
    orc_lattice Lb;
    const orc_lattice *L = nbr_lattice(nz, &Lb);
    const int64_t N = (int64_t)nx * ny * nz;
    int64_t count = 0;
    double W = 0.0;
    for (int pass = 0; pass < 2; pass++) {
        double target = xi * W, cum = 0.0;
        int64_t idx = 0, last_pos = -1;
        for (int64_t n = 0; n < N; n++) {
            if (cls[n] != ORC_FLUID)
                continue;
            int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
            if (x < 1 || x > nx - 2)
                continue;
            int adj = 0;
            for (int i = 1; i < L->q && !adj; i++) {
                int sx = x + L->c[i][0], sy = y + L->c[i][1], sz = z + L->c[i][2];
                if (sx < 0 || sx >= nx || sy < 0 || sy >= ny || sz < 0 || sz >= nz)
                    continue;
                if (cls[sx + (int64_t)nx * (sy + (int64_t)ny * sz)] == ORC_BIOFILM)
                    adj = 1;
            }
            if (!adj)
                continue;
            double wgt = C[n] > 0.0 ? C[n] : 0.0;
            if (pass == 0) {
                count++;
                W += wgt;
            } else {
                if (W == 0.0) {
                    int64_t want = (int64_t)floor(xi * (double)count);
                    if (want >= count)
                        want = count - 1;
                    if (idx == want)
                        return n;
                } else {
                    cum += wgt;
                    if (wgt > 0.0)
                        last_pos = n;
                    if (cum > target)
                        return n;
                }
            }
            idx++;
        }
        if (pass == 1)
            return last_pos;
        if (count == 0)
            return -1;
    }
    return -1;
}

/* Coupled loop: cold fluid + substrate solves on cls, then n_updates times:
 * pick a new biofilm cell from the current C with xi[m], mark it BIOFILM
 * (its fluid populations are dropped, its substrate populations kept),
 * re-converge fluid then substrate warm from the retained states, and add
 * the substrate consumed per step by the biofilm (sink_total) to J_accum.
 * Per-update picks, sink totals and iteration counts are returned.  cls is
 * updated in place.  2-D (D2Q9 + D2Q5) and 3-D (D3Q19 + D3Q7). */
int orc_coupled_run(int nx, int ny, int nz, uint8_t *cls, double tau,
                    double u_in, double D, double c_in, double k_sink, double k_half,
                    int ad_lat, double tol, int64_t max_iter, int check_every,
                    int stall_checks, int n_updates, const double *xi, int64_t *picked,
                    double *J, double *J_accum, int64_t *iters_fluid,
                    int64_t *iters_ad, double *U_out, double *C_out)
{
    int fl = nz > 1 ? ORC_D3Q19 : ORC_D2Q9;
    int ad = ad_lat >= 0 ? ad_lat : (nz > 1 ? ORC_D3Q7 : ORC_D2Q5);
    orc_lattice Lf, La;
    make_lattice(fl, &Lf);
    make_lattice(ad, &La);
    const int64_t N = (int64_t)nx * ny * nz;
    double *f = malloc(sizeof(double) * Lf.q * N);
    double *g = malloc(sizeof(double) * La.q * N);
    double *U = malloc(sizeof(double) * Lf.dim * N);
    double *C = malloc(sizeof(double) * N);
    int64_t it;
    double res;
    int st = ORC_OK;
    double acc = 0.0;
    orc_fluid_init(fl, nx, ny, nz, cls, f);
    for (int m = 0; m <= n_updates; m++) {
        if (m > 0) {
            int64_t p = orc_growth_pick(nx, ny, nz, cls, C, xi[m - 1]);
            picked[m - 1] = p;
            if (p < 0) {
                st = ORC_EINVAL;
                break;
            }
            cls[p] = ORC_BIOFILM;
            for (int i = 0; i < Lf.q; i++)
                f[i * N + p] = 0.0;
            if (!orc_percolates(nx, ny, nz, cls)) {
                st = ORC_EINVAL;
                break;
            }
        }
        int s1 = orc_fluid_solve(fl, nx, ny, nz, cls, tau, u_in, tol, max_iter,
                                 check_every, stall_checks, f, U, &it, &res);
        iters_fluid[m] = it;
        if (s1 < 0) {
            st = s1;
            break;
        }
        if (m == 0)
            orc_ad_init(ad, nx, ny, nz, cls, c_in, U, g);
        int s2 = orc_ad_solve(ad, nx, ny, nz, cls, U, D, c_in, k_sink, k_half, 0, 0.0, tol,
                              max_iter, check_every, stall_checks, g, C, &it, &res);
        iters_ad[m] = it;
        if (s2 < 0) {
            st = s2;
            break;
        }
        double fin, fout, sink;
        orc_ad_fluxes(ad, nx, ny, nz, cls, c_in, k_sink, k_half, 0, 0.0, U, g, &fin, &fout, &sink);
        J[m] = sink;
        if (m > 0)
            acc += sink;
    }
    *J_accum = acc;
    if (U_out)
        memcpy(U_out, U, sizeof(double) * Lf.dim * N);
    if (C_out)
        memcpy(C_out, C, sizeof(double) * N);
    free(f);
    free(g);
    free(U);
    free(C);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Fixed-step drivers (no residual logic): nsteps steps from the state in   */
/* f / g, in place; U / C (if not NULL) receive the last step's moments.    */

int orc_fluid_run(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
                  double tau, double u_in, const int *periodic,
                  const double *force, int64_t nsteps, double *f, double *U,
                  double *RHO)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L) || nsteps < 0)
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    double *b = malloc(sizeof(double) * L.q * N);
    uint8_t *dom = flow_domain(nx, ny, nz, cls);
    if (!b || !dom) {
        free(b);
        free(dom);
        return ORC_EINVAL;
    }
    double *a = f;
    for (int64_t t = 0; t < nsteps; t++) {
        int last = (t == nsteps - 1);
        fluid_step_dom(lat_id, nx, ny, nz, cls, dom, tau, u_in, periodic, force, a, b,
                       last ? U : NULL, last ? RHO : NULL);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != f) {
        memcpy(f, a, sizeof(double) * L.q * N);
        b = a;
    }
    free(b);
    free(dom);
    return ORC_OK;
}

int orc_ad_run(int lat_id, int nx, int ny, int nz, const uint8_t *cls,
               double D, double c_in, double k_sink, double k_half, int outlet_mode,
               double c_out, const int *periodic, const double *u,
               int64_t nsteps, double *g, double *C)
{
    orc_lattice L;
    if (make_lattice(lat_id, &L) || nsteps < 0)
        return ORC_EINVAL;
    const int64_t N = (int64_t)nx * ny * nz;
    double *b = malloc(sizeof(double) * L.q * N);
    if (!b)
        return ORC_EINVAL;
    double *a = g;
    for (int64_t t = 0; t < nsteps; t++) {
        int last = (t == nsteps - 1);
        orc_ad_step(lat_id, nx, ny, nz, cls, D, c_in, k_sink, k_half, outlet_mode, c_out,
                    periodic, u, a, b, last ? C : NULL);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != g) {
        memcpy(g, a, sizeof(double) * L.q * N);
        b = a;
    }
    free(b);
    return ORC_OK;
}

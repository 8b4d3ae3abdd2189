// kernels.hip -- gfx950 kernels of the anode-compartment LBM path
// (Tsompanas et al., arXiv 1802.07525, Sec. 2.1).
//
// Design (bandwidth-bound; no MFMA):
//  * Structure-of-arrays populations h[i][N] in two buffers (A/B) and a pull
//    scheme: one thread owns one node, gathers its Q incoming populations
//    (streaming, Eq. 4 left side, with the boundary rules folded in), takes
//    the moments (Eqs. 9-10 / Eq. 13), relaxes towards the equilibrium
//    (Eq. 5 / Eq. 12) and writes Q values at its own index: every population
//    is read once and written once per step, all stores are coalesced.
//  * A per-node descriptor word carries the node's activity and one bounce-
//    back bit per direction, so a step reads one small word per node instead
//    of the neighbours' classes.
//  * 256-thread blocks of 64 x 4 nodes (four wave64 rows).  Blocks are
//    renumbered so that each of the eight XCDs receives a contiguous band of
//    tiles: neighbouring rows meet in the same L2.
//  * Storage policies: FP64; FP32; FP32 or FP16 holding the shifted value
//    h = f - w_i * ref.  Arithmetic is FP32 for the FP32/FP16 forms, or FP64
//    over FP32 shifted storage (S::M, the collisions' type); FP16 stores
//    round stochastically (see pop_value).
//  * Residual checks are fused into the step kernel: on a check step it takes
//    max |U(t) - U(t-K)| / K in FP64 against the moments saved at the
//    previous check (and saves the new ones), reduces it across the wave
//    with shuffles, across the block in LDS, and stores one maximum per
//    block into its own slot; a one-block decide kernel reduces the slots.
//  * Every step kernel starts by reading the control word and returns when a
//    stop has been decided, so the host may queue steps ahead of decisions.
//  * Temporal blocking: 2-D launches take two to four steps over a tile and
//    a halo staged in LDS; 3-D launches take two steps in blocks that march
//    along z with rings of first-step planes in LDS.
//  * Serving: one block per tile of the device slot table runs the same
//    per-tile code over the tiles of many 2-D requests at once, each in its
//    own phase (fluid or substrate).
#include "lbm_kernels.h"

#include <math.h>
#include <stdlib.h>

#include <type_traits>

namespace lbmk {

// ---------------------------------------------------------------- lattices
// D2Q9 of Sec. 2.1 (Eqs. 1-3, weights Eqs. 6-8); c5..c8 = NE, NW, SW, SE so
// that Eq. 11's pairs 5-7, 2-4, 6-8 are opposites.
struct D2Q9 {
    static constexpr int Q = 9, DIM = 2;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int op[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr double inv_cs2 = 3.0;
};
// Substrate lattice in 2-D: the axis directions of D2Q9.
struct D2Q5 {
    static constexpr int Q = 5, DIM = 2;
    static constexpr int cx[5] = {0, 1, 0, -1, 0};
    static constexpr int cy[5] = {0, 0, 1, 0, -1};
    static constexpr int cz[5] = {0, 0, 0, 0, 0};
    static constexpr int op[5] = {0, 3, 4, 1, 2};
    static constexpr double w[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    static constexpr double inv_cs2 = 3.0;
};
// 3-D fluid lattice: rest, six axes, twelve edge diagonals (opposite pairs).
struct D3Q19 {
    static constexpr int Q = 19, DIM = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int op[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr double inv_cs2 = 3.0;
};
// 3-D substrate lattice: rest and six axes, c_s^2 = 1/4.
struct D3Q7 {
    static constexpr int Q = 7, DIM = 3;
    static constexpr int cx[7] = {0, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[7] = {0, 0, 0, 1, -1, 0, 0};
    static constexpr int cz[7] = {0, 0, 0, 0, 0, 1, -1};
    static constexpr int op[7] = {0, 2, 1, 4, 3, 6, 5};
    static constexpr double w[7] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};
    static constexpr double inv_cs2 = 4.0;
};
// Stand-in for the fluid lattice where a substrate descriptor holds no fluid
// bits (the D2Q9 substrate's own words): its Q = 1 puts the substrate bits
// at the bottom of the word.
struct NoFluid {
    static constexpr int Q = 1;
};
// Substrate equilibrium: on a lattice with diagonal directions (D2Q9) the
// second-order form of Eq. 5 with C for rho, else the linear form.
template <class L>
constexpr bool ad_second_order = L::Q == 9 || L::Q == 19;

// ---------------------------------------------------------- storage forms
// tile_mean: the residual compares tile means instead of nodes (see
// check_residual).  colref: the shift reference is a per-column array that
// moves at checks (see lbm_kernels.h); otherwise it is the constant 1 (fluid)
// or c_ref (substrate).
struct SF64 {
    typedef double T;
    typedef double C;
    typedef double M;
    static constexpr bool shifted = false;
    static constexpr bool tile_mean = false;
    static constexpr bool colref = false;
};
struct SF32 {
    typedef float T;
    typedef float C;
    typedef float M;
    static constexpr bool shifted = false;
    static constexpr bool tile_mean = false;
    static constexpr bool colref = false;
};
struct SF32S {
    typedef float T;
    typedef float C;
    typedef float M;
    static constexpr bool shifted = true;
    static constexpr bool tile_mean = false;
    static constexpr bool colref = false;
};
// FP32 shifted state (memory, LDS, registers between steps) with FP64
// collision arithmetic: each collision widens its inputs and rounds its
// results once.
struct SF32X {
    typedef float T;
    typedef float C;
    typedef double M;
    static constexpr bool shifted = true;
    static constexpr bool tile_mean = false;
    static constexpr bool colref = false;
};
struct SF16S {
    typedef _Float16 T; // stores round stochastically (pop_value)
    typedef float C;
    typedef float M;
    static constexpr bool tile_mean = true;
    static constexpr bool colref = true; // column reference moves at checks
    static constexpr bool shifted = true;
};

// Global-memory view of a pointer.  The batched kernels take their buffer
// pointers from the slot table in memory, where the compiler cannot see that
// they address global memory; generic (flat) accesses would then need a
// 64-bit address register per access.
#define LBM_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ LBM_GLOBAL T *gmem(T *p)
{
    return (LBM_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ const LBM_GLOBAL T *gmem(const T *p)
{
    return (const LBM_GLOBAL T *)p;
}

// 1 / x: the hardware reciprocal (1 ulp) in FP32, a division in FP64
__device__ __forceinline__ float recip(float x)
{
    return __builtin_amdgcn_rcpf(x);
}
__device__ __forceinline__ double recip(double x)
{
    return 1.0 / x;
}

template <class S>
__device__ __forceinline__ typename S::C ld(const typename S::T *p)
{
    return static_cast<typename S::C>(*gmem(p));
}
template <class S>
__device__ __forceinline__ void st(typename S::T *p, typename S::C v)
{
    *p = static_cast<typename S::T>(v);
}
// Counter-based integer hash (the "lowbias32" mixer of C. Wellons) of a node
// and a step; each direction then takes the next value of a Weyl sequence
// from it (steps of 0x9E3779B9, 2^32 divided by the golden ratio), whose top
// 13 bits are the rounding addend.  Over the steps the hash makes each
// direction's addend uniform and independent; within a node the sequence
// spreads the directions' addends evenly.  (A 32-bit multiply per direction
// -- a linear congruential step -- ran at a quarter of the add's rate.)
__device__ __forceinline__ unsigned int sr_seed(unsigned int n, unsigned int t)
{
    unsigned int x = n * 0x9E3779B1u ^ t * 0xC2B2AE3Du;
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

// Stored value of a population.  FP16 storage rounds stochastically: the 13
// float mantissa bits below the FP16 mantissa get a uniform random addend
// before they are cut, so a value is rounded up with probability equal to
// its fraction of an FP16 ulp.  Near a steady state round-to-nearest would
// repeat the same error every step -- a constant source that slow modes
// amplify by their relaxation time -- while these errors average to zero.
// The addends depend only on (node, step, direction): runs are
// reproducible.  gfx950 converts with stochastic rounding in one
// instruction (v_cvt_sr_f16_f32): it adds the top 13 bits of the random
// word below the FP16 mantissa and truncates -- bit for bit the add-and-cut
// on the float's bits, checked on the device over 2^20 normal-range values
// -- and below the FP16 normal range (|v| < 2^-14) it rounds at the
// subnormal ulp, also without bias (means of 2^16 draws within sampling
// noise), where the add-and-cut followed by an ordinary conversion rounded
// to nearest.
template <class S>
__device__ __forceinline__ typename S::T pop_value(typename S::C v, unsigned int &rng)
{
    if constexpr (sizeof(typename S::T) == 2) {
        typedef _Float16 half2v __attribute__((ext_vector_type(2)));
        rng += 0x9E3779B9u;
        half2v any;
        any = __builtin_nondeterministic_value(any); // the other half is not used
        return __builtin_amdgcn_cvt_sr_f16_f32(any, v, rng, false)[0];
    } else {
        return static_cast<typename S::T>(v);
    }
}

// Streaming store for domains far larger than the last-level cache: the
// next step reads these values from HBM anyway, so they need not displace
// cached data on the way.
template <class S, bool NT>
__device__ __forceinline__ void st_pop(typename S::T *p, typename S::C v, unsigned int &rng)
{
    const typename S::T h = pop_value<S>(v, rng);
    if constexpr (NT)
        __builtin_nontemporal_store(h, gmem(p));
    else
        *gmem(p) = h;
}

// Contiguous band of tiles per XCD: hardware block b runs on XCD b mod 8.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, xcd = b & 7, k = b >> 3;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

struct NodePos {
    int x, y, z;
    bool inb;
    unsigned int n; // element indices fit 32 bits: grids hold fewer than 2^31 / 19 nodes
};

__device__ __forceinline__ NodePos tile_node(const Geo &g, int tile)
{
    NodePos p;
    const int tx = tile % g.ntx;
    const int r1 = tile / g.ntx;
    const int ty = r1 % g.nty;
    p.z = r1 / g.nty;
    p.x = tx * 64 + (threadIdx.x & 63);
    p.y = ty * 4 + (threadIdx.x >> 6);
    p.inb = (p.x < g.nx) && (p.y < g.ny);
    p.n = p.inb ? (unsigned int)(p.x + g.nx * (p.y + g.ny * p.z)) : 0u;
    return p;
}

// Max over the block of two non-negative FP64 values given as bit patterns
// (ordering of the bits equals ordering of the values; NaN sorts last):
// shuffles within each wave, LDS across the four waves, and one plain store
// per block into its own slots (*pa, *pb) -- no contended atomics; the
// decide kernel reduces the slots.  Ends with a barrier so that a block may
// call it again for its next tile.
template <int NW = 4>
__device__ __forceinline__ void block_max_commit(unsigned long long a, unsigned long long b,
                                                 unsigned long long *pa, unsigned long long *pb)
{
    __shared__ unsigned long long sa[NW], sb[NW];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long oa = __shfl_xor(a, off);
        unsigned long long ob = __shfl_xor(b, off);
        a = oa > a ? oa : a;
        b = ob > b ? ob : b;
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[wv] = a;
        sb[wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ma = sa[0], mb = sb[0];
        for (int k = 1; k < NW; ++k) {
            ma = sa[k] > ma ? sa[k] : ma;
            mb = sb[k] > mb ? sb[k] : mb;
        }
        *pa = ma;
        *pb = mb;
    }
    __syncthreads();
}

__device__ __forceinline__ unsigned long long dbits(double v)
{
    return (unsigned long long)__double_as_longlong(fabs(v));
}

// Sums over the block of four doubles (valid in thread 0), in a fixed order.
__device__ __forceinline__ void block_sum4(double &a, double &b, double &c, double &d)
{
    __shared__ double sm[4][4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
        d += __shfl_xor(d, off);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[wv][0] = a;
        sm[wv][1] = b;
        sm[wv][2] = c;
        sm[wv][3] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = ((sm[0][0] + sm[1][0]) + sm[2][0]) + sm[3][0];
        b = ((sm[0][1] + sm[1][1]) + sm[2][1]) + sm[3][1];
        c = ((sm[0][2] + sm[1][2]) + sm[2][2]) + sm[3][2];
        d = ((sm[0][3] + sm[1][3]) + sm[2][3]) + sm[3][3];
    }
    __syncthreads();
}

// Residual of one tile at a check step from the per-node changes (dx, dy,
// dz) of its active nodes: the largest change of any node, or (MEAN) the
// largest change of the tile mean over its active nodes.  The mean serves FP16 storage: stochastic rounding injects
// zero-mean noise into quantities the collisions conserve (momentum, the
// substrate), so per-node changes carry a noise floor above ordinary
// tolerances; the mean averages it out and keeps the smooth evolution.
// A thread adds its nodes' changes; result() is then called by the whole
// block (valid in thread 0 for MEAN; per thread otherwise, for the block
// maximum that block_max_commit takes).  NaN is sticky.
template <bool MEAN>
struct CheckAcc {
    double a = 0.0, b = 0.0, c = 0.0, n = 0.0; // MEAN: sums and count; else a = max
    unsigned long long ub = 0ull;               // max |u| bits (fluid)
    __device__ __forceinline__ void add(bool act, double dx, double dy, double dz)
    {
        if (!act)
            return;
        if constexpr (MEAN) {
            a += dx;
            b += dy;
            c += dz;
            n += 1.0;
        } else {
            double m = fabs(dx);
            m = (fabs(dy) > m || dy != dy) ? fabs(dy) : m;
            m = (fabs(dz) > m || dz != dz) ? fabs(dz) : m;
            m = dx != dx ? __longlong_as_double(0x7ff8000000000000ll) : m;
            a = (m > a || m != m) ? m : a;
        }
    }
    __device__ __forceinline__ double result()
    {
        if constexpr (MEAN) {
            block_sum4(a, b, c, n);
            if (threadIdx.x != 0 || n == 0.0)
                return 0.0;
            const double r = fmax(fmax(fabs(a), fabs(b)), fabs(c)) / n;
            return (a != a || b != b || c != c) ? __longlong_as_double(0x7ff8000000000000ll) : r;
        } else {
            return a;
        }
    }
};

// ------------------------------------------------------------- the sink
// Consumption of one step on a BIOFILM node that collides with C: first
// order k C, or (kh > 0) the Monod form of the consumption rate (Eq. 16)
// k C / (C + kh) -- k the rate at saturation, kh the half-saturation
// concentration (the mediator factor of the double Monod rate is in k).
template <class T>
__device__ __forceinline__ T consumption(T c, double k, double kh)
{
    return kh > 0.0 ? T(k) * c * recip(c + T(kh)) : T(k) * c;
}
__device__ __forceinline__ double consumption(double c, double k, double kh)
{
    return kh > 0.0 ? k * c / (c + kh) : k * c;
}

// The C a BIOFILM node collided with, from the sum s of the populations it
// stored, s = C - consumption(C): s / (1 - k) for first order; for the Monod
// form the root C >= 0 of C^2 + b C - s kh = 0, b = kh - k - s, in the form
// free of cancellation for either sign of b.
__device__ __forceinline__ double collided_c(double s, double k, double kh)
{
    if (!(kh > 0.0))
        return s / (1.0 - k);
    const double b = kh - k - s;
    const double disc = sqrt(fmax(b * b + 4.0 * s * kh, 0.0));
    return b >= 0.0 ? 2.0 * s * kh / (b + disc) : 0.5 * (disc - b);
}

// ------------------------------------------------------ population sources
// Where a node's incoming populations come from.  own(i) is this node's
// population i; pull(i, o, cx, cy, cz, m) is population i of the pull source
// n - c_i, or this node's opposite population o on lanes whose mask m is all
// ones (a reversed link).  Values are relative to the column reference of
// the node they are read from.

// 0, or all ones when bit i of m is set
__device__ __forceinline__ unsigned int bit_mask(unsigned int m, int i)
{
    return (unsigned int)__builtin_amdgcn_sbfe((int)m, (unsigned int)i, 1u);
}

// Populations in global memory (the node's own step).  Element indices fit
// 32 bits (grids hold fewer than 2^31 / 19 nodes), so a reversed link only
// moves the index: i N + n - off becomes o N + n by adding the uniform
// (o - i) N + off under the mask -- one load, no branches.
template <class S>
struct GlobalSrc {
    typedef typename S::C C;
    const typename S::T *__restrict__ h;
    unsigned int N, n;
    int row, plane; // node offsets of y + 1 and z + 1
    __device__ __forceinline__ void set(unsigned int node) { n = node; }
    __device__ __forceinline__ C own(int i) const { return ld<S>(h + ((unsigned int)i * N + n)); }
    __device__ __forceinline__ C pull(int i, int o, int cx, int cy, int cz, unsigned int m) const
    {
        const unsigned int off = (unsigned int)(cx + cy * row + cz * plane);
        const unsigned int a = (unsigned int)i * N - off;
        const unsigned int delta = (unsigned int)(o - i) * N + off;
        return ld<S>(h + (n + a + (m & delta)));
    }
};

// Populations through a buffer resource, where the whole array fits 32-bit
// byte offsets (storage of at most 4 bytes: always in 2-D, in 3-D below
// 2^32 / (19 * 4) nodes).  The offset is the load's only per-lane address --
// no 64-bit address arithmetic and one register per address -- and the
// hardware range check returns 0 rather than reading past the array.
// EARLY: issue each streamed load before the descriptor arrives and load the
// node's own opposite value only on reversed links (3-D single steps with
// FP32 storage: 3% faster on 256 x 128 x 128); otherwise one load from an
// address selected by the descriptor bit (the 2-D kernels and FP16 storage,
// where the extra branches cost more than the latency they hide: 11% slower
// for the 3-D FP16 step; loading both values and selecting without branches
// did not help the 2-D kernels either).
template <class S, bool EARLY = false>
struct BufSrc {
    typedef typename S::C C;
    typedef typename S::T T;
    static_assert(sizeof(T) <= 4, "byte offsets of wider storage may exceed 32 bits");
    __amdgpu_buffer_rsrc_t r;
    unsigned int N4, n4; // N and n in bytes
    int row4, plane4;    // a y step and a z step in bytes
    __device__ __forceinline__ void set(unsigned int node) { n4 = node * (unsigned int)sizeof(T); }
    __device__ __forceinline__ C at(unsigned int b) const
    {
        if constexpr (sizeof(T) == 4) {
            return static_cast<C>(__builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, b, 0, 0)));
        } else {
            return static_cast<C>(__builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, b, 0, 0)));
        }
    }
    __device__ __forceinline__ C own(int i) const { return at((unsigned int)i * N4 + n4); }
    __device__ __forceinline__ C pull(int i, int o, int cx, int cy, int cz, unsigned int m) const
    {
        const unsigned int off = (unsigned int)(cx * (int)sizeof(T) + cy * row4 + cz * plane4);
        if constexpr (EARLY) {
            // the streamed address does not depend on the descriptor (a
            // source off the array -- node 0's west neighbour -- reads 0
            // through the range check)
            C v = at(n4 + (unsigned int)i * N4 - off);
            if (m)
                v = at(n4 + (unsigned int)o * N4);
            return v;
        } else {
            const unsigned int a = (unsigned int)i * N4 - off;
            const unsigned int delta = (unsigned int)(o - i) * N4 + off;
            return at(n4 + a + (m & delta));
        }
    }
};

// Buffer resource over q N elements of storage type T (raw, 32-bit format:
// the gfx9 word-3 value)
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const T *p, unsigned int q, unsigned int N)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), (short)0,
                                             (int)(q * N * (unsigned int)sizeof(T)), 0x00020000);
}

// Source of a single-step tile: a buffer resource where the host found the
// array within 32-bit byte offsets (BUF), else plain global pointers
template <class L, class S, bool BUF>
__device__ __forceinline__ auto node_src(const void *src, const Geo &g, unsigned int n)
{
    typedef typename S::T T;
    if constexpr (BUF)
        return BufSrc<S, L::DIM == 3 && sizeof(T) == 4>{pop_rsrc(static_cast<const T *>(src), (unsigned int)L::Q,
                                                              (unsigned int)g.N),
                         (unsigned int)g.N * (unsigned int)sizeof(T), n * (unsigned int)sizeof(T),
                         g.nx * (int)sizeof(T), g.nx * g.ny * (int)sizeof(T)};
    else
        return GlobalSrc<S>{static_cast<const T *>(src), (unsigned int)g.N, n, g.nx, g.nx * g.ny};
}

// Source of the first step of a 2-D pair (global memory): through a buffer
// resource where the storage allows it
template <class S, int Q>
__device__ __forceinline__ auto pair_src(const void *src, long long N, int nx)
{
    typedef typename S::T T;
    if constexpr (sizeof(T) <= 4)
        return BufSrc<S>{pop_rsrc(static_cast<const T *>(src), (unsigned int)Q, (unsigned int)N),
                         (unsigned int)N * (unsigned int)sizeof(T), 0u, nx * (int)sizeof(T), 0};
    else
        return GlobalSrc<S>{static_cast<const T *>(src), (unsigned int)N, 0u, nx, 0};
}

// The block's copy of the first step of a pair in LDS: [q][ly][lx] over the
// tile and its one-node halo (LX x LY nodes, lx = x - x0 + 1, ly = y - y0 + 1).
// Both candidates of a link sit at fixed offsets from the node's slot, so
// both are read and the value is selected.
template <class C, int Q, int LY, int LX>
struct LdsSrc {
    const C (*v)[LY][LX];
    int lx, ly;
    __device__ __forceinline__ C own(int i) const { return v[i][ly][lx]; }
    __device__ __forceinline__ C pull(int i, int o, int cx, int cy, int, unsigned int m) const
    {
        const C a = v[i][ly - cy][lx - cx], b = v[o][ly][lx];
        return m ? b : a;
    }
};

// Directions with c_ix = s as a bit mask.
template <class L>
__host__ __device__ constexpr unsigned int xdirs(int s)
{
    unsigned int m = 0;
    for (int i = 1; i < L::Q; ++i)
        if (L::cx[i] == s)
            m |= 1u << i;
    return m;
}

template <class L, int AX>
__device__ __forceinline__ constexpr int cdir(int i)
{
    return AX == 0 ? L::cx[i] : (AX == 1 ? L::cy[i] : L::cz[i]);
}

// sum_i c_i[AX] f_i in direction order, started from its first nonzero
// term (0 + x is not x for a compiler that keeps the sign of zero).  The
// order keeps the partial sums small -- the + and - terms alternate -- which
// matters where the stored values are whole populations.
template <class L, int AX, class C>
__device__ __forceinline__ C axis_sum(const C *f)
{
    C r = C(0);
    bool h = false;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int c = cdir<L, AX>(i);
        if (c == 0)
            continue;
        r = h ? (c > 0 ? r + f[i] : r - f[i]) : (c > 0 ? f[i] : -f[i]);
        h = true;
    }
    return r;
}

// c_i . u from the nonzero components of c_i only
template <class L, class C>
__device__ __forceinline__ C cdot(int i, C ux, C uy, C uz)
{
    C r = C(0);
    bool h = false;
    const int c[3] = {L::cx[i], L::cy[i], L::cz[i]};
    const C u[3] = {ux, uy, uz};
#pragma unroll
    for (int k = 0; k < L::DIM; ++k) {
        if (c[k] == 0)
            continue;
        const C t = c[k] > 0 ? u[k] : -u[k];
        r = h ? r + t : t;
        h = true;
    }
    return r;
}

// ------------------------------------------------------------ fluid step
// Pull rules per direction i (source s = n - c_i), first match wins:
//   inlet  (x == 0, c_ix = +1):   h_i = h*_opp(n) + 6 w_i u_in
//   outlet (x == nx-1, c_ix = -1): h_i = -h*_opp(n) + 2 w_i (rho_out (1 + P_i) - shift),
//       P_i = 9/2 (c_i.u*)^2 - 3/2 u*^2 with u* the velocity of this node's
//       stored state (twice the even part of the equilibrium, rho_out = 1)
//   blocked source (descriptor bit): h_i = h*_opp(n)     (Eq. 11, half-way)
//   otherwise:                      h_i = h*_i(s)         (streaming)
// then the moments (Eqs. 9-10) and the BGK relaxation (Eq. 4) towards the
// equilibrium of Eq. 5.  Fetch(i, o, cx, cy, cz, mode) returns one incoming
// value (see the sources above).  f[] comes back relative to this column's
// reference r0; the caller moves it to the reference it stores with.
template <class L, class S, class DT, class Src>
__device__ __forceinline__ void fluid_collide(const FluidArgs &a, int x, DT d, const Src &src,
                                              typename S::C r0, typename S::C dm, typename S::C dp,
                                              typename S::C f[L::Q], typename S::C &ux,
                                              typename S::C &uy, typename S::C &uz,
                                              typename S::C &rho)
{
    typedef typename S::C C;
    typedef typename S::M M; // arithmetic: the state type, or FP64 over FP32 state
    const bool xin = x == 0, xout = x == a.g.nx - 1;
    // reversed links: blocked sources, and the links through the inlet and
    // outlet faces (their rules below start from the reversed value)
    unsigned int rev = (unsigned int)d & ((1u << L::Q) - 2u);
    rev |= xin ? xdirs<L>(1) : 0u;
    rev |= xout ? xdirs<L>(-1) : 0u;
    M h[L::Q];
    h[0] = M(src.own(0));
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int cx = L::cx[i];
        const unsigned int m = bit_mask(rev, i);
        C v = src.pull(i, L::op[i], cx, L::cy[i], L::cz[i], m);
        if constexpr (S::colref) {
            // a value streamed from column x - c_ix, re-referenced to r0
            if (cx != 0)
                v = m ? v : v + C(L::w[i]) * (cx == 1 ? dm : dp);
        }
        h[i] = M(v);
    }
    const M mr0 = M(r0);
    // boundary columns (branches: waves without such a node skip them)
    if (xin) {
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            if (L::cx[i] == 1)
                h[i] = h[i] + M(6.0 * L::w[i]) * M(a.u_in);
    }
    if (xout) {
        // u* of this node's stored state
        M o[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            o[i] = M(src.own(i));
        M r = o[0];
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            r += o[i];
        const M ir = recip(S::shifted ? mr0 + r : r);
        const M ox = axis_sum<L, 0>(o) * ir, oy = axis_sum<L, 1>(o) * ir;
        const M oz = L::DIM == 3 ? axis_sum<L, 2>(o) * ir : M(0);
        const M ousq = M(1.5) * (L::DIM == 3 ? ox * ox + oy * oy + oz * oz : ox * ox + oy * oy);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            if (L::cx[i] != -1)
                continue;
            const M cu = cdot<L>(i, ox, oy, oz);
            const M even = M(4.5) * cu * cu - ousq;
            h[i] = M(2.0 * L::w[i]) * ((S::shifted ? M(1) - mr0 : M(1)) + even) - h[i];
        }
    }
    M rs = h[0];
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
        rs += h[i];
    const M mrho = S::shifted ? mr0 + rs : rs;
    const M inv = recip(mrho);
    const M mux = axis_sum<L, 0>(h) * inv;
    const M muy = axis_sum<L, 1>(h) * inv;
    M usq = mux * mux + muy * muy;
    M muz = M(0);
    if constexpr (L::DIM == 3) {
        muz = axis_sum<L, 2>(h) * inv;
        usq += muz * muz;
    }
    usq *= M(1.5);
    rho = C(mrho);
    ux = C(mux);
    uy = C(muy);
    uz = C(muz);
    const M om = M(a.omega);
    // Eq. 5 with c = 1: w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2), minus
    // the shift w_i r0 when stored shifted (rs = rho - r0).  Opposite
    // directions share the even part E = rs + rho (9/2 (c.u)^2 - 3/2 u^2)
    // and flip the odd part O = 3 rho c.u: one pair at a time.
    const M base = rs - mrho * usq;
    {
        const M feq = M(L::w[0]) * base;
        f[0] = C(h[0] + om * (feq - h[0]));
    }
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int o = L::op[i];
        if (o < i)
            continue;
        const M cu = cdot<L>(i, mux, muy, muz);
        const M rcu = mrho * cu;
        const M even = M(L::w[i]) * (base + M(4.5) * rcu * cu);
        const M odd = M(3.0 * L::w[i]) * rcu;
        f[i] = C(h[i] + om * ((even + odd) - h[i]));
        f[o] = C(h[o] + om * ((even - odd) - h[o]));
    }
}

// column references of node x: this column (r0), the neighbours' offsets
// from it (dm: x - 1, dp: x + 1) and the reference of the written buffer (rd)
template <class S>
__device__ __forceinline__ void column_refs(const float *src, const float *dst, int x, int nx,
                                            typename S::C &r0, typename S::C &dm,
                                            typename S::C &dp, typename S::C &rd)
{
    r0 = gmem(src)[x];
    dm = (x > 0 ? gmem(src)[x - 1] : r0) - r0;
    dp = (x < nx - 1 ? gmem(src)[x + 1] : r0) - r0;
    rd = gmem(dst)[x];
}

// Final part of a fluid step at one node: store (every in-grid lane, with
// zeros on blocked nodes: whole-wave stores write whole cache lines where
// lanes masked off by the geometry would turn stores into partial-line
// writes) and, on check steps, the residual and the reference sample.
template <class L, class S, bool NT>
__device__ __forceinline__ void fluid_store(const FluidArgs &a, const NodePos &p,
                                            typename S::C f[L::Q], unsigned int step)
{
    const long long N = a.g.N;
    typename S::T *__restrict__ dst = static_cast<typename S::T *>(a.dst);
    if (p.inb) {
        unsigned int rng = sizeof(typename S::T) == 2 ? sr_seed((unsigned int)p.n, step) : 0u;
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            st_pop<S, NT>(dst + ((unsigned int)i * (unsigned int)N + (unsigned int)p.n), f[i], rng);
    }
}

// Check-step work of one node: its change since the previous check into
// acc, the new moments into uprev, and the column reference sample.
template <class L, class S, class DT>
__device__ __forceinline__ void fluid_check(const FluidArgs &a, const NodePos &p, DT d, bool act,
                                            typename S::C ux, typename S::C uy, typename S::C uz,
                                            typename S::C rho, CheckAcc<S::tile_mean> &acc)
{
    typedef typename S::C C;
    if (!act)
        return;
    const long long N = a.g.N;
    LBM_GLOBAL C *up = gmem(static_cast<C *>(a.uprev));
    const double dx = (double)ux - (double)up[p.n];
    const double dy = (double)uy - (double)up[N + p.n];
    double dz = 0.0;
    double um = fmax(fabs((double)ux), fabs((double)uy));
    if (L::DIM == 3) {
        dz = (double)uz - (double)up[2 * N + p.n];
        um = fmax(um, fabs((double)uz));
    }
    if (ux != ux || uy != uy || uz != uz)
        um = __longlong_as_double(0x7ff8000000000000ll);
    const unsigned long long ubn = dbits(um);
    acc.ub = ubn > acc.ub ? ubn : acc.ub;
    up[p.n] = ux;
    up[N + p.n] = uy;
    if (L::DIM == 3)
        up[2 * N + p.n] = uz;
    if constexpr (S::colref) {
        constexpr int REF = L::Q + (L::DIM == 3 ? 7 : 5) + 1;
        if ((d >> REF) & DT(1))
            gmem(a.ref_out)[p.x] = rho;
    }
    acc.add(true, dx, dy, dz);
}

template <class L, class S, class DT, int MODE, bool NT>
__device__ __forceinline__ void fluid_finish(const FluidArgs &a, const NodePos &p, DT d, bool act,
                                             typename S::C f[L::Q], typename S::C ux,
                                             typename S::C uy, typename S::C uz,
                                             typename S::C rho, unsigned int step,
                                             unsigned long long *part_r, unsigned long long *part_u)
{
    fluid_store<L, S, NT>(a, p, f, step);
    if constexpr (MODE == MODE_CHECK) {
        CheckAcc<S::tile_mean> acc;
        fluid_check<L, S, DT>(a, p, d, act, ux, uy, uz, rho, acc);
        const double r = acc.result();
        block_max_commit(dbits(r * a.inv_uin), acc.ub, part_r, part_u);
    }
}

template <class L, class S, class DT, int MODE, bool NT, bool BUF>
__device__ __forceinline__ void fluid_tile(const FluidArgs &a, const NodePos &p,
                                           unsigned long long *part_r, unsigned long long *part_u)
{
    typedef typename S::C C;
    const DT d = p.inb ? static_cast<const DT *>(a.desc)[p.n] : DT(0);
    const bool act = (d & DT(1)) != 0;
    C ux = C(0), uy = C(0), uz = C(0), rho = C(0);
    C f[L::Q];
    C r0 = C(1), dm = C(0), dp = C(0), rd = C(1);
    if constexpr (S::colref) {
        if (act)
            column_refs<S>(a.ref_src, a.ref_dst, p.x, a.g.nx, r0, dm, dp, rd);
    }
    if (act) {
        const auto src = node_src<L, S, BUF>(a.src, a.g, p.n);
        fluid_collide<L, S, DT>(a, p.x, d, src, r0, dm, dp, f, ux, uy, uz, rho);
        if constexpr (S::colref) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                f[i] += C(L::w[i]) * (r0 - rd); // to the written buffer's reference
        }
    } else {
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            f[i] = C(0);
    }
    fluid_finish<L, S, DT, MODE, NT>(a, p, d, act, f, ux, uy, uz, rho, a.step, part_r, part_u);
}

// Tile height of the two-step kernels (2-D): 64 x PAIR_TY nodes per
// 256-thread block, one node per thread in the second step.  Four rows: the
// first step recomputes 1.55x the tile (66 x 6 nodes) against 1.29x for
// eight rows, but 256-thread blocks of eight rows (two nodes per thread)
// leave a CU half the waves -- 19% slower on a 512 x 256 grid, 2% on
// 1024 x 512 -- and the FP16 residual's tile means are the single-step
// kernels' 64 x 4 tiles.  Large grids without tile means take the wide
// form: 64 x 16 tiles on 1024-thread blocks, still one node per thread and
// full occupancy (two blocks, 32 waves per CU), and a first step of 19
// waves for 16 rows instead of 4 x 7 = 28 (the last wave of each pass is
// partly filled).  On 1024 x 512 the paired fluid launch went 10.23 ->
// 9.90 us with 64 x 8 on 512 threads, and to 9.57 us with 64 x 16.
constexpr int PAIR_TY = 4;
constexpr int WIDE_TY = 16, WIDE_NTH = 1024;
// blocks of the wide form needed to use it: two per CU
constexpr int WIDE_MIN_TILES = 512;
// middle form for grids of 256-511 tiles of 64 x 8 (e.g. 512 x 256): 64 x 8
// tiles on 512-thread blocks, the same 8 waves per CU as 64 x 4 there
constexpr int MID_TY = 8, MID_NTH = 512;
constexpr int MID_MIN_TILES = 256;
// most steps per launch of the multi-step form (wide tiles, FP32 forms)
constexpr int MULTI_NS = 4;

// Two fluid steps of one 64 x TY tile (2-D): the first over the tile and its
// one-node halo (66 x (TY + 2), the halo computed redundantly -- the same
// code on the same inputs as in its own tile) into LDS in the compute type,
// the second from LDS; only the second is stored.  With FP64/FP32 storage
// this equals two single steps (up to multiply-add contraction); FP16
// storage skips the intermediate rounding.  Step counter: a.step and
// a.step + 1; check (MODE_CHECK) on the second.
// LDS bytes of the two-step tile functions (their first-step copies)
template <class C, int Q, int TY = PAIR_TY>
constexpr int pair_lds_bytes()
{
    return Q * (TY + 2) * 66 * (int)sizeof(C);
}

template <class S, int MODE, bool NT, int TY = PAIR_TY, int NTH = 256>
__device__ __forceinline__ void fluid_tile2(const FluidArgs &a, int tile,
                                            unsigned long long *part_r, unsigned long long *part_u,
                                            void *smem)
{
    static_assert(NTH % 64 == 0 && (64 * TY) % NTH == 0, "whole rows per thread pass");
    static_assert(!S::tile_mean || (TY == 4 && NTH == 256), "tile means are over 64 x 4 tiles");
    typedef D2Q9 L;
    typedef uint16_t DT;
    typedef typename S::C C;
    constexpr int LX = 66, LY = TY + 2, NR = LX * LY;
    C(*v)[LY][LX] = reinterpret_cast<C(*)[LY][LX]>(smem);
    const long long N = a.g.N;
    const int nx = a.g.nx, ny = a.g.ny;
    const int x0 = (tile % a.g.ntx) * 64, y0 = (tile / a.g.ntx) * TY;
    const LBM_GLOBAL DT *desc = gmem(static_cast<const DT *>(a.desc));
    const auto gsrc = pair_src<S, L::Q>(a.src, N, nx);
    for (int r = threadIdx.x; r < NR; r += NTH) {
        const int lx = r % LX, ly = r / LX;
        const int x = x0 - 1 + lx, y = y0 - 1 + ly;
        const bool inb = x >= 0 && x < nx && y >= 0 && y < ny;
        const unsigned int n = inb ? (unsigned int)(x + nx * y) : 0u;
        const DT d = inb ? desc[n] : DT(0);
        C f[L::Q];
        if (d & DT(1)) {
            C r0 = C(1), dm = C(0), dp = C(0), rd = C(1), ux, uy, uz, rho;
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_src, x, nx, r0, dm, dp, rd);
            auto src = gsrc;
            src.set(n);
            fluid_collide<L, S, DT>(a, x, d, src, r0, dm, dp, f, ux, uy, uz, rho);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                v[i][ly][lx] = f[i];
        }
        // inactive nodes leave their slots unwritten: the second step reads
        // a slot only as one of a link's two candidates, and selects the
        // other one whenever the slot's node is blocked
    }
    __syncthreads();
    CheckAcc<S::tile_mean> acc;
#pragma unroll
    for (int k = 0; k < 64 * TY / NTH; ++k) {
        const int lx = threadIdx.x & 63, ly = (threadIdx.x >> 6) + (NTH / 64) * k;
        NodePos p;
        p.x = x0 + lx;
        p.y = y0 + ly;
        p.z = 0;
        p.inb = p.x < nx && p.y < ny;
        p.n = p.inb ? (unsigned int)(p.x + nx * p.y) : 0u;
        const DT d = p.inb ? desc[p.n] : DT(0);
        const bool act = (d & DT(1)) != 0;
        C ux = C(0), uy = C(0), uz = C(0), rho = C(0);
        C f[L::Q];
        if (act) {
            C r0 = C(1), dm = C(0), dp = C(0), rd = C(1);
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_dst, p.x, nx, r0, dm, dp, rd);
            const LdsSrc<C, L::Q, LY, LX> src{v, lx + 1, ly + 1};
            fluid_collide<L, S, DT>(a, p.x, d, src, r0, dm, dp, f, ux, uy, uz, rho);
            if constexpr (S::colref) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    f[i] += C(L::w[i]) * (r0 - rd);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                f[i] = C(0);
        }
        fluid_store<L, S, NT>(a, p, f, a.step + 1);
        if constexpr (MODE == MODE_CHECK)
            fluid_check<L, S, DT>(a, p, d, act, ux, uy, uz, rho, acc);
    }
    if constexpr (MODE == MODE_CHECK) {
        const double r = acc.result();
        block_max_commit<NTH / 64>(dbits(r * a.inv_uin), acc.ub, part_r, part_u);
    }
    __syncthreads(); // the block may run another tile: v is reused
}

// Source of an intermediate step updated in place in LDS: the values a node
// streams from its neighbours were read into registers (nb[i - 1]) before
// the block's barrier, since the neighbours overwrite their slots after it;
// the node's own slot is written only by its own thread, so its own values
// are read when needed.
template <class C, int LY, int LX>
struct StagedSrc {
    const C (*v)[LY][LX];
    int lx, ly;
    const C *nb;
    __device__ __forceinline__ C own(int i) const { return v[i][ly][lx]; }
    __device__ __forceinline__ C pull(int i, int o, int, int, int, unsigned int m) const
    {
        const C b = v[o][ly][lx];
        return m ? b : nb[i - 1];
    }
};

// LDS bytes of the NS-step tile: one population buffer over the tile and an
// (NS - 1)-node halo, updated in place, and the region's descriptor words
template <class C, int TY, int NS>
constexpr int multi_lds_bytes()
{
    return 9 * (TY + 2 * (NS - 1)) * (64 + 2 * (NS - 1)) * (int)sizeof(C) +
           (TY + 2 * (NS - 1)) * (64 + 2 * (NS - 1)) * 2;
}

// NS fluid steps of one 64 x TY tile (2-D), NS >= 3: the first over the
// tile and an (NS - 1)-node halo from global memory into LDS, the
// intermediate ones in place in LDS over a region one node narrower each
// step (the streamed values staged in registers across a barrier), the last
// over the tile from LDS, stored.  The same per-node code as the paired
// kernel, so the states equal NS single steps up to rounding order; a check
// (MODE_CHECK) is taken on the last step.  Compute types of 4 bytes: the
// staged values of two nodes per thread stay within the register budget of
// full occupancy.
//
// Storage that rounds on store (FP16: stochastic rounding, moving column
// references) takes NS = 4 as two paired launches fused: the second step
// ends as the paired kernel's store would -- the move to the written
// buffer's references and the rounding with that store's (node, step)
// draws -- in LDS, so the states equal those of the paired kernel bit for
// bit.  Such a launch is never the first after a check (source and
// destination references are the same) and never a check (tile means are
// taken over 64 x 4 tiles by the paired kernel).
template <class S>
constexpr bool rounds_on_store()
{
    return sizeof(typename S::T) != sizeof(typename S::C) || S::colref;
}

// Origin of 2-D tile t of 64 x TY nodes in the multi-step launches: tiles
// are numbered row by row within vertical strips of 16 tile columns, so the
// tiles one XCD works through (a contiguous range of t) keep a tile row's
// data small enough to stay in that XCD's L2 until the row below reads its
// halo (whole-width rows outgrew L2 on wide grids, and every tile read its
// halo rows from memory again).  The numbering only orders the work.
template <int TY>
__device__ __forceinline__ void strip_origin(const Geo &g, int t, int &x0, int &y0)
{
    constexpr int SW = 16;
    const int nty = (g.ny + TY - 1) / TY;
    const int per = SW * nty;
    const int s = t / per, l = t - s * per;
    const int w = min(SW, g.ntx - s * SW);
    x0 = (s * SW + l % w) * 64;
    y0 = (l / w) * TY;
}

template <class S, int MODE, bool NT, int TY, int NTH, int NS>
__device__ __forceinline__ void fluid_tileN(const FluidArgs &a, int tile, unsigned long long *part_r,
                                            unsigned long long *part_u, void *smem)
{
    typedef D2Q9 L;
    typedef uint16_t DT;
    typedef typename S::C C;
    constexpr bool EMU = rounds_on_store<S>();
    static_assert(NS >= 3 && sizeof(C) == 4 && (MODE == MODE_PLAIN || !S::tile_mean), "4-byte compute, no tile means");
    static_assert(!EMU || NS % 2 == 0, "rounding storage: whole paired launches");
    constexpr int H = NS - 1, LX = 64 + 2 * H, LY = TY + 2 * H, NR = LX * LY;
    static_assert(NTH == 64 * TY && (LX - 2) * (LY - 2) <= 2 * NTH, "two staged nodes per thread");
    C(*v)[LY][LX] = reinterpret_cast<C(*)[LY][LX]>(smem);
    DT(*dl)[LX] = reinterpret_cast<DT(*)[LX]>(static_cast<char *>(smem) + 9 * NR * sizeof(C));
    const long long N = a.g.N;
    const int nx = a.g.nx, ny = a.g.ny;
    int x0, y0;
    strip_origin<TY>(a.g, tile, x0, y0);
    const LBM_GLOBAL DT *desc = gmem(static_cast<const DT *>(a.desc));
    const auto gsrc = pair_src<S, L::Q>(a.src, N, nx);
    // step 1: the whole region from global memory
    for (int r = threadIdx.x; r < NR; r += NTH) {
        const int lx = r % LX, ly = r / LX;
        const int x = x0 - H + lx, y = y0 - H + ly;
        const bool inb = x >= 0 && x < nx && y >= 0 && y < ny;
        const unsigned int n = inb ? (unsigned int)(x + nx * y) : 0u;
        const DT d = inb ? desc[n] : DT(0);
        dl[ly][lx] = d;
        if (d & DT(1)) {
            C f[L::Q], ux, uy, uz, rho;
            C r0 = C(1), dm = C(0), dp = C(0), rd = C(1);
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_src, x, nx, r0, dm, dp, rd);
            auto src = gsrc;
            src.set(n);
            fluid_collide<L, S, DT>(a, x, d, src, r0, dm, dp, f, ux, uy, uz, rho);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                v[i][ly][lx] = f[i];
        }
    }
    __syncthreads();
    // intermediate steps: region [k - 1, LX - k] x [k - 1, LY - k], in place
#pragma unroll
    for (int k = 2; k < NS; ++k) {
        const int lo = k - 1, RW = LX - 2 * lo, RN = RW * (LY - 2 * lo);
        C nb[2][L::Q - 1];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = threadIdx.x + q * NTH;
            if (r < RN) {
                const int lx = lo + r % RW, ly = lo + r / RW;
                if (dl[ly][lx] & DT(1)) {
#pragma unroll
                    for (int i = 1; i < L::Q; ++i)
                        nb[q][i - 1] = v[i][ly - L::cy[i]][lx - L::cx[i]];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = threadIdx.x + q * NTH;
            if (r < RN) {
                const int lx = lo + r % RW, ly = lo + r / RW;
                const DT d = dl[ly][lx];
                if (d & DT(1)) {
                    C f[L::Q], ux, uy, uz, rho;
                    const int x = x0 - H + lx;
                    // step k ends a paired launch when k is even
                    const bool st_pt = EMU && (k % 2 == 0);
                    C r0 = C(1), dm = C(0), dp = C(0), rd = C(1);
                    if constexpr (S::colref)
                        column_refs<S>(a.ref_src, st_pt ? a.ref_dst : a.ref_src, x, nx, r0, dm, dp, rd);
                    const StagedSrc<C, LY, LX> src{v, lx, ly, nb[q]};
                    fluid_collide<L, S, DT>(a, x, d, src, r0, dm, dp, f, ux, uy, uz, rho);
                    if constexpr (EMU) {
                        if (st_pt) {
                            if constexpr (S::colref) {
#pragma unroll
                                for (int i = 0; i < L::Q; ++i)
                                    f[i] += C(L::w[i]) * (r0 - rd);
                            }
                            unsigned int rng = sr_seed((unsigned int)(x + nx * (y0 - H + ly)), a.step + k - 1);
#pragma unroll
                            for (int i = 0; i < L::Q; ++i)
                                f[i] = static_cast<C>(pop_value<S>(f[i], rng));
                        }
                    }
#pragma unroll
                    for (int i = 0; i < L::Q; ++i)
                        v[i][ly][lx] = f[i];
                }
            }
        }
        __syncthreads();
    }
    // last step: the tile, one node per thread, stored
    CheckAcc<false> acc;
    {
        const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
        NodePos p;
        p.x = x0 + lx;
        p.y = y0 + ly;
        p.z = 0;
        p.inb = p.x < nx && p.y < ny;
        p.n = p.inb ? (unsigned int)(p.x + nx * p.y) : 0u;
        const DT d = p.inb ? dl[ly + H][lx + H] : DT(0);
        const bool act = (d & DT(1)) != 0;
        C ux = C(0), uy = C(0), uz = C(0), rho = C(0);
        C f[L::Q];
        if (act) {
            C r0 = C(1), dm = C(0), dp = C(0), rd = C(1);
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_dst, p.x, nx, r0, dm, dp, rd);
            const LdsSrc<C, L::Q, LY, LX> src{v, lx + H, ly + H};
            fluid_collide<L, S, DT>(a, p.x, d, src, r0, dm, dp, f, ux, uy, uz, rho);
            if constexpr (S::colref) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    f[i] += C(L::w[i]) * (r0 - rd);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                f[i] = C(0);
        }
        fluid_store<L, S, NT>(a, p, f, a.step + NS - 1);
        if constexpr (MODE == MODE_CHECK)
            fluid_check<L, S, DT>(a, p, d, act, ux, uy, uz, rho, acc);
    }
    if constexpr (MODE == MODE_CHECK) {
        const double r = acc.result();
        block_max_commit<NTH / 64>(dbits(r * a.inv_uin), acc.ub, part_r, part_u);
    }
}

template <class S, int MODE, bool NT, int TY, int NTH, int NS>
__global__ void __launch_bounds__(NTH) k_fluid_stepN(FluidArgs a)
{
    __shared__ __align__(16) char smem[multi_lds_bytes<typename S::C, TY, NS>()];
    if (a.ctrl->stop)
        return;
    unsigned long long *part = a.ctrl->part;
    fluid_tileN<S, MODE, NT, TY, NTH, NS>(a, xcd_tile(blockIdx.x, gridDim.x), part + blockIdx.x,
                                          part + gridDim.x + blockIdx.x, smem);
}

template <class L, class S, class DT, int MODE, bool NT, bool BUF>
__global__ void __launch_bounds__(256) k_fluid_step(FluidArgs a)
{
    if (a.ctrl->stop)
        return;
    const NodePos p = tile_node(a.g, xcd_tile(blockIdx.x, gridDim.x));
    unsigned long long *part = a.ctrl->part;
    fluid_tile<L, S, DT, MODE, NT, BUF>(a, p, part + blockIdx.x, part + gridDim.x + blockIdx.x);
}

// -------------------------------------------------------- substrate step
// Pull rules (source s = n - c_i):
//   inlet  (x == 0, c_ix = +1):    h_i = -h*_opp(n) + 2 w_i (c_in - ref)
//   outlet (x == nx-1, c_ix = -1): zero gradient h_i = h*_i(n), or
//                                  Dirichlet h_i = -h*_opp(n) + 2 w_i (c_out - ref)
//   blocked source (SOLID/WALL):   h_i = h*_opp(n)       (zero flux)
//   otherwise:                     h_i = h*_i(s)
// Collision (Eq. 12) with the linear equilibrium w_i C (1 + c_i.u / c_s^2)
// and the biofilm consumption - w_i k C.  g[] comes back relative to r0.
template <class L, int QF, class S, class DT, class Src>
__device__ __forceinline__ void ad_collide(const AdArgs &a, int x, DT d, const Src &src,
                                           typename S::C ux_c, typename S::C uy_c, typename S::C uz_c,
                                           typename S::C r0, typename S::C dm, typename S::C dp,
                                           typename S::C g[L::Q], typename S::C &cfull)
{
    typedef typename S::C C;
    typedef typename S::M M; // arithmetic: the state type, or FP64 over FP32 state
    constexpr int BIO = QF + L::Q;
    constexpr int LNK = QF - 1;
    const bool xin = x == 0, xout = x == a.g.nx - 1;
    const M ux = M(ux_c), uy = M(uy_c), uz = M(uz_c);
    // Dirichlet values relative to this column's reference
    const M cin_s = M(C(a.c_in - (double)r0)), cout_s = M(C(a.c_out - (double)r0));
    // reversed links: blocked sources and the inlet and outlet faces (the
    // zero-gradient outlet replaces its value below)
    unsigned int rev = ((unsigned int)d >> LNK) & ((1u << L::Q) - 2u);
    rev |= xin ? xdirs<L>(1) : 0u;
    rev |= xout ? xdirs<L>(-1) : 0u;
    M h[L::Q];
    h[0] = M(src.own(0));
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int cx = L::cx[i];
        const unsigned int m = bit_mask(rev, i);
        C v = src.pull(i, L::op[i], cx, L::cy[i], L::cz[i], m);
        if constexpr (S::colref) {
            if (cx != 0)
                v = m ? v : v + C(L::w[i]) * (cx == 1 ? dm : dp);
        }
        h[i] = M(v);
    }
    // second-order form: 9/2 (c.u)^2 - 3/2 u^2 of direction i
    M usq = M(0);
    if constexpr (ad_second_order<L>)
        usq = M(1.5) * (L::DIM == 3 ? ux * ux + uy * uy + uz * uz : ux * ux + uy * uy);
    auto quad = [&](int i) {
        const M cu = cdot<L>(i, ux, uy, uz);
        return M(4.5) * cu * cu - usq;
    };
    // Dirichlet links of the boundary columns (branches: waves without such
    // a node skip them): twice the even part of the equilibrium at the
    // boundary value, w_i c (1 + 9/2 (c.u)^2 - 3/2 u^2) in the second-order
    // form, minus the reversed population
    if (xin) {
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            if (L::cx[i] == 1) {
                M e = S::colref ? M(2.0 * L::w[i]) * cin_s : M(2.0 * L::w[i] * a.cin_s);
                if constexpr (ad_second_order<L>)
                    e += M(2.0 * L::w[i] * a.c_in) * quad(i);
                h[i] = e - h[i];
            }
    }
    if (xout) {
#pragma unroll
        for (int i = 1; i < L::Q; ++i)
            if (L::cx[i] == -1) {
                if (a.outlet) {
                    M e = S::colref ? M(2.0 * L::w[i]) * cout_s : M(2.0 * L::w[i] * a.cout_s);
                    if constexpr (ad_second_order<L>)
                        e += M(2.0 * L::w[i] * a.c_out) * quad(i);
                    h[i] = e - h[i];
                } else {
                    h[i] = M(src.own(i)); // zero gradient: copy this node's population i
                }
            }
    }
    M cs = h[0];
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
        cs += h[i];
    const M mc = S::shifted ? M(r0) + cs : cs;
    cfull = C(mc);
    const M om = M(a.omega);
    const M kc = ((d >> BIO) & DT(1)) ? consumption(mc, a.k_sink, a.k_half) : M(0);
    {
        const M geq = M(L::w[0]) * cs;
        h[0] = h[0] + om * (geq - h[0]) - M(L::w[0]) * kc;
    }
    if constexpr (ad_second_order<L>) {
        // Eq. 5 with C for rho, minus the shift: w_i (cs + C (3 c.u +
        // 9/2 (c.u)^2 - 3/2 u^2)); the rest direction carries -3/2 u^2
        h[0] = h[0] - om * M(L::w[0]) * mc * usq;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const M cu = cdot<L>(i, ux, uy, uz);
            const M geq = M(L::w[i]) * (cs + mc * (M(3) * cu + (M(4.5) * cu * cu - usq)));
            h[i] = h[i] + om * (geq - h[i]) - M(L::w[i]) * kc;
        }
    } else {
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const M cu = cdot<L>(i, ux, uy, uz);
            const M geq = M(L::w[i]) * (cs + mc * (M(L::inv_cs2) * cu));
            h[i] = h[i] + om * (geq - h[i]) - M(L::w[i]) * kc;
        }
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        g[i] = C(h[i]);
}

template <class L, class S, bool NT>
__device__ __forceinline__ void ad_store(const AdArgs &a, const NodePos &p, typename S::C g[L::Q],
                                         unsigned int step)
{
    const long long N = a.g.N;
    typename S::T *__restrict__ dst = static_cast<typename S::T *>(a.dst);
    // whole-wave stores (blocked nodes store 0): see fluid_store
    if (p.inb) {
        unsigned int rng =
            sizeof(typename S::T) == 2 ? sr_seed((unsigned int)p.n, step ^ 0x5bd1e995u) : 0u;
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            st_pop<S, NT>(dst + ((unsigned int)i * (unsigned int)N + (unsigned int)p.n), g[i], rng);
    }
}

template <class L, int QF, class S, class DT>
__device__ __forceinline__ void ad_check(const AdArgs &a, const NodePos &p, DT d, bool act,
                                         typename S::C cfull, CheckAcc<S::tile_mean> &acc)
{
    typedef typename S::C C;
    constexpr int BIO = QF + L::Q;
    if (!act)
        return;
    LBM_GLOBAL C *cp = gmem(static_cast<C *>(a.cprev));
    const double dc = (double)cfull - (double)cp[p.n];
    cp[p.n] = cfull;
    if constexpr (S::colref) {
        if ((d >> (BIO + 1)) & DT(1))
            gmem(a.ref_out)[p.x] = cfull;
    }
    acc.add(true, dc, 0.0, 0.0);
}

template <class L, int QF, class S, class DT, int MODE, bool NT>
__device__ __forceinline__ void ad_finish(const AdArgs &a, const NodePos &p, DT d, bool act,
                                          typename S::C g[L::Q], typename S::C cfull,
                                          unsigned int step, unsigned long long *part_r,
                                          unsigned long long *part_u)
{
    ad_store<L, S, NT>(a, p, g, step);
    if constexpr (MODE == MODE_CHECK) {
        CheckAcc<S::tile_mean> acc;
        ad_check<L, QF, S, DT>(a, p, d, act, cfull, acc);
        const double r = acc.result();
        block_max_commit(dbits(r * a.inv_cin), 0ull, part_r, part_u);
    }
}

template <class L, int QF, class S, class DT, int MODE, bool NT, bool BUF>
__device__ __forceinline__ void ad_tile(const AdArgs &a, const NodePos &p,
                                        unsigned long long *part_r, unsigned long long *part_u)
{
    typedef typename S::C C;
    constexpr int ACT = QF - 1 + L::Q;
    const long long N = a.g.N;
    const DT d = p.inb ? static_cast<const DT *>(a.desc)[p.n] : DT(0);
    const bool act = ((d >> ACT) & DT(1)) != 0;
    C cfull = C(0);
    C g[L::Q];
    C r0 = C(a.c_ref), dm = C(0), dp = C(0), rd = r0;
    if constexpr (S::colref) {
        if (act)
            column_refs<S>(a.ref_src, a.ref_dst, p.x, a.g.nx, r0, dm, dp, rd);
    }
    if (act) {
        const auto src = node_src<L, S, BUF>(a.src, a.g, p.n);
        const C *U = static_cast<const C *>(a.u);
        const unsigned int NN = (unsigned int)N;
        const C ux = U[p.n], uy = U[NN + p.n];
        const C uz = (L::DIM == 3) ? U[2u * NN + p.n] : C(0);
        ad_collide<L, QF, S, DT>(a, p.x, d, src, ux, uy, uz, r0, dm, dp, g, cfull);
        if constexpr (S::colref) {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                g[i] += C(L::w[i]) * (r0 - rd);
        }
    } else {
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            g[i] = C(0);
    }
    ad_finish<L, QF, S, DT, MODE, NT>(a, p, d, act, g, cfull, a.step, part_r, part_u);
}

// Two substrate steps of one 64 x TY tile (2-D), as fluid_tile2.
template <class S, int MODE, bool NT, class L = D2Q5, int QF = 9, int TY = PAIR_TY, int NTH = 256>
__device__ __forceinline__ void ad_tile2(const AdArgs &a, int tile, unsigned long long *part_r,
                                         unsigned long long *part_u, void *smem)
{
    static_assert(NTH % 64 == 0 && (64 * TY) % NTH == 0, "whole rows per thread pass");
    static_assert(!S::tile_mean || (TY == 4 && NTH == 256), "tile means are over 64 x 4 tiles");
    typedef uint16_t DT;
    typedef typename S::C C;
    constexpr int ACT = QF - 1 + L::Q;
    constexpr int LX = 66, LY = TY + 2, NR = LX * LY;
    C(*v)[LY][LX] = reinterpret_cast<C(*)[LY][LX]>(smem);
    const long long N = a.g.N;
    const int nx = a.g.nx, ny = a.g.ny;
    const int x0 = (tile % a.g.ntx) * 64, y0 = (tile / a.g.ntx) * TY;
    const LBM_GLOBAL DT *desc = gmem(static_cast<const DT *>(a.desc));
    const LBM_GLOBAL C *U = gmem(static_cast<const C *>(a.u));
    const auto gsrc = pair_src<S, L::Q>(a.src, N, nx);
    const unsigned int NN = (unsigned int)N;
    for (int r = threadIdx.x; r < NR; r += NTH) {
        const int lx = r % LX, ly = r / LX;
        const int x = x0 - 1 + lx, y = y0 - 1 + ly;
        const bool inb = x >= 0 && x < nx && y >= 0 && y < ny;
        const unsigned int n = inb ? (unsigned int)(x + nx * y) : 0u;
        const DT d = inb ? desc[n] : DT(0);
        C g[L::Q];
        if ((d >> ACT) & DT(1)) {
            C r0 = C(a.c_ref), dm = C(0), dp = C(0), rd = r0, cfull;
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_src, x, nx, r0, dm, dp, rd);
            auto src = gsrc;
            src.set(n);
            ad_collide<L, QF, S, DT>(a, x, d, src, U[n], U[NN + n], C(0), r0, dm, dp, g, cfull);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                v[i][ly][lx] = g[i];
        }
        // inactive nodes leave their slots unwritten (see fluid_tile2)
    }
    __syncthreads();
    CheckAcc<S::tile_mean> acc;
#pragma unroll
    for (int k = 0; k < 64 * TY / NTH; ++k) {
        const int lx = threadIdx.x & 63, ly = (threadIdx.x >> 6) + (NTH / 64) * k;
        NodePos p;
        p.x = x0 + lx;
        p.y = y0 + ly;
        p.z = 0;
        p.inb = p.x < nx && p.y < ny;
        p.n = p.inb ? (unsigned int)(p.x + nx * p.y) : 0u;
        const DT d = p.inb ? desc[p.n] : DT(0);
        const bool act = ((d >> ACT) & DT(1)) != 0;
        C cfull = C(0);
        C g[L::Q];
        if (act) {
            C r0 = C(a.c_ref), dm = C(0), dp = C(0), rd = r0;
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_dst, p.x, nx, r0, dm, dp, rd);
            const LdsSrc<C, L::Q, LY, LX> src{v, lx + 1, ly + 1};
            ad_collide<L, QF, S, DT>(a, p.x, d, src, U[p.n], U[NN + p.n], C(0), r0, dm, dp, g, cfull);
            if constexpr (S::colref) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    g[i] += C(L::w[i]) * (r0 - rd);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                g[i] = C(0);
        }
        ad_store<L, S, NT>(a, p, g, a.step + 1);
        if constexpr (MODE == MODE_CHECK)
            ad_check<L, QF, S, DT>(a, p, d, act, cfull, acc);
    }
    if constexpr (MODE == MODE_CHECK) {
        const double r = acc.result();
        block_max_commit<NTH / 64>(dbits(r * a.inv_cin), 0ull, part_r, part_u);
    }
    __syncthreads();
}

template <class L, int QF, class S, class DT, int MODE, bool NT, bool BUF>
__global__ void __launch_bounds__(256) k_ad_step(AdArgs a)
{
    if (a.ctrl->stop)
        return;
    const NodePos p = tile_node(a.g, xcd_tile(blockIdx.x, gridDim.x));
    unsigned long long *part = a.ctrl->part;
    ad_tile<L, QF, S, DT, MODE, NT, BUF>(a, p, part + blockIdx.x, part + gridDim.x + blockIdx.x);
}

// Two steps per launch (2-D)
template <class S, int MODE, bool NT, int TY = PAIR_TY, int NTH = 256>
__global__ void __launch_bounds__(NTH) k_fluid_step2(FluidArgs a)
{
    __shared__ __align__(16) char smem[pair_lds_bytes<typename S::C, 9, TY>()];
    if (a.ctrl->stop)
        return;
    unsigned long long *part = a.ctrl->part;
    fluid_tile2<S, MODE, NT, TY, NTH>(a, xcd_tile(blockIdx.x, gridDim.x), part + blockIdx.x,
                                      part + gridDim.x + blockIdx.x, smem);
}

template <class S, int MODE, bool NT, class L, int QF, int TY = PAIR_TY, int NTH = 256>
__global__ void __launch_bounds__(NTH) k_ad_step2(AdArgs a)
{
    __shared__ __align__(16) char smem[pair_lds_bytes<typename S::C, L::Q, TY>()];
    if (a.ctrl->stop)
        return;
    unsigned long long *part = a.ctrl->part;
    ad_tile2<S, MODE, NT, L, QF, TY, NTH>(a, xcd_tile(blockIdx.x, gridDim.x), part + blockIdx.x,
                                          part + gridDim.x + blockIdx.x, smem);
}

// NS substrate steps of one 64 x TY tile (2-D), as fluid_tileN: the first
// from global memory over the tile and an (NS - 1)-node halo, the
// intermediate ones in place in LDS with the streamed values staged in
// registers, the last stored; the frozen velocity is read from global memory
// (cache-resident) at each step.
template <class S, int MODE, bool NT, class L, int QF, int TY, int NTH, int NS>
__device__ __forceinline__ void ad_tileN(const AdArgs &a, int tile, unsigned long long *part_r,
                                         unsigned long long *part_u, void *smem)
{
    typedef uint16_t DT;
    typedef typename S::C C;
    // storage that rounds on store: as in fluid_tileN
    constexpr bool EMU = rounds_on_store<S>();
    static_assert(NS >= 3 && sizeof(C) == 4 && (MODE == MODE_PLAIN || !S::tile_mean), "4-byte compute, no tile means");
    static_assert(!EMU || NS % 2 == 0, "rounding storage: whole paired launches");
    constexpr int ACT = QF - 1 + L::Q;
    constexpr int H = NS - 1, LX = 64 + 2 * H, LY = TY + 2 * H, NR = LX * LY;
    static_assert(NTH == 64 * TY && (LX - 2) * (LY - 2) <= 2 * NTH, "two staged nodes per thread");
    C(*v)[LY][LX] = reinterpret_cast<C(*)[LY][LX]>(smem);
    DT(*dl)[LX] = reinterpret_cast<DT(*)[LX]>(static_cast<char *>(smem) + L::Q * NR * sizeof(C));
    const long long N = a.g.N;
    const int nx = a.g.nx, ny = a.g.ny;
    int x0, y0;
    strip_origin<TY>(a.g, tile, x0, y0);
    const LBM_GLOBAL DT *desc = gmem(static_cast<const DT *>(a.desc));
    const LBM_GLOBAL C *U = gmem(static_cast<const C *>(a.u));
    const auto gsrc = pair_src<S, L::Q>(a.src, N, nx);
    const unsigned int NN = (unsigned int)N;
    // node index of region slot (lx, ly) (only read for active slots)
    auto node = [&](int lx, int ly) { return (unsigned int)(x0 - H + lx + nx * (y0 - H + ly)); };
    for (int r = threadIdx.x; r < NR; r += NTH) {
        const int lx = r % LX, ly = r / LX;
        const int x = x0 - H + lx, y = y0 - H + ly;
        const bool inb = x >= 0 && x < nx && y >= 0 && y < ny;
        const unsigned int n = inb ? (unsigned int)(x + nx * y) : 0u;
        const DT d = inb ? desc[n] : DT(0);
        dl[ly][lx] = d;
        if ((d >> ACT) & DT(1)) {
            C g[L::Q], cfull;
            C r0 = C(a.c_ref), dm = C(0), dp = C(0), rd = r0;
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_src, x, nx, r0, dm, dp, rd);
            auto src = gsrc;
            src.set(n);
            ad_collide<L, QF, S, DT>(a, x, d, src, U[n], U[NN + n], C(0), r0, dm, dp, g, cfull);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                v[i][ly][lx] = g[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 2; k < NS; ++k) {
        const int lo = k - 1, RW = LX - 2 * lo, RN = RW * (LY - 2 * lo);
        C nb[2][L::Q - 1];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = threadIdx.x + q * NTH;
            if (r < RN) {
                const int lx = lo + r % RW, ly = lo + r / RW;
                if ((dl[ly][lx] >> ACT) & DT(1)) {
#pragma unroll
                    for (int i = 1; i < L::Q; ++i)
                        nb[q][i - 1] = v[i][ly - L::cy[i]][lx - L::cx[i]];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = threadIdx.x + q * NTH;
            if (r < RN) {
                const int lx = lo + r % RW, ly = lo + r / RW;
                const DT d = dl[ly][lx];
                if ((d >> ACT) & DT(1)) {
                    const unsigned int n = node(lx, ly);
                    const int x = x0 - H + lx;
                    C g[L::Q], cfull;
                    // step k ends a paired launch when k is even
                    const bool st_pt = EMU && (k % 2 == 0);
                    C r0 = C(a.c_ref), dm = C(0), dp = C(0), rd = r0;
                    if constexpr (S::colref)
                        column_refs<S>(a.ref_src, st_pt ? a.ref_dst : a.ref_src, x, nx, r0, dm, dp, rd);
                    const StagedSrc<C, LY, LX> src{v, lx, ly, nb[q]};
                    ad_collide<L, QF, S, DT>(a, x, d, src, U[n], U[NN + n], C(0), r0, dm, dp, g, cfull);
                    if constexpr (EMU) {
                        if (st_pt) {
                            if constexpr (S::colref) {
#pragma unroll
                                for (int i = 0; i < L::Q; ++i)
                                    g[i] += C(L::w[i]) * (r0 - rd);
                            }
                            unsigned int rng = sr_seed(n, (a.step + k - 1) ^ 0x5bd1e995u);
#pragma unroll
                            for (int i = 0; i < L::Q; ++i)
                                g[i] = static_cast<C>(pop_value<S>(g[i], rng));
                        }
                    }
#pragma unroll
                    for (int i = 0; i < L::Q; ++i)
                        v[i][ly][lx] = g[i];
                }
            }
        }
        __syncthreads();
    }
    CheckAcc<false> acc;
    {
        const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
        NodePos p;
        p.x = x0 + lx;
        p.y = y0 + ly;
        p.z = 0;
        p.inb = p.x < nx && p.y < ny;
        p.n = p.inb ? (unsigned int)(p.x + nx * p.y) : 0u;
        const DT d = p.inb ? dl[ly + H][lx + H] : DT(0);
        const bool act = ((d >> ACT) & DT(1)) != 0;
        C cfull = C(0);
        C g[L::Q];
        if (act) {
            C r0 = C(a.c_ref), dm = C(0), dp = C(0), rd = r0;
            if constexpr (S::colref)
                column_refs<S>(a.ref_src, a.ref_dst, p.x, nx, r0, dm, dp, rd);
            const LdsSrc<C, L::Q, LY, LX> src{v, lx + H, ly + H};
            ad_collide<L, QF, S, DT>(a, p.x, d, src, U[p.n], U[NN + p.n], C(0), r0, dm, dp, g, cfull);
            if constexpr (S::colref) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    g[i] += C(L::w[i]) * (r0 - rd);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                g[i] = C(0);
        }
        ad_store<L, S, NT>(a, p, g, a.step + NS - 1);
        if constexpr (MODE == MODE_CHECK)
            ad_check<L, QF, S, DT>(a, p, d, act, cfull, acc);
    }
    if constexpr (MODE == MODE_CHECK) {
        const double r = acc.result();
        block_max_commit<NTH / 64>(dbits(r * a.inv_cin), 0ull, part_r, part_u);
    }
}

template <class S, int MODE, bool NT, class L, int QF, int TY, int NTH, int NS>
__global__ void __launch_bounds__(NTH) k_ad_stepN(AdArgs a)
{
    __shared__ __align__(16) char smem[L::Q * (TY + 2 * (NS - 1)) * (64 + 2 * (NS - 1)) * sizeof(typename S::C) +
                                       (TY + 2 * (NS - 1)) * (64 + 2 * (NS - 1)) * 2];
    if (a.ctrl->stop)
        return;
    unsigned long long *part = a.ctrl->part;
    ad_tileN<S, MODE, NT, L, QF, TY, NTH, NS>(a, xcd_tile(blockIdx.x, gridDim.x), part + blockIdx.x,
                                              part + gridDim.x + blockIdx.x, smem);
}

// -------------------------------------------- two steps per launch (3-D)
// A block owns a 32 x TY column of the grid and marches along z over
// a segment of planes [z0, z1).  At plane k it takes the first step on the
// column and a one-node halo in x and y (34 x (TY + 2) nodes, from global
// memory), then the second step on plane k - 1 from those results.  A
// population of the first step moves by c_z to the plane where the second
// step pulls it, so the block keeps three groups of directions in LDS with
// as many planes as each needs: c_z = -1 (pulled by plane k - 1 at once:
// one plane), c_z = 0 (pulled one plane later: two) and c_z = +1 (two
// planes later: three).  A column thread's own values -- every direction,
// for bounce-back and the outlet's u* -- stay in its registers until the
// next plane.  Each segment repeats the first step on the planes z0 - 1 and
// z1 of its neighbours.  The populations cross global memory once per two
// steps; the intermediate state stays in the compute type, so FP32 results
// equal two single steps up to rounding order and FP16 storage skips one
// rounding.  Step counters: a.step and a.step + 1; a check (MODE_CHECK,
// storage without tile means) is taken on the second step.
// Column shape: 32 x TY nodes (TY = 8 or 16; 32 x TY threads), the region
// of the first step 34 x (TY + 2)
constexpr int Z3_TX = 32, Z3_LX = Z3_TX + 2;
template <int TY>
struct Z3T {
    static constexpr int NTH = Z3_TX * TY, LY = TY + 2, R = Z3_LX * LY, HALO = R - Z3_TX * TY;
    static_assert(HALO <= NTH, "one halo node per thread at most");
};

// Position of each moving direction within its c_z group, and group sizes
// (index c_z + 1)
template <class L>
struct ZGroupTable {
    int pos[L::Q];
    int n[3];
};
template <class L>
constexpr ZGroupTable<L> make_zgroups()
{
    ZGroupTable<L> t{};
    for (int i = 1; i < L::Q; ++i) {
        const int g = L::cz[i] + 1;
        t.pos[i] = t.n[g]++;
    }
    return t;
}
template <class L>
struct ZG {
    static constexpr ZGroupTable<L> t = make_zgroups<L>();
    static constexpr int NM = t.n[0], NZ = t.n[1], NP = t.n[2];
};
// LDS bytes: c_z = +1 over three planes, 0 over two, -1 over one
template <class L, class C, int TY>
constexpr int z3_lds_bytes()
{
    return (3 * ZG<L>::NP + 2 * ZG<L>::NZ + ZG<L>::NM) * Z3T<TY>::R * (int)sizeof(C);
}

// LDS plane bases of one step-2 plane z: the c_z = +1 group of plane z - 1,
// the c_z = 0 group of plane z, the c_z = -1 group of plane z + 1, and the
// c_z = +1 group of plane z (the node's own values of those directions)
template <class C>
struct Z3Planes {
    const C *p, *z, *m, *po;
};

// Slot of a direction among the values a thread keeps in registers for its
// own node: the rest direction and the c_z = -1 group, whose LDS plane is
// overwritten before the second step reads its own values
template <class L>
__device__ __forceinline__ constexpr int keep_pos(int i)
{
    return i == 0 ? 0 : 1 + ZG<L>::t.pos[i];
}
template <class L>
constexpr int keep_count()
{
    return 1 + ZG<L>::NM;
}

// The second step's source: streamed values from the LDS groups at the
// region index r of this node; own values from the groups still holding
// this node's plane, and from registers (kept) for the rest direction and
// the c_z = -1 group
template <class L, class C, int TY>
struct RingSrc {
    static constexpr int Z3_R = Z3T<TY>::R;
    const C *kept;
    Z3Planes<C> pl;
    int r;
    __device__ __forceinline__ C own(int i) const
    {
        if (i == 0 || L::cz[i] < 0)
            return kept[keep_pos<L>(i)];
        const C *base = L::cz[i] > 0 ? pl.po : pl.z;
        return base[ZG<L>::t.pos[i] * Z3_R + r];
    }
    __device__ __forceinline__ C pull(int i, int o, int cx, int cy, int cz, unsigned int m) const
    {
        const C *base = cz > 0 ? pl.p : (cz == 0 ? pl.z : pl.m);
        const C v = base[ZG<L>::t.pos[i] * Z3_R + r - cx - cy * Z3_LX];
        return m ? own(o) : v;
    }
};

// Block layout of a segment: column tile and planes
struct Z3Block {
    int x0, y0, z0, z1;
};
template <int TY>
__device__ __forceinline__ Z3Block z3_block(const Geo &g, int zseg, int tile)
{
    const int ntx = (g.nx + Z3_TX - 1) / Z3_TX, nty = (g.ny + TY - 1) / TY;
    const int col = tile % (ntx * nty), seg = tile / (ntx * nty);
    Z3Block b;
    b.x0 = (col % ntx) * Z3_TX;
    b.y0 = (col / ntx) * TY;
    b.z0 = seg * zseg;
    b.z1 = min(b.z0 + zseg, g.nz);
    return b;
}

// Region coordinates (lx, ly) of this thread's node in pass 0 (the column)
// or pass 1 (the halo: top row, bottom row, left column, right column)
template <int TY>
__device__ __forceinline__ void z3_region(int pass, int t, int &lx, int &ly)
{
    constexpr int Z3_LY = Z3T<TY>::LY;
    if (pass == 0) {
        lx = 1 + t % Z3_TX;
        ly = 1 + t / Z3_TX;
    } else if (t < Z3_LX) {
        lx = t;
        ly = 0;
    } else if (t < 2 * Z3_LX) {
        lx = t - Z3_LX;
        ly = Z3_LY - 1;
    } else if (t < 2 * Z3_LX + TY) {
        lx = 0;
        ly = 1 + t - 2 * Z3_LX;
    } else {
        lx = Z3_LX - 1;
        ly = 1 + t - 2 * Z3_LX - TY;
    }
}

// Store the first-step values f of the node at region index r of plane k
// into the LDS groups (the rest direction is never pulled)
template <class L, class C, int TY>
__device__ __forceinline__ void z3_put(C *lds, int k, int r, const C f[L::Q])
{
    constexpr int NP = ZG<L>::NP, NZ = ZG<L>::NZ, Z3_R = Z3T<TY>::R;
    C *gp = lds + ((k % 3 + 3) % 3) * NP * Z3_R;
    C *gz = lds + 3 * NP * Z3_R + (k & 1) * NZ * Z3_R;
    C *gm = lds + (3 * NP + 2 * NZ) * Z3_R;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        C *base = L::cz[i] > 0 ? gp : (L::cz[i] == 0 ? gz : gm);
        base[ZG<L>::t.pos[i] * Z3_R + r] = f[i];
    }
}

template <class L, class C, int TY>
__device__ __forceinline__ Z3Planes<C> z3_planes(const C *lds, int z)
{
    constexpr int NP = ZG<L>::NP, NZ = ZG<L>::NZ, Z3_R = Z3T<TY>::R;
    Z3Planes<C> pl;
    pl.p = lds + (((z - 1) % 3 + 3) % 3) * NP * Z3_R;
    pl.z = lds + 3 * NP * Z3_R + (z & 1) * NZ * Z3_R;
    pl.m = lds + (3 * NP + 2 * NZ) * Z3_R;
    pl.po = lds + (z % 3) * NP * Z3_R;
    return pl;
}

// A node's first-step inputs, loaded one plane ahead of their use: the value
// each direction pulls, its address already selected by the node's reversed
// links (v[0] = own(0)), the frozen velocity (substrate), and on the outlet
// column the node's own values the outlet rule reads that no pull supplies
// (directions in OWN; HASO, else loaded when used).
template <class L, class C, int NO>
struct PreVals {
    C v[L::Q];
    C o[NO > 0 ? NO : 1];
    C u[3];
};

// Directions whose own value an outlet rule reads besides the pulled ones:
// the fluid's u* reads every own value -- those with c_x = +1 are the
// reversed pulls of the outlet's c_x = -1 links -- the substrate's
// zero-gradient copy reads its c_x = -1 ones.
template <class L>
constexpr unsigned int fluid_out_own()
{
    unsigned int m = 0;
    for (int i = 1; i < L::Q; ++i)
        if (L::cx[i] <= 0)
            m |= 1u << i;
    return m;
}
template <class L>
constexpr int own_count(unsigned int m)
{
    int n = 0;
    for (int i = 1; i < L::Q; ++i)
        n += (m >> i) & 1u;
    return n;
}
__device__ __forceinline__ constexpr int own_pos(unsigned int m, int i)
{
    return __builtin_popcount(m & ((1u << i) - 1u));
}

// Source over prefetched values (see PreVals); g: the node's global source
template <class L, class C, unsigned int OWN, bool HASO, class G>
struct PreSrc {
    const C *v, *o;
    G g;
    __device__ __forceinline__ C own(int i) const
    {
        if (i == 0)
            return v[0];
        if ((OWN >> i) & 1u) {
            if constexpr (HASO)
                return o[own_pos(OWN, i)];
            else
                return g.own(i);
        }
        return v[L::op[i]];
    }
    __device__ __forceinline__ C pull(int i, int, int, int, int, unsigned int) const { return v[i]; }
};

// Global source of a first-step node: one load per direction from the
// address the reversed links select (buffer resource where the array fits
// 32-bit byte offsets)
template <class L, class S, bool BUF>
__device__ __forceinline__ auto z3_src(const void *src, const Geo &g, unsigned int n)
{
    typedef typename S::T T;
    if constexpr (BUF)
        return BufSrc<S, false>{pop_rsrc(static_cast<const T *>(src), (unsigned int)L::Q, (unsigned int)g.N),
                                (unsigned int)g.N * (unsigned int)sizeof(T), n * (unsigned int)sizeof(T),
                                g.nx * (int)sizeof(T), g.nx * g.ny * (int)sizeof(T)};
    else
        return GlobalSrc<S>{static_cast<const T *>(src), (unsigned int)g.N, n, g.nx, g.nx * g.ny};
}

// Issue the loads of a first-step node with reversed links rev
template <class L, unsigned int OWN, bool HASO, class G, class C, int NO>
__device__ __forceinline__ void z3_prefetch(const G &g, unsigned int rev, bool xout, PreVals<L, C, NO> &p)
{
    p.v[0] = g.own(0);
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
        p.v[i] = g.pull(i, L::op[i], L::cx[i], L::cy[i], L::cz[i], bit_mask(rev, i));
    if constexpr (HASO) {
        if (xout) {
#pragma unroll
            for (int i = 1; i < L::Q; ++i)
                if ((OWN >> i) & 1u)
                    p.o[own_pos(OWN, i)] = g.own(i);
        }
    }
}

// Reversed links of a node (as the collide functions form them): blocked
// sources, and the links through the inlet and outlet faces
template <class L>
__device__ __forceinline__ unsigned int z3_rev(unsigned int blocked, bool xin, bool xout)
{
    unsigned int rev = blocked & ((1u << L::Q) - 2u);
    rev |= xin ? xdirs<L>(1) : 0u;
    rev |= xout ? xdirs<L>(-1) : 0u;
    return rev;
}

// The two step-1 nodes of a thread: its column node (c) and, for threads
// below Z3_HALO, one halo node (h); their grid positions do not depend on z
struct Z3Nodes {
    int xc, yc, xh, yh, rc, rh;
    bool inc, inh;
};
template <int TY>
__device__ __forceinline__ Z3Nodes z3_nodes(const Z3Block &b, int nx, int ny)
{
    constexpr int Z3_HALO = Z3T<TY>::HALO;
    Z3Nodes q;
    const int t = threadIdx.x;
    int lx, ly;
    z3_region<TY>(0, t, lx, ly);
    q.xc = b.x0 + lx - 1;
    q.yc = b.y0 + ly - 1;
    q.rc = ly * Z3_LX + lx;
    q.inc = q.xc < nx && q.yc < ny;
    z3_region<TY>(1, t < Z3_HALO ? t : 0, lx, ly);
    q.xh = b.x0 + lx - 1;
    q.yh = b.y0 + ly - 1;
    q.rh = ly * Z3_LX + lx;
    q.inh = t < Z3_HALO && q.xh >= 0 && q.xh < nx && q.yh >= 0 && q.yh < ny;
    return q;
}

// Stores of a z-marching second step.  With a buffer resource (BUF) every
// lane issues its Q stores: no branch separates them from the loads of the
// next plane, so the compiler's waits for those loads count the stores
// issued after them and let the stores drain in the background.  A lane
// with nothing to write (off the grid, or a plane outside the block's
// segment) stores at offsets from the resource's end on, which the
// hardware drops (the host takes this form only where (2Q - 1) N sizeof(T)
// bytes fit 32-bit offsets).  Values and rounding as fluid_store /
// ad_store: seed is their stochastic-rounding seed.
template <class L, class S, bool NT, bool BUF>
__device__ __forceinline__ void z3_store(void *dst, unsigned int N, unsigned int n, bool ok,
                                         typename S::C f[L::Q], unsigned int seed)
{
    typedef typename S::T T;
    unsigned int rng = seed;
    if constexpr (BUF) {
        const unsigned int stride = N * (unsigned int)sizeof(T);
        const unsigned int numrec = (unsigned int)L::Q * stride;
        const auto r = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)numrec, 0x00020000);
        const unsigned int base = ok ? n * (unsigned int)sizeof(T) : numrec;
        constexpr int aux = NT ? 2 : 0; // non-temporal
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const T h = pop_value<S>(f[i], rng);
            if constexpr (sizeof(T) == 4)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, h), r,
                                                      base + (unsigned int)i * stride, 0, aux);
            else
                __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, h), r,
                                                      base + (unsigned int)i * stride, 0, aux);
        }
    } else if (ok) {
        T *d = static_cast<T *>(dst);
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            st_pop<S, NT>(d + ((unsigned int)i * N + n), f[i], rng);
    }
}

// Q stores that write nothing (offsets past the resource's end), issued
// once before a z-marching loop right after its first descriptor loads.
// The loop's entry then has as many stores in flight behind those loads as
// its back edge has behind the next plane's, and the compiler's wait for
// the loaded values at the loop head -- the smaller count over both edges --
// lets the previous plane's stores drain instead of waiting for them.
template <class L, class S, bool NT, bool BUF>
__device__ __forceinline__ void z3_entry_stores(void *dst, unsigned int N)
{
    if constexpr (BUF) {
        typename S::C zero[L::Q];
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
            zero[i] = typename S::C(0);
        z3_store<L, S, NT, BUF>(dst, N, 0u, false, zero, 0u);
    }
}

// Node descriptor of a z-marching block (0 off the grid and outside the
// planes 0..nz-1): a buffer load, so that no branch guards it
template <class DT>
__device__ __forceinline__ DT z3_desc(__amdgpu_buffer_rsrc_t r, bool ok, unsigned int n)
{
    static_assert(sizeof(DT) == 4, "3-D descriptor words are 32-bit");
    return __builtin_amdgcn_raw_buffer_load_b32(r, ok ? n * 4u : 0xFFFFFFFFu, 0, 0);
}

template <class S, int MODE, bool NT, bool BUF, int TY>
__device__ __forceinline__ void fluid_tile3d2(const FluidArgs &a, int tile, unsigned long long *part_r,
                                              unsigned long long *part_u, void *smem)
{
    typedef D3Q19 L;
    typedef uint32_t DT;
    typedef typename S::C C;
    constexpr unsigned int OWN = fluid_out_own<L>();
    constexpr int NO = own_count<L>(OWN);
    static_assert(MODE == MODE_PLAIN || !S::tile_mean, "checks with tile means take single steps");
    C *lds = static_cast<C *>(smem);
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const Z3Block b = z3_block<TY>(a.g, a.zseg, tile);
    const auto drs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.desc), (short)0,
                                                       (int)((unsigned int)a.g.N * 4u), 0x00020000);
    const Z3Nodes q = z3_nodes<TY>(b, nx, ny);
    const bool xin_c = q.xc == 0, xout_c = q.xc == nx - 1;
    const bool xin_h = q.xh == 0, xout_h = q.xh == nx - 1;
    // column references (FP16 storage): constant over the launch
    C r0c = C(1), dmc = C(0), dpc = C(0), r0h = C(1), dmh = C(0), dph = C(0), rdc = C(1), rd2 = C(1);
    C s2m = C(0), s2p = C(0), s2r = C(1);
    if constexpr (S::colref) {
        if (q.inc) {
            column_refs<S>(a.ref_src, a.ref_src, q.xc, nx, r0c, dmc, dpc, rdc);
            column_refs<S>(a.ref_src, a.ref_dst, q.xc, nx, s2r, s2m, s2p, rd2);
        }
        if (q.inh)
            column_refs<S>(a.ref_src, a.ref_src, q.xh, nx, r0h, dmh, dph, rdc);
    }
    auto nidx = [&](int x, int y, int k) { return (unsigned int)(x + nx * (y + ny * k)); };
    auto dload = [&](bool in, int x, int y, int k) {
        return z3_desc<DT>(drs, in && k >= 0 && k < nz, nidx(x, y, k));
    };
    const int kb = b.z0 - 1, ke = b.z1;
    PreVals<L, C, NO> pc, ph;
    DT dc = dload(q.inc, q.xc, q.yc, kb), dh = dload(q.inh, q.xh, q.yh, kb);
    auto issue = [&](int k) {
        if (dc & DT(1)) {
            const auto g = z3_src<L, S, BUF>(a.src, a.g, nidx(q.xc, q.yc, k));
            z3_prefetch<L, OWN, true>(g, z3_rev<L>((unsigned int)dc, xin_c, xout_c), xout_c, pc);
        }
        if (dh & DT(1)) {
            const auto g = z3_src<L, S, BUF>(a.src, a.g, nidx(q.xh, q.yh, k));
            z3_prefetch<L, OWN, false>(g, z3_rev<L>((unsigned int)dh, xin_h, xout_h), xout_h, ph);
        }
    };
    issue(kb);
    DT dcn = dload(q.inc, q.xc, q.yc, kb + 1), dhn = dload(q.inh, q.xh, q.yh, kb + 1);
    z3_entry_stores<L, S, NT, BUF>(a.dst, (unsigned int)a.g.N);
    constexpr int NK = keep_count<L>();
    C own[NK], nxt[NK];
    DT dnx = DT(0);
#pragma unroll
    for (int i = 0; i < NK; ++i)
        nxt[i] = C(0);
    CheckAcc<S::tile_mean> acc;
    for (int k = kb; k <= ke; ++k) {
        // the kept values of plane k - 1 become this node's own
        const DT d = dnx;
#pragma unroll
        for (int i = 0; i < NK; ++i)
            own[i] = nxt[i];
        __syncthreads(); // the previous plane's second step has read the LDS
        // first step at plane k from the prefetched values
        if (dc & DT(1)) {
            C f[L::Q], ux, uy, uz, rho;
            const auto g = z3_src<L, S, BUF>(a.src, a.g, nidx(q.xc, q.yc, k));
            const PreSrc<L, C, OWN, true, decltype(g)> src{pc.v, pc.o, g};
            fluid_collide<L, S, DT>(a, q.xc, dc, src, r0c, dmc, dpc, f, ux, uy, uz, rho);
            z3_put<L, C, TY>(lds, k, q.rc, f);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                if (i == 0 || L::cz[i] < 0)
                    nxt[keep_pos<L>(i)] = f[i];
        }
        if (dh & DT(1)) {
            C f[L::Q], ux, uy, uz, rho;
            const auto g = z3_src<L, S, BUF>(a.src, a.g, nidx(q.xh, q.yh, k));
            const PreSrc<L, C, OWN, false, decltype(g)> src{ph.v, ph.o, g};
            fluid_collide<L, S, DT>(a, q.xh, dh, src, r0h, dmh, dph, f, ux, uy, uz, rho);
            z3_put<L, C, TY>(lds, k, q.rh, f);
        }
        // inactive nodes leave their slots unwritten: a second step reads a
        // slot only as one of a link's two candidates and selects its own
        // value whenever the slot's node is blocked
        dnx = dc;
        // loads of plane k + 1 (in flight during the second step below)
        dc = dcn;
        dh = dhn;
        if (k + 1 <= ke)
            issue(k + 1);
        dcn = dload(q.inc, q.xc, q.yc, k + 2);
        dhn = dload(q.inh, q.xh, q.yh, k + 2);
        __syncthreads();
        // second step at plane z = k - 1 (the first two passes have none:
        // their results are not stored)
        const int z = k - 1;
        const bool zok = z >= b.z0 && z < b.z1;
        NodePos p;
        p.x = q.xc;
        p.y = q.yc;
        p.z = z;
        p.inb = q.inc && zok;
        p.n = p.inb ? nidx(q.xc, q.yc, z) : 0u;
        const bool act = zok && (d & DT(1)) != 0;
        C ux = C(0), uy = C(0), uz = C(0), rho = C(0);
        C f[L::Q];
        if (act) {
            const RingSrc<L, C, TY> src{own, z3_planes<L, C, TY>(lds, z), q.rc};
            fluid_collide<L, S, DT>(a, q.xc, d, src, s2r, s2m, s2p, f, ux, uy, uz, rho);
            if constexpr (S::colref) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    f[i] += C(L::w[i]) * (s2r - rd2);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                f[i] = C(0);
        }
        z3_store<L, S, NT, BUF>(a.dst, (unsigned int)a.g.N, p.n, p.inb, f,
                                sizeof(typename S::T) == 2 ? sr_seed(p.n, a.step + 1) : 0u);
        if constexpr (MODE == MODE_CHECK)
            if (p.inb)
                fluid_check<L, S, DT>(a, p, d, act, ux, uy, uz, rho, acc);
    }
    if constexpr (MODE == MODE_CHECK) {
        const double r = acc.result();
        block_max_commit<Z3T<TY>::NTH / 64>(dbits(r * a.inv_uin), acc.ub, part_r, part_u);
    }
}

template <class S, int MODE, bool NT, bool BUF, int TY>
__global__ void __launch_bounds__(Z3T<TY>::NTH) k_fluid_step3d2(FluidArgs a)
{
    __shared__ __align__(16) char smem[z3_lds_bytes<D3Q19, typename S::C, TY>()];
    if (a.ctrl->stop)
        return;
    unsigned long long *part = a.ctrl->part;
    fluid_tile3d2<S, MODE, NT, BUF, TY>(a, xcd_tile(blockIdx.x, gridDim.x), part + blockIdx.x,
                                    part + gridDim.x + blockIdx.x, smem);
}

template <class S, int MODE, bool NT, bool BUF, int TY>
__device__ __forceinline__ void ad_tile3d2(const AdArgs &a, int tile, unsigned long long *part_r,
                                           unsigned long long *part_u, void *smem)
{
    typedef D3Q7 L;
    typedef uint32_t DT;
    typedef typename S::C C;
    constexpr int QF = 19;
    constexpr int ACT = QF - 1 + L::Q;
    constexpr int LNK = QF - 1;
    constexpr unsigned int OWN = xdirs<L>(-1);
    constexpr int NO = own_count<L>(OWN);
    static_assert(MODE == MODE_PLAIN || !S::tile_mean, "checks with tile means take single steps");
    C *lds = static_cast<C *>(smem);
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const Z3Block b = z3_block<TY>(a.g, a.zseg, tile);
    const auto drs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(a.desc), (short)0,
                                                       (int)((unsigned int)a.g.N * 4u), 0x00020000);
    const LBM_GLOBAL C *U = gmem(static_cast<const C *>(a.u));
    const unsigned int NN = (unsigned int)a.g.N;
    const Z3Nodes q = z3_nodes<TY>(b, nx, ny);
    const bool xin_c = q.xc == 0, xout_c = q.xc == nx - 1;
    const bool xin_h = q.xh == 0, xout_h = q.xh == nx - 1;
    C r0c = C(a.c_ref), dmc = C(0), dpc = C(0), r0h = C(a.c_ref), dmh = C(0), dph = C(0), rdc = r0c;
    C s2r = C(a.c_ref), s2m = C(0), s2p = C(0), rd2 = s2r;
    if constexpr (S::colref) {
        if (q.inc) {
            column_refs<S>(a.ref_src, a.ref_src, q.xc, nx, r0c, dmc, dpc, rdc);
            column_refs<S>(a.ref_src, a.ref_dst, q.xc, nx, s2r, s2m, s2p, rd2);
        }
        if (q.inh)
            column_refs<S>(a.ref_src, a.ref_src, q.xh, nx, r0h, dmh, dph, rdc);
    }
    auto nidx = [&](int x, int y, int k) { return (unsigned int)(x + nx * (y + ny * k)); };
    auto dload = [&](bool in, int x, int y, int k) {
        return z3_desc<DT>(drs, in && k >= 0 && k < nz, nidx(x, y, k));
    };
    const int kb = b.z0 - 1, ke = b.z1;
    PreVals<L, C, NO> pc, ph;
    DT dc = dload(q.inc, q.xc, q.yc, kb), dh = dload(q.inh, q.xh, q.yh, kb);
    auto issue = [&](int k) {
        if ((dc >> ACT) & DT(1)) {
            const unsigned int n = nidx(q.xc, q.yc, k);
            const auto g = z3_src<L, S, BUF>(a.src, a.g, n);
            z3_prefetch<L, OWN, true>(g, z3_rev<L>((unsigned int)dc >> LNK, xin_c, xout_c), xout_c, pc);
            pc.u[0] = U[n];
            pc.u[1] = U[NN + n];
            pc.u[2] = U[2u * NN + n];
        }
        if ((dh >> ACT) & DT(1)) {
            const unsigned int n = nidx(q.xh, q.yh, k);
            const auto g = z3_src<L, S, BUF>(a.src, a.g, n);
            z3_prefetch<L, OWN, false>(g, z3_rev<L>((unsigned int)dh >> LNK, xin_h, xout_h), xout_h, ph);
            ph.u[0] = U[n];
            ph.u[1] = U[NN + n];
            ph.u[2] = U[2u * NN + n];
        }
    };
    issue(kb);
    DT dcn = dload(q.inc, q.xc, q.yc, kb + 1), dhn = dload(q.inh, q.xh, q.yh, kb + 1);
    z3_entry_stores<L, S, NT, BUF>(a.dst, (unsigned int)a.g.N);
    constexpr int NK = keep_count<L>();
    C own[NK], nxt[NK];
    C ou[3], nu[3];
    DT dnx = DT(0);
#pragma unroll
    for (int i = 0; i < NK; ++i)
        nxt[i] = C(0);
    nu[0] = nu[1] = nu[2] = C(0);
    CheckAcc<S::tile_mean> acc;
    for (int k = kb; k <= ke; ++k) {
        const DT d = dnx;
#pragma unroll
        for (int i = 0; i < NK; ++i)
            own[i] = nxt[i];
        ou[0] = nu[0];
        ou[1] = nu[1];
        ou[2] = nu[2];
        __syncthreads();
        if ((dc >> ACT) & DT(1)) {
            C g[L::Q], cfull;
            const auto gs = z3_src<L, S, BUF>(a.src, a.g, nidx(q.xc, q.yc, k));
            const PreSrc<L, C, OWN, true, decltype(gs)> src{pc.v, pc.o, gs};
            ad_collide<L, QF, S, DT>(a, q.xc, dc, src, pc.u[0], pc.u[1], pc.u[2], r0c, dmc, dpc, g, cfull);
            z3_put<L, C, TY>(lds, k, q.rc, g);
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                if (i == 0 || L::cz[i] < 0)
                    nxt[keep_pos<L>(i)] = g[i];
            nu[0] = pc.u[0];
            nu[1] = pc.u[1];
            nu[2] = pc.u[2];
        }
        if ((dh >> ACT) & DT(1)) {
            C g[L::Q], cfull;
            const auto gs = z3_src<L, S, BUF>(a.src, a.g, nidx(q.xh, q.yh, k));
            const PreSrc<L, C, OWN, false, decltype(gs)> src{ph.v, ph.o, gs};
            ad_collide<L, QF, S, DT>(a, q.xh, dh, src, ph.u[0], ph.u[1], ph.u[2], r0h, dmh, dph, g, cfull);
            z3_put<L, C, TY>(lds, k, q.rh, g);
        }
        dnx = dc;
        dc = dcn;
        dh = dhn;
        if (k + 1 <= ke)
            issue(k + 1);
        dcn = dload(q.inc, q.xc, q.yc, k + 2);
        dhn = dload(q.inh, q.xh, q.yh, k + 2);
        __syncthreads();
        // second step at plane z = k - 1 (none in the first two passes)
        const int z = k - 1;
        const bool zok = z >= b.z0 && z < b.z1;
        NodePos p;
        p.x = q.xc;
        p.y = q.yc;
        p.z = z;
        p.inb = q.inc && zok;
        p.n = p.inb ? nidx(q.xc, q.yc, z) : 0u;
        const bool act = zok && ((d >> ACT) & DT(1)) != 0;
        C cfull = C(0);
        C g[L::Q];
        if (act) {
            const RingSrc<L, C, TY> src{own, z3_planes<L, C, TY>(lds, z), q.rc};
            ad_collide<L, QF, S, DT>(a, q.xc, d, src, ou[0], ou[1], ou[2], s2r, s2m, s2p, g, cfull);
            if constexpr (S::colref) {
#pragma unroll
                for (int i = 0; i < L::Q; ++i)
                    g[i] += C(L::w[i]) * (s2r - rd2);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L::Q; ++i)
                g[i] = C(0);
        }
        z3_store<L, S, NT, BUF>(a.dst, (unsigned int)a.g.N, p.n, p.inb, g,
                                sizeof(typename S::T) == 2 ? sr_seed(p.n, (a.step + 1) ^ 0x5bd1e995u) : 0u);
        if constexpr (MODE == MODE_CHECK)
            if (p.inb)
                ad_check<L, QF, S, DT>(a, p, d, act, cfull, acc);
    }
    if constexpr (MODE == MODE_CHECK) {
        const double r = acc.result();
        block_max_commit<Z3T<TY>::NTH / 64>(dbits(r * a.inv_cin), 0ull, part_r, part_u);
    }
}

template <class S, int MODE, bool NT, bool BUF, int TY>
__global__ void __launch_bounds__(Z3T<TY>::NTH) k_ad_step3d2(AdArgs a)
{
    __shared__ __align__(16) char smem[z3_lds_bytes<D3Q7, typename S::C, TY>()];
    if (a.ctrl->stop)
        return;
    unsigned long long *part = a.ctrl->part;
    ad_tile3d2<S, MODE, NT, BUF, TY>(a, xcd_tile(blockIdx.x, gridDim.x), part + blockIdx.x,
                                 part + gridDim.x + blockIdx.x, smem);
}

// ------------------------------------------------------- init / export
template <class L, class S, class DT>
__global__ void __launch_bounds__(256) k_fluid_init(typename S::T *f, const DT *desc, long long N)
{
    const long long n = blockIdx.x * 256ll + threadIdx.x;
    if (n >= N)
        return;
    const bool act = (desc[n] & DT(1)) != 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        st<S>(f + (long long)i * N + n,
              act ? (S::shifted ? typename S::C(0) : typename S::C(L::w[i])) : typename S::C(0));
}

template <class L, int QF, class S, class DT>
__global__ void __launch_bounds__(256) k_ad_init(typename S::T *gp, const DT *desc,
                                                  const typename S::C *U, long long N,
                                                  double c_init, double c_ref)
{
    typedef typename S::C C;
    constexpr int ACT = QF - 1 + L::Q;
    const long long n = blockIdx.x * 256ll + threadIdx.x;
    if (n >= N)
        return;
    const bool act = ((desc[n] >> ACT) & DT(1)) != 0;
    const C ux = act ? U[n] : C(0), uy = act ? U[N + n] : C(0);
    const C uz = (act && L::DIM == 3) ? U[2 * N + n] : C(0);
    const C cs = S::shifted ? C(c_init - c_ref) : C(c_init);
    const C usq = C(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const C cu = i == 0 ? C(0) : cdot<L>(i, ux, uy, uz);
        const C t = ad_second_order<L> ? C(3) * cu + (C(4.5) * cu * cu - usq) : C(L::inv_cs2) * cu;
        const C v = C(L::w[i]) * (cs + C(c_init) * t);
        st<S>(gp + (long long)i * N + n, act ? v : C(0));
    }
}

template <class L, class S, class DT, class O>
__global__ void __launch_bounds__(256) k_fluid_export(const typename S::T *f, const DT *desc,
                                                       long long N, const float *ref, int nx, O *U,
                                                       O *RHO)
{
    const long long n = blockIdx.x * 256ll + threadIdx.x;
    if (n >= N)
        return;
    const bool act = (desc[n] & DT(1)) != 0;
    O rs = O(0), jx = O(0), jy = O(0), jz = O(0);
    if (act) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const O v = static_cast<O>(f[(long long)i * N + n]);
            rs += v;
            if (L::cx[i] == 1) jx += v;
            if (L::cx[i] == -1) jx -= v;
            if (L::cy[i] == 1) jy += v;
            if (L::cy[i] == -1) jy -= v;
            if (L::cz[i] == 1) jz += v;
            if (L::cz[i] == -1) jz -= v;
        }
    }
    const O rho = act ? (S::shifted ? O(ref[n % nx]) + rs : rs) : O(0);
    const O inv = act ? O(1) / rho : O(0);
    if (U) {
        U[n] = jx * inv;
        U[N + n] = jy * inv;
        if (L::DIM == 3)
            U[2 * N + n] = jz * inv;
    }
    if (RHO)
        RHO[n] = rho;
}

template <class L, int QF, class S, class DT, class O>
__global__ void __launch_bounds__(256) k_ad_export(const typename S::T *gp, const DT *desc,
                                                    long long N, const float *ref, int nx,
                                                    Sink sink, O *Cout)
{
    constexpr int ACT = QF - 1 + L::Q;
    constexpr int BIO = ACT + 1;
    const long long n = blockIdx.x * 256ll + threadIdx.x;
    if (n >= N)
        return;
    const DT d = desc[n];
    if (!((d >> ACT) & DT(1))) {
        Cout[n] = O(0);
        return;
    }
    O s = O(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        s += static_cast<O>(gp[(long long)i * N + n]);
    if (S::shifted)
        s += O(ref[n % nx]);
    Cout[n] = ((d >> BIO) & DT(1)) ? O(collided_c((double)s, sink.k, sink.kh)) : s;
}

template <class L, class S, class DT>
__global__ void __launch_bounds__(256) k_pops_export(const typename S::T *h, const DT *desc,
                                                      long long N, int act_bit, const float *ref,
                                                      int nx, double *out)
{
    const long long n = blockIdx.x * 256ll + threadIdx.x;
    if (n >= N)
        return;
    const bool act = ((desc[n] >> act_bit) & DT(1)) != 0;
    const double r = S::shifted ? (double)ref[n % nx] : 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double v = static_cast<double>(h[(long long)i * N + n]);
        out[(long long)i * N + n] = act ? v + L::w[i] * r : 0.0;
    }
}

template <class L, class S, class DT>
__global__ void __launch_bounds__(256) k_pops_import(typename S::T *h, const DT *desc, long long N,
                                                      int act_bit, const float *ref, int nx,
                                                      const double *in)
{
    const long long n = blockIdx.x * 256ll + threadIdx.x;
    if (n >= N)
        return;
    const bool act = ((desc[n] >> act_bit) & DT(1)) != 0;
    const double r = S::shifted ? (double)ref[n % nx] : 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double v = in[(long long)i * N + n] - L::w[i] * r;
        h[(long long)i * N + n] = static_cast<typename S::T>(act ? v : 0.0);
    }
}

// vals: unshifted values [L::Q], stored at the listed nodes (ref may be null
// when every value is 0)
template <class L, class S>
__global__ void __launch_bounds__(256) k_pops_set_nodes(typename S::T *h, long long N,
                                                        const float *ref, int nx,
                                                        const long long *idx, int count,
                                                        const double *vals)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= count)
        return;
    const long long n = idx[k];
    const double r = (S::shifted && ref) ? (double)ref[n % nx] : 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        h[(long long)i * N + n] = static_cast<typename S::T>(vals[i] - L::w[i] * r);
}

__global__ void __launch_bounds__(256) k_ref_fill(float *ref, int n, float v)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x < n)
        ref[x] = v;
}

__global__ void __launch_bounds__(256) k_ref_roll(const Ctrl *ctrl, float *cur, const float *next,
                                                  int n)
{
    if (ctrl->stop != STOP_RUN)
        return;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x < n)
        cur[x] = next[x];
}

// ---------------------------------------------------------------- fluxes
// Per node, in FP64 on the unshifted values:
//   fluid in   = sum over inlet links (incoming - outgoing)
//   fluid out  = sum over outlet links (outgoing - incoming)
//   sub in/out = same for the substrate links, sink = k * sum g* / (1 - k)
// Each block reduces a fixed node range in a fixed tree order; the second
// pass sums the block partials in index order: the result is reproducible.
template <class LF, class LA, class S, class DT>
__global__ void __launch_bounds__(256) k_flux_partials(const typename S::T *f,
                                                        const typename S::T *gp, const DT *desc,
                                                        Geo g, const float *ref_f,
                                                        const float *ref_g, double u_in,
                                                        double c_in, Sink sink, int outlet,
                                                        double c_out, const typename S::C *U,
                                                        double *part)
{
    constexpr int ACT = LF::Q - 1 + LA::Q;
    constexpr int BIO = ACT + 1;
    const long long N = g.N;
    const long long per = (N + gridDim.x - 1) / gridDim.x;
    const long long lo = blockIdx.x * per;
    const long long hi = lo + per < N ? lo + per : N;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long n = lo + threadIdx.x; n < hi; n += 256) {
        const int x = (int)(n % g.nx);
        if (x != 0 && x != g.nx - 1) {
            if (!gp)
                continue;
        }
        const DT d = desc[n];
        const double fs = (S::shifted && f) ? (double)ref_f[x] : 0.0;
        const double gs = (S::shifted && gp) ? (double)ref_g[x] : 0.0;
        if constexpr (LF::Q > 1) {
        if (f && (d & DT(1)) && (x == 0 || x == g.nx - 1)) {
            double r = 0.0, qx = 0.0, qy = 0.0, qz = 0.0;
#pragma unroll
            for (int k = 0; k < LF::Q; ++k) {
                const double v = static_cast<double>(f[(long long)k * N + n]) + fs * LF::w[k];
                r += v;
                qx += LF::cx[k] * v;
                qy += LF::cy[k] * v;
                qz += LF::cz[k] * v;
            }
            const double ux = qx / r, uy = qy / r, uz = qz / r;
            const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
            for (int i = 1; i < LF::Q; ++i) {
                const int o = LF::op[i];
                const double fo = static_cast<double>(f[(long long)o * N + n]) + fs * LF::w[o];
                if (x == 0 && LF::cx[i] == 1) {
                    const double incoming = fo + 6.0 * LF::w[i] * u_in;
                    acc[0] += incoming - fo;
                }
                if (x == g.nx - 1 && LF::cx[i] == -1) {
                    const double cu = LF::cx[i] * ux + LF::cy[i] * uy + LF::cz[i] * uz;
                    const double incoming = -fo + 2.0 * LF::w[i] * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                    acc[1] += fo - incoming;
                }
            }
        }
        }
        if (gp && ((d >> ACT) & DT(1))) {
            if (x == 0 || x == g.nx - 1) {
                // even part of the equilibrium per unit concentration: 1, or
                // 1 + 9/2 (c.u)^2 - 3/2 u^2 in the second-order form
                double ux = 0.0, uy = 0.0, uz = 0.0;
                if (ad_second_order<LA> && U) {
                    ux = (double)U[n];
                    uy = (double)U[N + n];
                    uz = LA::DIM == 3 ? (double)U[2 * N + n] : 0.0;
                }
                const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
                for (int i = 1; i < LA::Q; ++i) {
                    const int o = LA::op[i];
                    const double go = static_cast<double>(gp[(long long)o * N + n]) + gs * LA::w[o];
                    const double cu = LA::cx[i] * ux + LA::cy[i] * uy + LA::cz[i] * uz;
                    const double ev = ad_second_order<LA> ? 1.0 + 4.5 * cu * cu - 1.5 * uu : 1.0;
                    if (x == 0 && LA::cx[i] == 1) {
                        const double incoming = -go + 2.0 * LA::w[i] * c_in * ev;
                        acc[2] += incoming - go;
                    }
                    if (x == g.nx - 1 && LA::cx[i] == -1) {
                        const double gi = static_cast<double>(gp[(long long)i * N + n]) + gs * LA::w[i];
                        const double incoming = outlet ? -go + 2.0 * LA::w[i] * c_out * ev : gi;
                        acc[3] += go - incoming;
                    }
                }
            }
            if ((d >> BIO) & DT(1)) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < LA::Q; ++i)
                    s += static_cast<double>(gp[(long long)i * N + n]) + gs * LA::w[i];
                acc[4] += sink.kh > 0.0 ? collided_c(s, sink.k, sink.kh) - s : sink.k * s / (1.0 - sink.k);
            }
        }
    }
    __shared__ double red[5][256];
    for (int k = 0; k < 5; ++k)
        red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 5; ++k)
                red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k)
            part[k * gridDim.x + blockIdx.x] = red[k][0];
}

// One wave per component: each lane sums a fixed stride of the partials in
// index order, then a fixed shuffle tree combines the lanes.
__global__ void __launch_bounds__(320) k_flux_final(const double *part, int nb, double *out5)
{
    const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < nb; b += 64)
        s += part[k * nb + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_down(s, off);
    if (lane == 0)
        out5[k] = s;
}

// ------------------------------------------------------------- control
__global__ void k_ctrl_reset(Ctrl *c, double tol, int window, int is_fluid, int K,
                             unsigned long long *part, int nparts, long long t_max)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->part = part;
        c->nparts = nparts;
        c->res_bits = 0ull;
        c->umax_bits = 0ull;
        c->tol = tol;
        c->best = __longlong_as_double(0x7ff0000000000000ll); // +inf
        c->peak = __longlong_as_double((long long)0xfff0000000000000ull); // -inf
        c->r_last = __longlong_as_double(0x7ff8000000000000ll);
        c->t = 0;
        c->t_stop = -1;
        c->checks = 0;
        c->stop = STOP_RUN;
        c->since_best = 0;
        c->window = window;
        c->is_fluid = is_fluid;
        c->K = K;
        c->t_max = t_max;
    }
}

// Block-wide max of the per-tile maxima part_r[0..n), part_u[0..n); the
// result is valid in thread 0.
__device__ __forceinline__ void reduce_parts(const unsigned long long *part_r,
                                             const unsigned long long *part_u, int n,
                                             unsigned long long &mr_out, unsigned long long &mu_out)
{
    __shared__ unsigned long long sr[256], su[256];
    unsigned long long mr = 0ull, mu = 0ull;
    for (int b = threadIdx.x; b < n; b += 256) {
        const unsigned long long r = part_r[b], u = part_u[b];
        mr = r > mr ? r : mr;
        mu = u > mu ? u : mu;
    }
    sr[threadIdx.x] = mr;
    su[threadIdx.x] = mu;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sr[threadIdx.x] = sr[threadIdx.x + s] > sr[threadIdx.x] ? sr[threadIdx.x + s] : sr[threadIdx.x];
            su[threadIdx.x] = su[threadIdx.x + s] > su[threadIdx.x] ? su[threadIdx.x + s] : su[threadIdx.x];
        }
        __syncthreads();
    }
    mr_out = sr[0];
    mu_out = su[0];
}

// Stop rule after a check with residual bits rb and max |u| bits ub: OK at
// r <= tol; DIVERGED on NaN/Inf or |u| > 0.3 (fluid); STALLED after
// `window` checks that set neither a new maximum of r nor a new minimum
// since the last maximum (a flat round-off floor); MAXITER once t_max
// steps are covered.
__device__ void decide_apply(Ctrl *c, unsigned long long rb, unsigned long long ub)
{
    c->res_bits = rb;
    c->umax_bits = ub;
    c->t += c->K;
    c->checks += 1;
    const double r = __longlong_as_double((long long)rb);
    const double um = __longlong_as_double((long long)ub);
    c->r_last = r;
    int stop = STOP_RUN;
    if (r != r || isinf(r) || um != um || (c->is_fluid && um > 0.3)) {
        stop = STOP_DIVERGED;
    } else if (r <= c->tol) {
        stop = STOP_OK;
    } else if (r > c->peak) {
        c->peak = r;
        c->best = r;
        c->since_best = 0;
    } else if (r < c->best) {
        c->best = r;
        c->since_best = 0;
    } else {
        c->since_best += 1;
        if (c->window > 0 && c->since_best >= c->window)
            stop = STOP_STALLED;
    }
    if (stop == STOP_RUN && c->t >= c->t_max)
        stop = STOP_MAXITER;
    if (stop != STOP_RUN) {
        c->t_stop = c->t;
        c->stop = stop;
    }
}

__global__ void __launch_bounds__(256) k_decide(Ctrl *c)
{
    if (c->stop != STOP_RUN)
        return;
    const int np = c->nparts;
    unsigned long long mr, mu;
    reduce_parts(c->part, c->part + np, np, mr, mu);
    if (threadIdx.x == 0)
        decide_apply(c, mr, mu);
}

// ------------------------------------------------------ batched serving
// One launch advances every request of the slot table by the same number of
// steps: block b takes tile v of the table (XCD-banded numbering), finds the
// owning request by binary search over the tile offsets and runs the tile
// code of the single-domain kernels in that request's phase; blocks past the
// table's tiles exit.  The grid is a power of two at least the table's tile
// count (one captured graph per size).  All of this is uniform across the
// block.  Requests are 2-D (D2Q9 + D2Q5).  Every phase starts in buffer 0
// and a chunk has an even number of launches, so launch j of a chunk reads
// buffer j & 1.

// Table entry owning tile v (entries are in tile order)
__device__ __forceinline__ int srv_entry(const SrvTable *tab, int v)
{
    int lo = 0, hi = tab->n_active - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab->begin[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Step arguments of a slot in launch j of a chunk whose first step is step
__device__ __forceinline__ FluidArgs srv_fluid_args(const SrvSlot &sl, Ctrl *c, int j, unsigned int step)
{
    FluidArgs a;
    a.src = sl.f[j & 1];
    a.dst = sl.f[(j & 1) ^ 1];
    a.desc = sl.desc;
    a.uprev = sl.prev;
    a.ctrl = c;
    a.g = sl.g;
    a.omega = sl.omega_f;
    a.u_in = sl.u_in;
    a.inv_uin = sl.inv_uin;
    a.streaming_stores = 0;
    a.step = step;
    a.ref_src = sl.ref_cur;
    a.ref_dst = j == 0 ? sl.ref_next : sl.ref_cur;
    a.ref_out = sl.ref_next;
    return a;
}
__device__ __forceinline__ AdArgs srv_ad_args(const SrvSlot &sl, Ctrl *c, int j, unsigned int step)
{
    AdArgs a;
    a.src = sl.gp[j & 1];
    a.dst = sl.gp[(j & 1) ^ 1];
    a.desc = sl.desc;
    a.u = sl.u;
    a.cprev = sl.prev;
    a.ctrl = c;
    a.g = sl.g;
    a.omega = sl.omega_a;
    a.cin_s = sl.cin_s;
    a.cout_s = sl.cout_s;
    a.c_ref = sl.c_ref;
    a.k_sink = sl.k_sink;
    a.k_half = sl.k_half;
    a.inv_cin = sl.inv_cin;
    a.outlet = sl.outlet;
    a.streaming_stores = 0;
    a.step = step;
    a.c_in = sl.c_in;
    a.c_out = sl.c_out;
    a.ref_src = sl.ref_cur;
    a.ref_dst = j == 0 ? sl.ref_next : sl.ref_cur;
    a.ref_out = sl.ref_next;
    return a;
}

// Two steps (2j, 2j + 1 of the chunk) over 64 x 4 tiles, 256-thread blocks:
// every storage form.
template <class S, int MODE>
__global__ void __launch_bounds__(256) k_srv_step(const SrvSlot *__restrict__ slots,
                                                  const SrvTable *__restrict__ tab, Ctrl *ctrl,
                                                  unsigned long long *part, int part_cap, int j)
{
    typedef typename S::C C;
    constexpr int LF = pair_lds_bytes<C, 9>(), LA = pair_lds_bytes<C, 5>();
    __shared__ __align__(16) char smem[LF > LA ? LF : LA];
    const int v = xcd_tile(blockIdx.x, gridDim.x);
    if (v >= tab->total_tiles)
        return;
    const int e = srv_entry(tab, v);
    const int sid = tab->slot[e];
    const SrvSlot &sl = slots[sid];
    Ctrl *c = ctrl + sid;
    if (sl.phase == SRV_IDLE || c->stop != STOP_RUN)
        return;
    const int tile = v - tab->begin[e];
    const unsigned int step = (unsigned int)(c->t + 2 * j);
    if (sl.phase == SRV_FLUID)
        fluid_tile2<S, MODE, false>(srv_fluid_args(sl, c, j, step), tile, part + v, part + part_cap + v, smem);
    else
        ad_tile2<S, MODE, false>(srv_ad_args(sl, c, j, step), tile, part + v, part + part_cap + v, smem);
}

// NS steps (2 or 4) over 64 x 16 tiles, 1024-thread blocks: the FP32
// storage forms, with the wide paired or multi-step tile code of the single
// solves.  t_off is the launch's first step within the chunk.
template <class S, int MODE, int NS>
__global__ void __launch_bounds__(WIDE_NTH) k_srv_stepN(const SrvSlot *__restrict__ slots,
                                                        const SrvTable *__restrict__ tab, Ctrl *ctrl,
                                                        unsigned long long *part, int part_cap, int j,
                                                        int t_off)
{
    typedef typename S::C C;
    constexpr int H = NS - 1, NR = (WIDE_TY + 2 * H) * (64 + 2 * H);
    constexpr int LF = NS == 2 ? pair_lds_bytes<C, 9, WIDE_TY>() : multi_lds_bytes<C, WIDE_TY, NS>();
    constexpr int LA = NS == 2 ? pair_lds_bytes<C, 5, WIDE_TY>() : 5 * NR * (int)sizeof(C) + NR * 2;
    __shared__ __align__(16) char smem[LF > LA ? LF : LA];
    const int v = xcd_tile(blockIdx.x, gridDim.x);
    if (v >= tab->total_tiles)
        return;
    const int e = srv_entry(tab, v);
    const int sid = tab->slot[e];
    const SrvSlot &sl = slots[sid];
    Ctrl *c = ctrl + sid;
    if (sl.phase == SRV_IDLE || c->stop != STOP_RUN)
        return;
    const int tile = v - tab->begin[e];
    const unsigned int step = (unsigned int)(c->t + t_off);
    unsigned long long *pr = part + v, *pu = part + part_cap + v;
    if (sl.phase == SRV_FLUID) {
        const FluidArgs a = srv_fluid_args(sl, c, j, step);
        if constexpr (NS == 2)
            fluid_tile2<S, MODE, false, WIDE_TY, WIDE_NTH>(a, tile, pr, pu, smem);
        else
            fluid_tileN<S, MODE, false, WIDE_TY, WIDE_NTH, NS>(a, tile, pr, pu, smem);
    } else {
        const AdArgs a = srv_ad_args(sl, c, j, step);
        if constexpr (NS == 2)
            ad_tile2<S, MODE, false, D2Q5, 9, WIDE_TY, WIDE_NTH>(a, tile, pr, pu, smem);
        else
            ad_tileN<S, MODE, false, D2Q5, 9, WIDE_TY, WIDE_NTH, NS>(a, tile, pr, pu, smem);
    }
}

// One block per table entry: reduce that request's tile maxima of the check
// step and apply the stop rule to its control block.
__global__ void __launch_bounds__(256) k_srv_decide(const SrvSlot *__restrict__ slots,
                                                    const SrvTable *__restrict__ tab, Ctrl *ctrl,
                                                    const unsigned long long *part, int part_cap)
{
    const int e = blockIdx.x;
    if (e >= tab->n_active)
        return;
    const int sid = tab->slot[e];
    Ctrl *c = ctrl + sid;
    if (slots[sid].phase == SRV_IDLE || c->stop != STOP_RUN)
        return;
    const int b0 = tab->begin[e], n = tab->begin[e + 1] - b0;
    unsigned long long mr, mu;
    reduce_parts(part + b0, part + part_cap + b0, n, mr, mu);
    if (threadIdx.x == 0)
        decide_apply(c, mr, mu);
}

// Reference roll of every running request: one block per table entry.
__global__ void __launch_bounds__(256) k_srv_ref_roll(const SrvSlot *__restrict__ slots,
                                                      const SrvTable *__restrict__ tab,
                                                      const Ctrl *ctrl)
{
    const int e = blockIdx.x;
    if (e >= tab->n_active)
        return;
    const int sid = tab->slot[e];
    const SrvSlot &sl = slots[sid];
    if (sl.phase == SRV_IDLE || ctrl[sid].stop != STOP_RUN)
        return;
    for (int x = threadIdx.x; x < sl.g.nx; x += 256)
        sl.ref_cur[x] = sl.ref_next[x];
}

__global__ void k_srv_slot_set(SrvSlot *slots, int sid, SrvSlot v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        slots[sid] = v;
}

__global__ void k_srv_table_set(SrvTable *tab, SrvTable v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *tab = v;
}

// Plain streaming copy used to calibrate bandwidth and counters: each block
// moves 16 KiB (four 16-byte vectors per thread, all loads issued first).
__global__ void __launch_bounds__(256) k_copy(const float4 *__restrict__ src,
                                              float4 *__restrict__ dst, long long n4)
{
    const long long base = blockIdx.x * 1024ll + threadIdx.x;
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long i = base + 256ll * k;
        if (i < n4)
            v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long i = base + 256ll * k;
        if (i < n4)
            dst[i] = v[k];
    }
}

// ------------------------------------------------------------ dispatch
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

size_t storage_bytes(int s)
{
    return s == ST_F64 ? 8 : (s == ST_F16S ? 2 : 4);
}
size_t compute_bytes(int s)
{
    return s == ST_F64 ? 8 : 4;
}
bool storage_shifted(int s)
{
    return s == ST_F32S || s == ST_F16S || s == ST_F32X;
}
bool storage_moving_ref(int s)
{
    return s == ST_F16S;
}

static inline dim3 flat_grid(long long N)
{
    return dim3((unsigned)((N + 255) / 256));
}

template <class F>
static hipError_t by_storage(int storage, F &&fn)
{
    switch (storage) {
    case ST_F32:
        return fn(SF32{});
    case ST_F32S:
        return fn(SF32S{});
    case ST_F16S:
        return fn(SF16S{});
    case ST_F64:
        return fn(SF64{});
    case ST_F32X:
        return fn(SF32X{});
    default:
        return hipErrorInvalidValue;
    }
}

template <class LF, class LA, class DT, class F>
static hipError_t with_lattices(F &&fn)
{
    return fn(LF{}, LA{}, DT{});
}

template <class F>
static hipError_t by_dim(int dim, F &&fn)
{
    if (dim == 2)
        return fn(D2Q9{}, D2Q5{}, uint16_t{});
    if (dim == 3)
        return fn(D3Q19{}, D3Q7{}, uint32_t{});
    return hipErrorInvalidValue;
}

// Lattices of a layout code for substrate calls: 2 and 3 as by_dim, or
// LAY_2D_AD9, the D2Q9 substrate with its own 16-bit words (no fluid bits)
template <class F>
static hipError_t by_lay(int lay, F &&fn)
{
    if (lay == LAY_2D_AD9)
        return fn(NoFluid{}, D2Q9{}, uint16_t{});
    return by_dim(lay, fn);
}

hipError_t fluid_step(int dim, int storage, int mode, const FluidArgs &a, hipStream_t st)
{
    return by_dim(dim, [&](auto lf, auto, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            dim3 grid(a.g.ntiles), block(256);
            const bool nt = a.streaming_stores != 0;
            constexpr bool B = sizeof(typename S::T) <= 4;
            const bool buf = B && (unsigned long long)LF::Q * (unsigned long long)a.g.N *
                                          sizeof(typename S::T) <= 0xFFFFFFFFull;
#define LBM_FLUID_LAUNCH(M, NTV)                                                                  \
    do {                                                                                          \
        if (buf)                                                                                  \
            hipLaunchKernelGGL((k_fluid_step<LF, S, DT, M, NTV, B>), grid, block, 0, st, a);    \
        else                                                                                      \
            hipLaunchKernelGGL((k_fluid_step<LF, S, DT, M, NTV, false>), grid, block, 0, st, a);\
    } while (0)
            if (mode == MODE_CHECK) {
                if (nt)
                    LBM_FLUID_LAUNCH(MODE_CHECK, true);
                else
                    LBM_FLUID_LAUNCH(MODE_CHECK, false);
            } else {
                if (nt)
                    LBM_FLUID_LAUNCH(MODE_PLAIN, true);
                else
                    LBM_FLUID_LAUNCH(MODE_PLAIN, false);
            }
#undef LBM_FLUID_LAUNCH
            return hipGetLastError();
        });
    });
}

int pair_tiles(const Geo &g, int ty)
{
    return g.ntx * ((g.ny + ty - 1) / ty) * g.nz;
}
int pair_tiles(const Geo &g)
{
    return pair_tiles(g, PAIR_TY);
}

int pair_ty(int storage, const Geo &g)
{
    // FP16 storage (the only one with tile means) keeps 64 x 4
    const bool means = storage == ST_F16S;
    static_assert(SF16S::tile_mean && !SF32S::tile_mean && !SF32::tile_mean && !SF64::tile_mean,
                  "tile means are FP16 storage's alone");
    if (means)
        return PAIR_TY;
    if (pair_tiles(g, WIDE_TY) >= WIDE_MIN_TILES)
        return WIDE_TY;
    return pair_tiles(g, MID_TY) >= MID_MIN_TILES ? MID_TY : PAIR_TY;
}

hipError_t fluid_step2(int storage, int mode, const FluidArgs &a, hipStream_t st)
{
    const int ty = pair_ty(storage, a.g);
    return by_storage(storage, [&](auto s) -> hipError_t {
        typedef decltype(s) S;
        auto go = [&](auto ty, auto nth) {
            constexpr int TY = decltype(ty)::value, NTH = decltype(nth)::value;
            const dim3 grid(pair_tiles(a.g, TY));
            if (a.streaming_stores) {
                if (mode == MODE_CHECK)
                    hipLaunchKernelGGL((k_fluid_step2<S, MODE_CHECK, true, TY, NTH>), grid, dim3(NTH), 0, st, a);
                else
                    hipLaunchKernelGGL((k_fluid_step2<S, MODE_PLAIN, true, TY, NTH>), grid, dim3(NTH), 0, st, a);
            } else {
                if (mode == MODE_CHECK)
                    hipLaunchKernelGGL((k_fluid_step2<S, MODE_CHECK, false, TY, NTH>), grid, dim3(NTH), 0, st, a);
                else
                    hipLaunchKernelGGL((k_fluid_step2<S, MODE_PLAIN, false, TY, NTH>), grid, dim3(NTH), 0, st, a);
            }
        };
        if constexpr (S::tile_mean) {
            go(std::integral_constant<int, PAIR_TY>{}, std::integral_constant<int, 256>{});
        } else {
            if (ty == WIDE_TY)
                go(std::integral_constant<int, WIDE_TY>{}, std::integral_constant<int, WIDE_NTH>{});
            else if (ty == MID_TY)
                go(std::integral_constant<int, MID_TY>{}, std::integral_constant<int, MID_NTH>{});
            else
                go(std::integral_constant<int, PAIR_TY>{}, std::integral_constant<int, 256>{});
        }
        return hipGetLastError();
    });
}

// Tile height of the multi-step launches on grid g: 16 (1024-thread
// blocks) or 8 (512), as the FP32 forms' paired launches take; 0 where the
// grid is too small for them.  Storage with tile means runs its checks as
// 64 x 4 paired launches and its plain launches at this height.
int multi_ty(const Geo &g)
{
    if (pair_tiles(g, WIDE_TY) >= WIDE_MIN_TILES)
        return WIDE_TY;
    return pair_tiles(g, MID_TY) >= MID_MIN_TILES ? MID_TY : 0;
}

int fluid_launch_steps(int storage, const Geo &g)
{
    // FP64 keeps paired launches (its staged values would exceed the
    // register budget of full occupancy)
    return storage != ST_F64 && multi_ty(g) ? MULTI_NS : 2;
}

// Multi-step launch of one solver: FP32 forms take three or four steps,
// either mode; storage that rounds on store takes four, plain, with equal
// source and destination references (see fluid_tileN).  K(NS, MODE, NT)
// launches the kernel instance.
template <class S, class K>
hipError_t launch_multi(int mode, int ns, bool nt, const void *ref_src, const void *ref_dst, K k)
{
    if constexpr (sizeof(typename S::C) != 4) {
        return hipErrorInvalidValue;
    } else {
        if (rounds_on_store<S>() && (ns != 4 || mode != MODE_PLAIN || ref_src != ref_dst))
            return hipErrorInvalidValue;
        auto go = [&](auto nsc, auto mc, auto ntc) -> hipError_t {
            constexpr int NS = decltype(nsc)::value, M = decltype(mc)::value;
            if constexpr ((rounds_on_store<S>() && NS % 2) || (S::tile_mean && M != MODE_PLAIN)) {
                return hipErrorInvalidValue;
            } else {
                k(nsc, mc, ntc);
                return hipGetLastError();
            }
        };
        auto by_nt = [&](auto nsc, auto mc) {
            return nt ? go(nsc, mc, std::true_type{}) : go(nsc, mc, std::false_type{});
        };
        auto by_mode = [&](auto nsc) {
            return mode == MODE_CHECK ? by_nt(nsc, std::integral_constant<int, MODE_CHECK>{})
                                      : by_nt(nsc, std::integral_constant<int, MODE_PLAIN>{});
        };
        return ns == 4 ? by_mode(std::integral_constant<int, 4>{}) : by_mode(std::integral_constant<int, 3>{});
    }
}

hipError_t fluid_stepN(int storage, int mode, int ns, const FluidArgs &a, hipStream_t st)
{
    if (fluid_launch_steps(storage, a.g) < 3 || ns < 3 || ns > MULTI_NS)
        return hipErrorInvalidValue;
    const bool wide = multi_ty(a.g) == WIDE_TY;
    const dim3 grid(pair_tiles(a.g, wide ? WIDE_TY : MID_TY));
    return by_storage(storage, [&](auto s) -> hipError_t {
        typedef decltype(s) S;
        return launch_multi<S>(mode, ns, a.streaming_stores, a.ref_src, a.ref_dst, [&](auto nsc, auto mc, auto ntc) {
            constexpr int NS = decltype(nsc)::value, M = decltype(mc)::value;
            constexpr bool NT = decltype(ntc)::value;
            if (wide)
                hipLaunchKernelGGL((k_fluid_stepN<S, M, NT, WIDE_TY, WIDE_NTH, NS>), grid, dim3(WIDE_NTH), 0, st, a);
            else
                hipLaunchKernelGGL((k_fluid_stepN<S, M, NT, MID_TY, MID_NTH, NS>), grid, dim3(MID_NTH), 0, st, a);
        });
    });
}

hipError_t ad_stepN(int lay, int storage, int mode, int ns, const AdArgs &a, hipStream_t st)
{
    if (fluid_launch_steps(storage, a.g) < 3 || ns < 3 || ns > MULTI_NS)
        return hipErrorInvalidValue;
    const bool wide = multi_ty(a.g) == WIDE_TY;
    const dim3 grid(pair_tiles(a.g, wide ? WIDE_TY : MID_TY));
    return by_storage(storage, [&](auto s) -> hipError_t {
        typedef decltype(s) S;
        return launch_multi<S>(mode, ns, a.streaming_stores, a.ref_src, a.ref_dst, [&](auto nsc, auto mc, auto ntc) {
            constexpr int NS = decltype(nsc)::value, M = decltype(mc)::value;
            constexpr bool NT = decltype(ntc)::value;
            auto go = [&](auto la, auto qf) {
                typedef decltype(la) L;
                constexpr int QF = decltype(qf)::value;
                if (wide)
                    hipLaunchKernelGGL((k_ad_stepN<S, M, NT, L, QF, WIDE_TY, WIDE_NTH, NS>), grid, dim3(WIDE_NTH), 0,
                                       st, a);
                else
                    hipLaunchKernelGGL((k_ad_stepN<S, M, NT, L, QF, MID_TY, MID_NTH, NS>), grid, dim3(MID_NTH), 0,
                                       st, a);
            };
            if (lay == LAY_2D_AD9)
                go(D2Q9{}, std::integral_constant<int, 1>{});
            else
                go(D2Q5{}, std::integral_constant<int, 9>{});
        });
    });
}

// Two-step 3-D launches: column height, output planes per block, and
// blocks.  32 x 16 columns (512 threads, 88 KB of LDS for the fluid: one
// block per CU) recompute 1.2x the column in the first step, 32 x 8 (256
// threads, 49 KB) 1.3x.  The planes per block are chosen so that the grid is
// about one round of resident blocks, at least 4 (on 256 x 128 x 128 with
// 32 x 16 columns: 64 columns x 4 segments of 32 planes).  The environment
// variable LBM_3D_TILE_Y (8 or 16) overrides the column height (tuning).
int z3_tile_y(const Geo &g)
{
    (void)g;
    if (const char *e = getenv("LBM_3D_TILE_Y"))
        if (atoi(e) == 8 || atoi(e) == 16)
            return atoi(e);
    return 16;
}
int z3_planes_per_block(const Geo &g, int ty, int blocks_per_cu)
{
    const int ncol = ((g.nx + Z3_TX - 1) / Z3_TX) * ((g.ny + ty - 1) / ty);
    const int want = 256 * blocks_per_cu;
    int nseg = (want + ncol / 2) / ncol;
    nseg = nseg < 1 ? 1 : nseg;
    int zs = (g.nz + nseg - 1) / nseg;
    return zs < 4 ? (g.nz < 4 ? g.nz : 4) : zs;
}
int z3_blocks(const Geo &g, int zseg, int ty)
{
    const int ncol = ((g.nx + Z3_TX - 1) / Z3_TX) * ((g.ny + ty - 1) / ty);
    return ncol * ((g.nz + zseg - 1) / zseg);
}

template <class S, class K>
static hipError_t launch_z3(int mode, const Geo &g, int zseg, int ty, bool nt, unsigned long long n_elems, K k)
{
    if constexpr (sizeof(typename S::C) != 4) {
        return hipErrorInvalidValue;
    } else {
        if (g.nz < 3 || zseg < 1 || (ty != 8 && ty != 16) || (S::tile_mean && mode != MODE_PLAIN))
            return hipErrorInvalidValue;
        const dim3 grid(z3_blocks(g, zseg, ty));
        // z3_store addresses up to (2Q - 1) N elements from the buffer start
        const bool buf = 2ull * n_elems * sizeof(typename S::T) <= 0xFFFFFFFFull;
        auto go = [&](auto mc, auto ntc, auto bc) {
            constexpr int M = decltype(mc)::value;
            if constexpr (!(S::tile_mean && M != MODE_PLAIN)) {
                if (ty == 16)
                    k(mc, ntc, bc, std::integral_constant<int, 16>{}, grid);
                else
                    k(mc, ntc, bc, std::integral_constant<int, 8>{}, grid);
            }
        };
        auto by_buf = [&](auto mc, auto ntc) {
            if (buf)
                go(mc, ntc, std::true_type{});
            else
                go(mc, ntc, std::false_type{});
        };
        auto by_nt = [&](auto mc) {
            if (nt)
                by_buf(mc, std::true_type{});
            else
                by_buf(mc, std::false_type{});
        };
        if (mode == MODE_CHECK)
            by_nt(std::integral_constant<int, MODE_CHECK>{});
        else
            by_nt(std::integral_constant<int, MODE_PLAIN>{});
        return hipGetLastError();
    }
}

hipError_t fluid_step3d2(int storage, int mode, const FluidArgs &a, hipStream_t st)
{
    return by_storage(storage, [&](auto s) -> hipError_t {
        typedef decltype(s) S;
        return launch_z3<S>(mode, a.g, a.zseg, a.ty3, a.streaming_stores != 0, 19ull * (unsigned long long)a.g.N,
                            [&](auto mc, auto ntc, auto bc, auto tyc, dim3 grid) {
                                constexpr int M = decltype(mc)::value, TY = decltype(tyc)::value;
                                constexpr bool NT = decltype(ntc)::value, B = decltype(bc)::value;
                                hipLaunchKernelGGL((k_fluid_step3d2<S, M, NT, B, TY>), grid, dim3(Z3T<TY>::NTH), 0,
                                                   st, a);
                            });
    });
}

hipError_t ad_step3d2(int storage, int mode, const AdArgs &a, hipStream_t st)
{
    return by_storage(storage, [&](auto s) -> hipError_t {
        typedef decltype(s) S;
        return launch_z3<S>(mode, a.g, a.zseg, a.ty3, a.streaming_stores != 0, 7ull * (unsigned long long)a.g.N,
                            [&](auto mc, auto ntc, auto bc, auto tyc, dim3 grid) {
                                constexpr int M = decltype(mc)::value, TY = decltype(tyc)::value;
                                constexpr bool NT = decltype(ntc)::value, B = decltype(bc)::value;
                                hipLaunchKernelGGL((k_ad_step3d2<S, M, NT, B, TY>), grid, dim3(Z3T<TY>::NTH), 0, st,
                                                   a);
                            });
    });
}

hipError_t ad_step2(int lay, int storage, int mode, const AdArgs &a, hipStream_t st)
{
    const int ty = pair_ty(storage, a.g);
    return by_storage(storage, [&](auto s) -> hipError_t {
        typedef decltype(s) S;
        auto go = [&](auto la, auto qf, auto ty, auto nth) {
            typedef decltype(la) L;
            constexpr int QF = decltype(qf)::value;
            constexpr int TY = decltype(ty)::value, NTH = decltype(nth)::value;
            const dim3 grid(pair_tiles(a.g, TY));
            if (a.streaming_stores) {
                if (mode == MODE_CHECK)
                    hipLaunchKernelGGL((k_ad_step2<S, MODE_CHECK, true, L, QF, TY, NTH>), grid, dim3(NTH), 0, st, a);
                else
                    hipLaunchKernelGGL((k_ad_step2<S, MODE_PLAIN, true, L, QF, TY, NTH>), grid, dim3(NTH), 0, st, a);
            } else {
                if (mode == MODE_CHECK)
                    hipLaunchKernelGGL((k_ad_step2<S, MODE_CHECK, false, L, QF, TY, NTH>), grid, dim3(NTH), 0, st, a);
                else
                    hipLaunchKernelGGL((k_ad_step2<S, MODE_PLAIN, false, L, QF, TY, NTH>), grid, dim3(NTH), 0, st, a);
            }
        };
        auto shape = [&](auto la, auto qf) {
            if constexpr (S::tile_mean) {
                go(la, qf, std::integral_constant<int, PAIR_TY>{}, std::integral_constant<int, 256>{});
            } else {
                if (ty == WIDE_TY)
                    go(la, qf, std::integral_constant<int, WIDE_TY>{}, std::integral_constant<int, WIDE_NTH>{});
                else if (ty == MID_TY)
                    go(la, qf, std::integral_constant<int, MID_TY>{}, std::integral_constant<int, MID_NTH>{});
                else
                    go(la, qf, std::integral_constant<int, PAIR_TY>{}, std::integral_constant<int, 256>{});
            }
        };
        if (lay == LAY_2D_AD9)
            shape(D2Q9{}, std::integral_constant<int, 1>{});
        else
            shape(D2Q5{}, std::integral_constant<int, 9>{});
        return hipGetLastError();
    });
}

hipError_t ad_step(int dim, int storage, int mode, const AdArgs &a, hipStream_t st)
{
    return by_lay(dim, [&](auto lf, auto la, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            dim3 grid(a.g.ntiles), block(256);
            const bool nt = a.streaming_stores != 0;
            constexpr bool B = sizeof(typename S::T) <= 4;
            const bool buf = B && (unsigned long long)LA::Q * (unsigned long long)a.g.N *
                                          sizeof(typename S::T) <= 0xFFFFFFFFull;
#define LBM_AD_LAUNCH(M, NTV)                                                                     \
    do {                                                                                          \
        if (buf)                                                                                  \
            hipLaunchKernelGGL((k_ad_step<LA, LF::Q, S, DT, M, NTV, B>), grid, block, 0, st, a);\
        else                                                                                      \
            hipLaunchKernelGGL((k_ad_step<LA, LF::Q, S, DT, M, NTV, false>), grid, block, 0, st,  \
                               a);                                                                \
    } while (0)
            if (mode == MODE_CHECK) {
                if (nt)
                    LBM_AD_LAUNCH(MODE_CHECK, true);
                else
                    LBM_AD_LAUNCH(MODE_CHECK, false);
            } else {
                if (nt)
                    LBM_AD_LAUNCH(MODE_PLAIN, true);
                else
                    LBM_AD_LAUNCH(MODE_PLAIN, false);
            }
#undef LBM_AD_LAUNCH
            return hipGetLastError();
        });
    });
}

hipError_t fluid_init(int dim, int storage, void *f, const void *desc, const Geo &g,
                      hipStream_t st)
{
    return by_dim(dim, [&](auto lf, auto, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            hipLaunchKernelGGL((k_fluid_init<LF, S, DT>), flat_grid(g.N), dim3(256), 0, st,
                               static_cast<typename S::T *>(f), static_cast<const DT *>(desc), g.N);
            return hipGetLastError();
        });
    });
}

hipError_t ad_init(int dim, int storage, void *gp, const void *desc, const void *u,
                   const Geo &g, double c_init, double c_ref, hipStream_t st)
{
    return by_lay(dim, [&](auto lf, auto la, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            hipLaunchKernelGGL((k_ad_init<LA, LF::Q, S, DT>), flat_grid(g.N), dim3(256), 0, st,
                               static_cast<typename S::T *>(gp), static_cast<const DT *>(desc),
                               static_cast<const typename S::C *>(u), g.N, c_init,
                               S::shifted ? c_ref : 0.0);
            return hipGetLastError();
        });
    });
}

hipError_t fluid_export(int dim, int storage, const void *f, const void *desc, const Geo &g,
                        const float *ref, void *U, void *RHO, int out_double, hipStream_t st)
{
    return by_dim(dim, [&](auto lf, auto, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            typedef typename S::C C;
            if (out_double)
                hipLaunchKernelGGL((k_fluid_export<LF, S, DT, double>), flat_grid(g.N), dim3(256), 0,
                                   st, static_cast<const typename S::T *>(f),
                                   static_cast<const DT *>(desc), g.N, ref, g.nx,
                                   static_cast<double *>(U), static_cast<double *>(RHO));
            else
                hipLaunchKernelGGL((k_fluid_export<LF, S, DT, C>), flat_grid(g.N), dim3(256), 0, st,
                                   static_cast<const typename S::T *>(f),
                                   static_cast<const DT *>(desc), g.N, ref, g.nx,
                                   static_cast<C *>(U), static_cast<C *>(RHO));
            return hipGetLastError();
        });
    });
}

hipError_t ad_export(int dim, int storage, const void *gp, const void *desc, const Geo &g,
                     const float *ref, Sink sink, void *C, int out_double, hipStream_t st)
{
    return by_lay(dim, [&](auto lf, auto la, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            typedef typename S::C CT;
            if (out_double)
                hipLaunchKernelGGL((k_ad_export<LA, LF::Q, S, DT, double>), flat_grid(g.N), dim3(256),
                                   0, st, static_cast<const typename S::T *>(gp),
                                   static_cast<const DT *>(desc), g.N, ref, g.nx, sink,
                                   static_cast<double *>(C));
            else
                hipLaunchKernelGGL((k_ad_export<LA, LF::Q, S, DT, CT>), flat_grid(g.N), dim3(256), 0,
                                   st, static_cast<const typename S::T *>(gp),
                                   static_cast<const DT *>(desc), g.N, ref, g.nx, sink,
                                   static_cast<CT *>(C));
            return hipGetLastError();
        });
    });
}

hipError_t pops_export(int which, int dim, int storage, const void *h, const void *desc,
                       const Geo &g, const float *ref, double *out, hipStream_t st)
{
    return by_lay(dim, [&](auto lf, auto la, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            const typename S::T *hp = static_cast<const typename S::T *>(h);
            const DT *dp = static_cast<const DT *>(desc);
            if constexpr (LF::Q > 1) {
                if (which == 0) {
                    hipLaunchKernelGGL((k_pops_export<LF, S, DT>), flat_grid(g.N), dim3(256), 0, st, hp,
                                       dp, g.N, 0, ref, g.nx, out);
                    return hipGetLastError();
                }
            }
            if (which == 0)
                return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_pops_export<LA, S, DT>), flat_grid(g.N), dim3(256), 0, st, hp,
                                   dp, g.N, LF::Q - 1 + LA::Q, ref, g.nx, out);
            return hipGetLastError();
        });
    });
}

hipError_t pops_import(int which, int dim, int storage, void *h, const void *desc,
                       const Geo &g, const float *ref, const double *in, hipStream_t st)
{
    return by_lay(dim, [&](auto lf, auto la, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            typename S::T *hp = static_cast<typename S::T *>(h);
            const DT *dp = static_cast<const DT *>(desc);
            if constexpr (LF::Q > 1) {
                if (which == 0) {
                    hipLaunchKernelGGL((k_pops_import<LF, S, DT>), flat_grid(g.N), dim3(256), 0, st, hp,
                                       dp, g.N, 0, ref, g.nx, in);
                    return hipGetLastError();
                }
            }
            if (which == 0)
                return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_pops_import<LA, S, DT>), flat_grid(g.N), dim3(256), 0, st, hp,
                                   dp, g.N, LF::Q - 1 + LA::Q, ref, g.nx, in);
            return hipGetLastError();
        });
    });
}

hipError_t pops_set_nodes(int which, int dim, int storage, void *h, const Geo &g,
                          const float *ref, const long long *idx, int count, const double *vals_q,
                          hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    return by_lay(dim, [&](auto lf, auto la, auto) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typename S::T *hp = static_cast<typename S::T *>(h);
            if constexpr (LF::Q > 1) {
                if (which == 0) {
                    hipLaunchKernelGGL((k_pops_set_nodes<LF, S>), dim3((count + 255) / 256), dim3(256), 0,
                                       st, hp, g.N, ref, g.nx, idx, count, vals_q);
                    return hipGetLastError();
                }
            }
            if (which == 0)
                return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_pops_set_nodes<LA, S>), dim3((count + 255) / 256), dim3(256), 0,
                                   st, hp, g.N, ref, g.nx, idx, count, vals_q);
            return hipGetLastError();
        });
    });
}

hipError_t ref_fill(float *ref, int n, float v, hipStream_t st)
{
    hipLaunchKernelGGL(k_ref_fill, dim3((n + 255) / 256), dim3(256), 0, st, ref, n, v);
    return hipGetLastError();
}

hipError_t ref_roll(const Ctrl *ctrl, float *cur, const float *next, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_ref_roll, dim3((n + 255) / 256), dim3(256), 0, st, ctrl, cur, next, n);
    return hipGetLastError();
}

hipError_t fluxes(int dim, int storage, const void *f, const void *gp, const void *desc,
                  const Geo &g, const float *ref_f, const float *ref_g, double u_in, double c_in,
                  Sink sink, int outlet, double c_out, const void *u, double *partials,
                  double *out5, hipStream_t st)
{
    hipError_t e = by_lay(dim, [&](auto lf, auto la, auto dt) {
        return by_storage(storage, [&](auto s) {
            typedef decltype(lf) LF;
            typedef decltype(la) LA;
            typedef decltype(s) S;
            typedef decltype(dt) DT;
            hipLaunchKernelGGL((k_flux_partials<LF, LA, S, DT>), dim3(FLUX_BLOCKS), dim3(256), 0, st,
                               static_cast<const typename S::T *>(f),
                               static_cast<const typename S::T *>(gp), static_cast<const DT *>(desc),
                               g, ref_f, ref_g, u_in, c_in, sink, outlet, c_out,
                               static_cast<const typename S::C *>(u), partials);
            return hipGetLastError();
        });
    });
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_flux_final, dim3(1), dim3(320), 0, st, partials, (int)FLUX_BLOCKS, out5);
    return hipGetLastError();
}

hipError_t ctrl_reset(Ctrl *c, double tol, int window, int is_fluid, int K,
                      unsigned long long *part, int nparts, hipStream_t st, long long t_max)
{
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, c, tol, window, is_fluid, K, part,
                       nparts, t_max);
    return hipGetLastError();
}

hipError_t srv_step(int storage, int mode, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                    unsigned long long *part, int part_cap, int j, int blocks, hipStream_t st)
{
    auto go = [&](auto sp) -> hipError_t {
        typedef decltype(sp) S;
        if (mode == MODE_CHECK)
            hipLaunchKernelGGL((k_srv_step<S, MODE_CHECK>), dim3(blocks), dim3(256), 0, st, slots,
                               tab, ctrl, part, part_cap, j);
        else
            hipLaunchKernelGGL((k_srv_step<S, MODE_PLAIN>), dim3(blocks), dim3(256), 0, st, slots,
                               tab, ctrl, part, part_cap, j);
        return hipGetLastError();
    };
    switch (storage) {
    case ST_F32:
        return go(SF32());
    case ST_F32S:
        return go(SF32S());
    case ST_F16S:
        return go(SF16S());
    case ST_F32X:
        return go(SF32X());
    default:
        return hipErrorInvalidValue;
    }
}

// FP32 and FP32-shifted requests are served over 64 x 16 tiles (srv_stepN,
// up to four steps per launch); FP16 storage keeps the 64 x 4 tiles of its
// tile means, and FP32 storage with FP64 arithmetic the paired 64 x 4 form.
int srv_tile_ty(int storage)
{
    return storage == ST_F32 || storage == ST_F32S ? WIDE_TY : PAIR_TY;
}

hipError_t srv_stepN(int storage, int mode, int ns, const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                     unsigned long long *part, int part_cap, int j, int t_off, int blocks, hipStream_t st)
{
    if (srv_tile_ty(storage) != WIDE_TY || (ns != 2 && ns != MULTI_NS))
        return hipErrorInvalidValue;
    auto go = [&](auto sp) -> hipError_t {
        typedef decltype(sp) S;
        if (ns == 2) {
            if (mode == MODE_CHECK)
                hipLaunchKernelGGL((k_srv_stepN<S, MODE_CHECK, 2>), dim3(blocks), dim3(WIDE_NTH), 0, st, slots,
                                   tab, ctrl, part, part_cap, j, t_off);
            else
                hipLaunchKernelGGL((k_srv_stepN<S, MODE_PLAIN, 2>), dim3(blocks), dim3(WIDE_NTH), 0, st, slots,
                                   tab, ctrl, part, part_cap, j, t_off);
        } else {
            if (mode == MODE_CHECK)
                hipLaunchKernelGGL((k_srv_stepN<S, MODE_CHECK, MULTI_NS>), dim3(blocks), dim3(WIDE_NTH), 0, st,
                                   slots, tab, ctrl, part, part_cap, j, t_off);
            else
                hipLaunchKernelGGL((k_srv_stepN<S, MODE_PLAIN, MULTI_NS>), dim3(blocks), dim3(WIDE_NTH), 0, st,
                                   slots, tab, ctrl, part, part_cap, j, t_off);
        }
        return hipGetLastError();
    };
    return storage == ST_F32 ? go(SF32()) : go(SF32S());
}

hipError_t srv_decide(const SrvSlot *slots, const SrvTable *tab, Ctrl *ctrl,
                      const unsigned long long *part, int part_cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_srv_decide, dim3(SRV_MAX_SLOTS), dim3(256), 0, st, slots, tab, ctrl, part,
                       part_cap);
    return hipGetLastError();
}

hipError_t srv_ref_roll(const SrvSlot *slots, const SrvTable *tab, const Ctrl *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_srv_ref_roll, dim3(SRV_MAX_SLOTS), dim3(256), 0, st, slots, tab, ctrl);
    return hipGetLastError();
}

hipError_t srv_slot_set(SrvSlot *slots, int sid, const SrvSlot &v, hipStream_t st)
{
    hipLaunchKernelGGL(k_srv_slot_set, dim3(1), dim3(64), 0, st, slots, sid, v);
    return hipGetLastError();
}

hipError_t srv_table_set(SrvTable *tab, const SrvTable &v, hipStream_t st)
{
    hipLaunchKernelGGL(k_srv_table_set, dim3(1), dim3(64), 0, st, tab, v);
    return hipGetLastError();
}

hipError_t decide(Ctrl *c, hipStream_t st)
{
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, st, c);
    return hipGetLastError();
}

hipError_t copy_kernel(const void *src, void *dst, size_t bytes, hipStream_t st)
{
    const long long n4 = (long long)(bytes / 16);
    const long long blocks = (n4 + 1023) / 1024;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const float4 *>(src), static_cast<float4 *>(dst), n4);
    return hipGetLastError();
}

} // namespace lbmk

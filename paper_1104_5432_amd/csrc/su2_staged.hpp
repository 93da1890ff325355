// su2_staged.hpp -- slab plan and index arithmetic of the LDS-staged update
// kernels (su2_staged.hip).  Host and device share these functions, so the
// host test of the index arithmetic runs exactly what the kernels run.
//
// A class (mu, parity) is cut into slabs: every x, a range of A rows in y,
// a range of B in a third dimension b, marched slice by slice along a fourth
// dimension s (s = t, b = z for mu = x, y, z; s = z, b = t for mu = t).
// While a block updates slice s, its LDS holds four arrays:
//   0: the s-direction links of slices s-1 and s (both parities),
//   1, 2: the links of the two directions other than mu and s, slice s
//         (both parities; the lower-numbered direction is array 1),
//   3: the mu-links of the opposite parity, slices s-1, s, s+1,
// each over the slab's A x B rows plus the one-row halo in y and b that the
// staples reach; rows hold all x (Nx/2 checkerboard entries per parity).
#pragma once

#include "su2_device.hpp"

namespace su2 {

constexpr int kStagedThreads = 512; // threads per block; at most one update per thread and slice
// The two-threads-per-site overrelaxation: at most 2 x 512 threads, each
// holding up to 5 links of the next slices' loads (the plan's at most
// 512 x 10 links per slice).
constexpr int kStagedPairThreads = 1024;
constexpr int kStagedPairPrefetch = 5;

// Next-slice links a thread holds in registers: 16-byte links 10, 32-byte 6.
__host__ __device__ constexpr int staged_prefetch(uint32_t link_bytes)
{
    return link_bytes <= 16 ? 10 : 6;
}

// One staged array inside the block's LDS (in links).
struct ArrayShape {
    uint32_t base;  // first element
    uint32_t ra;    // rows per b position: A + halo in y
    uint32_t rows;  // ra x (B + halo in b)
    uint32_t lo_a, lo_b;
    uint32_t count; // elements: rows x nxh x slots x parities
};

struct StagePlan {
    uint32_t A, B, S;    // slab: rows in y, extent in b, slices per chunk
    uint32_t na, nb, ns; // slabs: Ny / A, Nb / B, Ns / S
    uint32_t nxh;        // Nx / 2
    uint32_t lds_bytes;  // dynamic LDS per block
    uint32_t n_fresh;    // links a block loads per slice (arrays 0-2 of the
                         // slice, array 3 of the next)
    ArrayShape arr[4];   // the four arrays (array_shape)
    // divisions by run-time constants of the load decoding: by nxh, by the
    // links of one parity of array k (rows x nxh) and by its row length ra
    FastDiv div_nxh, div_pp[4], div_ra[4];
};

// Roles of the dimensions in class MU: b is the slab's third dimension, s
// the marched one; slot(d) is the position of direction d in (x, y, b, s).
template <int MU>
struct Roles {
    static constexpr int b = MU == 3 ? 3 : 2;
    static constexpr int s = MU == 3 ? 2 : 3;
    __host__ __device__ static constexpr int slot(int d) { return d == 0 ? 0 : (d == 1 ? 1 : (d == b ? 2 : 3)); }
};

// The staged arrays of class MU.
template <int MU>
struct Arrays {
    using R = Roles<MU>;
    // direction held by array k
    __host__ __device__ static constexpr int dir(int k)
    {
        return k == 0 ? R::s : (k == 3 ? MU : other(k - 1));
    }
    // the i-th (0 or 1) direction of {0, 1, b} other than MU, increasing
    __host__ __device__ static constexpr int other(int i)
    {
        int seen = 0;
        for (int d = 0; d < 4; ++d) {
            if (d == MU || d == R::s)
                continue;
            if (seen == i)
                return d;
            ++seen;
        }
        return -1;
    }
    __host__ __device__ static constexpr int array_of(int d)
    {
        return d == MU ? 3 : (d == R::s ? 0 : (d == other(0) ? 1 : 2));
    }
    __host__ __device__ static constexpr int slots(int k) { return k == 0 ? 2 : (k == 3 ? 3 : 1); }
    __host__ __device__ static constexpr int parities(int k) { return k == 3 ? 1 : 2; }
    // Halo rows of array k below (lo) and above (hi) the slab in lattice
    // dimension d (1 = y or R::b).  The staples take the s-direction links
    // at x and x + mu; a direction nu at x, x + mu, x - nu and x + mu - nu;
    // the opposite-parity mu-links at x +- nu for every nu != mu.
    __host__ __device__ static constexpr int lo(int k, int d)
    {
        return k == 3 ? (MU != d ? 1 : 0) : ((k == 1 || k == 2) && dir(k) == d ? 1 : 0);
    }
    __host__ __device__ static constexpr int hi(int k, int d)
    {
        return k == 3 ? (MU != d ? 1 : 0) : (MU == d ? 1 : 0);
    }
};

// Shape of array k from the slab extents (k = 4: base = total elements of
// all four); plans carry the four in StagePlan::arr.
template <int MU>
__host__ __device__ inline ArrayShape array_shape(const StagePlan &p, int k)
{
    using Ar = Arrays<MU>;
    uint32_t base = 0;
    ArrayShape out = {};
    for (int j = 0; j < 4; ++j) {
        ArrayShape sh;
        sh.lo_a = (uint32_t)Ar::lo(j, 1);
        sh.lo_b = (uint32_t)Ar::lo(j, Roles<MU>::b);
        sh.ra = p.A + sh.lo_a + (uint32_t)Ar::hi(j, 1);
        sh.rows = sh.ra * (p.B + sh.lo_b + (uint32_t)Ar::hi(j, Roles<MU>::b));
        sh.base = base;
        sh.count = sh.rows * p.nxh * (uint32_t)(Ar::slots(j) * Ar::parities(j));
        if (j == k)
            out = sh;
        base += sh.count;
    }
    if (k == 4)
        out.base = base;
    return out;
}

// Ring slot of slice sl in an array of `slots` slots (chunk starting at s0;
// sl >= s0 - 1).
__host__ __device__ inline uint32_t ring_slot(int32_t sl, int32_t s0, int slots)
{
    return slots == 1 ? 0u : (uint32_t)((sl - s0 + 6) % slots);
}

// Element index of (ring slot, parity slot q, slab-relative row (a, b), xh).
__host__ __device__ inline uint32_t lds_index(const ArrayShape &sh, uint32_t nxh, uint32_t slotq, int32_t a, int32_t b,
                                              uint32_t xh)
{
    const uint32_t row = (uint32_t)(a + (int32_t)sh.lo_a) + sh.ra * (uint32_t)(b + (int32_t)sh.lo_b);
    return sh.base + (slotq * sh.rows + row) * nxh + xh;
}

// Global row index y + Ny (z + Nz t) of slab-relative (a, b) in slice sl,
// every coordinate wrapped into the lattice, as the sum of a part without
// the marched coordinate (global_row_base) and that coordinate's term
// (slice_row).
template <int MU>
__host__ __device__ inline uint32_t global_row_base(const Geom &g, uint32_t y0, uint32_t b0, int32_t a, int32_t b)
{
    const int32_t ny = g.n[1], nb = g.n[Roles<MU>::b];
    int32_t y = (int32_t)y0 + a;
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    int32_t bb = (int32_t)b0 + b;
    bb = bb < 0 ? bb + nb : (bb >= nb ? bb - nb : bb);
    // b is z (mu != t: row term Ny z) or t (mu = t: row term Ny Nz t)
    return (uint32_t)y + (uint32_t)g.n[1] * (uint32_t)bb * (MU == 3 ? (uint32_t)g.n[2] : 1u);
}

template <int MU>
__host__ __device__ inline uint32_t slice_row(const Geom &g, int32_t sl)
{
    const int32_t ns = g.n[Roles<MU>::s];
    const int32_t ss = sl < 0 ? sl + ns : (sl >= ns ? sl - ns : sl);
    // s is t (mu != t: row term Ny Nz t) or z (mu = t: row term Ny z)
    return (uint32_t)g.n[1] * (uint32_t)ss * (MU == 3 ? 1u : (uint32_t)g.n[2]);
}

template <int MU>
__host__ __device__ inline uint32_t global_row(const Geom &g, uint32_t y0, uint32_t b0, int32_t a, int32_t b,
                                               int32_t sl)
{
    return global_row_base<MU>(g, y0, b0, a, b) + slice_row<MU>(g, sl);
}

// The i-th link a slab loads of the arrays in `which` (bit k = array k):
// arrays 0-2 for slice sl_s, array 3 for slice sl_m.  Sets the link's
// direction, parity (array 3: the class's opposite parity opp), global
// checkerboard index and element index in LDS; false if i is beyond them.
struct LoadItem {
    int dir, parity;
    uint32_t cb;
    uint32_t lds;
};

template <int MU>
__host__ __device__ inline bool load_item(const Geom &g, const StagePlan &p, uint32_t y0, uint32_t b0, int32_t s0,
                                          uint32_t which, int32_t sl_s, int32_t sl_m, int opp, uint32_t i,
                                          LoadItem &it)
{
    using Ar = Arrays<MU>;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!(which & (1u << k)))
            continue;
        const ArrayShape &sh = p.arr[k];
        const uint32_t per_par = sh.rows * p.nxh;
        const uint32_t n = per_par * (uint32_t)Ar::parities(k);
        if (i >= n) {
            i -= n;
            continue;
        }
        const uint32_t q = Ar::parities(k) == 1 ? 0u : fdiv(i, p.div_pp[k]);
        const uint32_t rem = i - q * per_par;
        const uint32_t row = fdiv(rem, p.div_nxh);
        const uint32_t xh = rem - row * p.nxh;
        const uint32_t bb = fdiv(row, p.div_ra[k]);
        const int32_t a = (int32_t)(row - bb * sh.ra) - (int32_t)sh.lo_a;
        const int32_t b = (int32_t)bb - (int32_t)sh.lo_b;
        const int32_t sl = k == 3 ? sl_m : sl_s;
        it.dir = Ar::dir(k);
        it.parity = k == 3 ? opp : (int)q;
        it.cb = xh + p.nxh * global_row<MU>(g, y0, b0, a, b, sl);
        it.lds = lds_index(sh, p.nxh, ring_slot(sl, s0, Ar::slots(k)) * (uint32_t)Ar::parities(k) + q, a, b, xh);
        return true;
    }
    return false;
}

// Links of arrays `which` per slice.
template <int MU>
__host__ __device__ inline uint32_t load_count(const StagePlan &p, uint32_t which)
{
    uint32_t n = 0;
    for (int k = 0; k < 4; ++k)
        if (which & (1u << k))
            n += p.arr[k].rows * p.nxh * (uint32_t)Arrays<MU>::parities(k);
    return n;
}

// A load item of the slice loop split into what does not depend on the
// slice (computed once per block and thread) and the per-slice terms: the
// kernel forms each slice's checkerboard index and LDS element by two
// additions (load_at).  The same split as load_item, which the host test
// checks.
struct LoadBase {
    uint32_t cb0;  // checkerboard index without the marched coordinate's term
    uint32_t lds0; // LDS element in ring slot 0
    uint32_t info; // plane 2 dir + parity | array << 8
};

template <int MU>
__host__ __device__ inline bool load_base(const Geom &g, const StagePlan &p, uint32_t y0, uint32_t b0, int opp,
                                          uint32_t i, LoadBase &lb)
{
    using Ar = Arrays<MU>;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const ArrayShape &sh = p.arr[k];
        const uint32_t per_par = sh.rows * p.nxh;
        const uint32_t n = per_par * (uint32_t)Ar::parities(k);
        if (i >= n) {
            i -= n;
            continue;
        }
        const uint32_t q = Ar::parities(k) == 1 ? 0u : fdiv(i, p.div_pp[k]);
        const uint32_t rem = i - q * per_par;
        const uint32_t row = fdiv(rem, p.div_nxh);
        const uint32_t xh = rem - row * p.nxh;
        const uint32_t bb = fdiv(row, p.div_ra[k]);
        const int32_t a = (int32_t)(row - bb * sh.ra) - (int32_t)sh.lo_a;
        const int32_t b = (int32_t)bb - (int32_t)sh.lo_b;
        const int parity = k == 3 ? opp : (int)q;
        lb.cb0 = xh + p.nxh * global_row_base<MU>(g, y0, b0, a, b);
        lb.lds0 = lds_index(sh, p.nxh, q, a, b, xh);
        lb.info = (uint32_t)(2 * Ar::dir(k) + parity) | ((uint32_t)k << 8);
        return true;
    }
    return false;
}

// The per-slice terms of arrays 0-2 at slice sl and of array 3 at sl + 1.
struct SliceTerms {
    uint32_t cb_s, cb_m;   // checkerboard-index terms of the marched coordinate
    uint32_t lds_0, lds_3; // ring-slot offsets of arrays 0 and 3
};

template <int MU>
__host__ __device__ inline SliceTerms slice_terms(const Geom &g, const StagePlan &p, int32_t s0, int32_t sl)
{
    using Ar = Arrays<MU>;
    SliceTerms t;
    t.cb_s = p.nxh * slice_row<MU>(g, sl);
    t.cb_m = p.nxh * slice_row<MU>(g, sl + 1);
    t.lds_0 = ring_slot(sl, s0, Ar::slots(0)) * (uint32_t)Ar::parities(0) * p.arr[0].rows * p.nxh;
    t.lds_3 = ring_slot(sl + 1, s0, Ar::slots(3)) * (uint32_t)Ar::parities(3) * p.arr[3].rows * p.nxh;
    return t;
}

__host__ __device__ inline void load_at(const LoadBase &lb, const SliceTerms &t, uint32_t &cb, uint32_t &lds)
{
    const uint32_t k = lb.info >> 8;
    cb = lb.cb0 + (k == 3 ? t.cb_m : t.cb_s);
    lds = lb.lds0 + (k == 0 ? t.lds_0 : (k == 3 ? t.lds_3 : 0u));
}

// LDS element of a staple link as the sum of a per-thread row base of its
// array (fixed for a block's thread), a uniform offset of the displacement
// and ring slot, and the displaced x position (staged_link_index).
template <int MU>
__host__ __device__ inline uint32_t staple_row_base(const StagePlan &p, int k, int32_t a, int32_t b)
{
    const ArrayShape &sh = p.arr[k];
    return sh.base + ((uint32_t)(a + (int32_t)sh.lo_a) + sh.ra * (uint32_t)(b + (int32_t)sh.lo_b)) * p.nxh;
}

__host__ __device__ inline uint32_t staple_shift(const StagePlan &p, int k, uint32_t slotq, int32_t ea, int32_t eb)
{
    const ArrayShape &sh = p.arr[k];
    return slotq * sh.rows * p.nxh + (uint32_t)((ea + (int32_t)sh.ra * eb) * (int32_t)p.nxh);
}

// checkerboard x position of x = xs displaced by ex in {-1, 0, 1}
__host__ __device__ inline uint32_t shifted_xh(uint32_t xs, int32_t ex, uint32_t nx)
{
    int32_t xx = (int32_t)xs + ex;
    xx = xx < 0 ? xx + (int32_t)nx : (xx >= (int32_t)nx ? xx - (int32_t)nx : xx);
    return (uint32_t)xx >> 1;
}

// ring and parity slot of a staple link of array k (parity of its site q)
template <int MU>
__host__ __device__ inline uint32_t staple_slotq(int k, int32_t sl, int32_t s0, int q)
{
    using Ar = Arrays<MU>;
    return ring_slot(sl, s0, Ar::slots(k)) * (uint32_t)Ar::parities(k) + (k == 3 ? 0u : (uint32_t)q);
}

// LDS element of the direction-d link at the site displaced by (ex, ea, eb,
// es) (in x, y, b, s) from the site at x = xs, slab-relative (a, b), slice
// sl, of parity par.
template <int MU>
__host__ __device__ inline uint32_t staged_link_index(const StagePlan &p, int32_t s0, int32_t sl, uint32_t nx,
                                                      uint32_t xs, int32_t a, int32_t b, int par, int d, int32_t ex,
                                                      int32_t ea, int32_t eb, int32_t es)
{
    const int k = Arrays<MU>::array_of(d);
    const int q = par ^ ((ex + ea + eb + es) & 1);
    return staple_row_base<MU>(p, k, a, b) + staple_shift(p, k, staple_slotq<MU>(k, sl + es, s0, q), ea, eb) +
           shifted_xh(xs, ex, nx);
}

// Host: a slab plan for class MU of lattice n, or false if none fits in
// lds_limit bytes of LDS per block (link = link_bytes).  Slabs of A x B
// rows with A | Ny, B | Nb, S | Ns and at least `min_blocks` slabs; the
// plan loading the fewest links per update.
template <int MU>
__host__ inline bool make_stage_plan(const int32_t n[4], uint32_t link_bytes, uint32_t lds_limit, uint32_t min_blocks,
                                     StagePlan &out)
{
    const uint32_t nx = (uint32_t)n[0], ny = (uint32_t)n[1];
    const uint32_t nb = (uint32_t)n[Roles<MU>::b], ns = (uint32_t)n[Roles<MU>::s];
    bool found = false;
    double best = 0.0;
    for (uint32_t A = 1; A <= ny; ++A) {
        if (ny % A)
            continue;
        for (uint32_t B = 1; B <= nb; ++B) {
            if (nb % B)
                continue;
            StagePlan p = {};
            p.A = A;
            p.B = B;
            p.nxh = nx / 2;
            p.na = ny / A;
            p.nb = nb / B;
            const uint32_t sites = A * B * p.nxh;
            if (sites % 64 || sites < 256 || sites > (uint32_t)kStagedThreads)
                continue;
            const uint64_t lds = (uint64_t)array_shape<MU>(p, 4).base * link_bytes;
            if (lds > lds_limit)
                continue;
            p.lds_bytes = (uint32_t)lds;
            p.div_nxh = make_fastdiv(p.nxh);
            for (int k = 0; k < 4; ++k) {
                p.arr[k] = array_shape<MU>(p, k);
                p.div_pp[k] = make_fastdiv(p.arr[k].rows * p.nxh);
                p.div_ra[k] = make_fastdiv(p.arr[k].ra);
            }
            p.n_fresh = load_count<MU>(p, 15u);
            if (p.n_fresh > (uint32_t)(kStagedThreads * staged_prefetch(link_bytes)))
                continue;
            // shortest chunks that give min_blocks slabs, no shorter than 8
            // slices (each chunk re-reads two slices of the previous)
            uint32_t S = ns;
            while (p.na * p.nb * (ns / S) < min_blocks && S % 2 == 0 && S / 2 >= 8 && ns % (S / 2) == 0)
                S /= 2;
            p.S = S;
            p.ns = ns / S;
            if (p.na * p.nb * p.ns < min_blocks)
                continue;
            // links loaded per update, the chunk's prologue included
            const double per = ((double)p.n_fresh * S + (double)load_count<MU>(p, 1u) + 2.0 * load_count<MU>(p, 8u)) /
                                   ((double)sites * S) + 1.0;
            if (!found || per < best) {
                best = per;
                out = p;
                found = true;
            }
        }
    }
    return found;
}

} // namespace su2

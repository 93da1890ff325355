// su2_device.hpp -- device primitives of the SU(2) heat-bath library for
// gfx950: Philox4x32-10, uniform conversions, quaternion SU(2) algebra, the
// checkerboard geometry and the link-plane accessors.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace su2 {

constexpr double kPi = 3.14159265358979323846;
constexpr uint32_t kFlagCap = 1u;
constexpr uint32_t kFlagNonFinite = 2u;
constexpr uint32_t kFlagSync = 4u; // a grid-wide barrier wait gave up (persistent batched sweep)
constexpr uint32_t kMaxAttempts = 4096u;
constexpr int kBlock = 256; // threads per block of every lattice kernel

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64-bit products whose halves are mixed with the other two counter
// words and the round key; the key advances by the Weyl constants.
// ---------------------------------------------------------------------------
struct U32x4 {
    uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ U32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Open-interval uniforms.  FP64: 52 bits (the high word and the top 20 bits
// of the low word) plus one half ulp; every step is exact in double.
__device__ __forceinline__ double u01_f64(uint32_t hi, uint32_t lo)
{
    return __builtin_fma((double)hi, 0x1p-32, ((double)(lo >> 12) + 0.5) * 0x1p-52);
}

// FP32: the top 23 bits of the even word plus one half ulp (exact).
__device__ __forceinline__ float u01_f32(uint32_t w)
{
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

// Two uniforms per Philox call, in the sampler's working precision.
template <class T>
struct Draw;
template <>
struct Draw<double> {
    __device__ static __forceinline__ void two(const U32x4 &r, double &a, double &b)
    {
        a = u01_f64(r.r0, r.r1);
        b = u01_f64(r.r2, r.r3);
    }
};
template <>
struct Draw<float> {
    __device__ static __forceinline__ void two(const U32x4 &r, double &a, double &b)
    {
        a = (double)u01_f32(r.r0);
        b = (double)u01_f32(r.r2);
    }
};

// ---------------------------------------------------------------------------
// SU(2) as unit quaternions q = q0 + i q.sigma:
//   (a0,a)(b0,b) = (a0 b0 - a.b, a0 b + b0 a - a x b),  q^dagger = (q0, -q).
// ---------------------------------------------------------------------------
template <class T>
struct Quat {
    T w, x, y, z;
};

template <class T>
__device__ __forceinline__ Quat<T> qmul(const Quat<T> &a, const Quat<T> &b)
{
    Quat<T> r;
    r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    r.x = a.w * b.x + b.w * a.x - a.y * b.z + a.z * b.y;
    r.y = a.w * b.y + b.w * a.y - a.z * b.x + a.x * b.z;
    r.z = a.w * b.z + b.w * a.z - a.x * b.y + a.y * b.x;
    return r;
}

// a * b^dagger
template <class T>
__device__ __forceinline__ Quat<T> qmul_nd(const Quat<T> &a, const Quat<T> &b)
{
    Quat<T> r;
    r.w = a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
    r.x = -a.w * b.x + b.w * a.x + a.y * b.z - a.z * b.y;
    r.y = -a.w * b.y + b.w * a.y + a.z * b.x - a.x * b.z;
    r.z = -a.w * b.z + b.w * a.z + a.x * b.y - a.y * b.x;
    return r;
}

// a^dagger * b
template <class T>
__device__ __forceinline__ Quat<T> qmul_dn(const Quat<T> &a, const Quat<T> &b)
{
    Quat<T> r;
    r.w = a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
    r.x = a.w * b.x - b.w * a.x + a.y * b.z - a.z * b.y;
    r.y = a.w * b.y - b.w * a.y + a.z * b.x - a.x * b.z;
    r.z = a.w * b.z - b.w * a.z + a.x * b.y - a.y * b.x;
    return r;
}

// a^dagger * b^dagger = (b a)^dagger
template <class T>
__device__ __forceinline__ Quat<T> qmul_dd(const Quat<T> &a, const Quat<T> &b)
{
    Quat<T> r;
    r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    r.x = -a.w * b.x - b.w * a.x - a.y * b.z + a.z * b.y;
    r.y = -a.w * b.y - b.w * a.y - a.z * b.x + a.x * b.z;
    r.z = -a.w * b.z - b.w * a.z - a.x * b.y + a.y * b.x;
    return r;
}

// scalar part of a * b^dagger (= 4-D dot product)
template <class T>
__device__ __forceinline__ T qdot(const Quat<T> &a, const Quat<T> &b)
{
    return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}

template <class T>
__device__ __forceinline__ void qacc(Quat<T> &s, const Quat<T> &a)
{
    s.w += a.w;
    s.x += a.x;
    s.y += a.y;
    s.z += a.z;
}

// ---------------------------------------------------------------------------
// Unsigned division by a run-time constant (n < 2^31): q = (mulhi(m,n)+n)>>l
// with l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1 (Granlund and
// Montgomery, PLDI 1994).
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, l;
};

__host__ inline FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d)
        ++l;
    uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return {d, (uint32_t)m, l};
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    return ((uint32_t)(((uint64_t)n * f.m) >> 32) + n) >> f.l;
}

// Order in which the threads of one checkerboard class walk its V/2 sites.
// A block takes 256 consecutive indices i of the walk; hardware blocks are
// renumbered (xcd_tile) so that each XCD takes one contiguous range of the
// walk.  In strip mode the walk visits (z,t) columns (C = Nx*Ny/2 cb indices
// each) strip by strip of W z-values, t-major inside a strip: the +-t halo
// of a column is W columns behind in the walk, still in the XCD's L2,
// instead of a whole t-slice behind.  With S > 1 each strip is walked S
// times, once per range of Ny/S rows (contiguous in memory), which shrinks
// the data between a column and its t-neighbour S-fold at the price of
// re-reading two boundary rows per range.  Mode 0 walks plain cb order.
// Every walk is a bijection onto the class, so results do not depend on it.
struct BlockOrder {
    uint32_t strip;  // 0 = plain cb order, else the strip width W (divides Nz)
    uint32_t cols;   // C
    uint32_t nz;     // Nz
    uint32_t ysplit; // S: each column is walked as S contiguous ranges of Ny/S rows
    uint32_t seg;    // C / S, the cb indices of one range
    FastDiv div_cols, div_w, div_nt, div_seg, div_ys;
};

// ---------------------------------------------------------------------------
// Geometry: periodic Nx x Ny x Nz x Nt, x fastest, checkerboard index
// cb = site/2; a "row" is a line of constant (y,z,t): row = y + Ny(z + Nz t).
// ---------------------------------------------------------------------------
struct Geom {
    int32_t n[4];
    uint32_t nxh;  // Nx/2: checkerboard sites per row
    uint32_t half; // V/2
    uint32_t vs;   // Nx Ny Nz
    FastDiv div_nx, div_nxh, div_ny, div_nz;
    BlockOrder ord;
};

// One lattice of a batched launch (filled on the host, read by every block).
struct BatchEntry {
    Geom g;
    void *links;
    uint32_t *flags;
    double beta;
    uint32_t lid16;   // 16 * lattice_id, the lattice's share of counter word c1
    uint32_t block0;  // first block of this lattice in the batched grid (multiple of 8)
    uint32_t nblocks; // blocks of this lattice (multiple of 8)
    // first block in the grid of the batched overrelaxation launches, which
    // leave out the lattices that batch_own_launch gives launches of their
    // own (their range there is empty: sub_block0 of the next lattice)
    uint32_t sub_block0;
    uint32_t col;     // 1: the lattice qualifies for column addressing
    // Polyakov loop and correlator (the regions of the lattice's workspace
    // and the block counts its single-lattice launches use)
    double *lfield;    // L of every spatial site
    double *poly_part; // 2 columns of pnblk block partials
    double *corr_part; // rmax columns of cnblk block partials
    uint32_t pblock0, pnblk; // Polyakov blocks: first in the batched grid, count
    uint32_t cblock0, cnblk; // correlator blocks: first in the batched grid, count per separation group
    uint32_t rmax, ocol0;    // separations; first of the lattice's 2 + rmax output columns
};

// Index of the batch entry whose range of the batched grid holds block b:
// the last entry with (entry.*FIRST) <= b (the firsts ascend).  Each lane
// tests one entry and a wave ballot counts the hits, so the lookup is one
// round of independent loads per 64 lattices.
template <uint32_t BatchEntry::*FIRST>
__device__ __forceinline__ int find_entry_index(const BatchEntry *tab, int count, uint32_t b)
{
    const int lane = (int)(threadIdx.x & 63u);
    int hits = 0;
    for (int base = 0; base < count; base += 64) {
        const int j = base + lane;
        const bool le = j < count && tab[j].*FIRST <= b;
        hits += (int)__popcll(__ballot(le));
    }
    return __builtin_amdgcn_readfirstlane(hits > 0 ? hits - 1 : 0);
}

// ---------------------------------------------------------------------------
// Geometry construction (host).  Walk of a class: tile > 0 is the strip width
// (it divides Nz; the caller checked), tile == 0 the default (Nz/8 rounded
// down to a divisor of Nz, so that each of the 8 XCDs takes one strip),
// tile < 0 plain cb order.  Every field is set in every mode.
// ---------------------------------------------------------------------------
__host__ inline int default_strip(const int32_t n[4])
{
    const uint32_t nz = (uint32_t)n[2];
    uint32_t w = nz / 8u > 0 ? nz / 8u : 1u;
    while (nz % w)
        --w;
    return (int)w;
}

__host__ inline BlockOrder make_block_order(const int32_t n[4], int tile, int tile_y)
{
    BlockOrder o = {};
    o.cols = (uint32_t)n[0] / 2u * (uint32_t)n[1];
    o.nz = (uint32_t)n[2];
    o.div_cols = make_fastdiv(o.cols);
    o.div_nt = make_fastdiv((uint32_t)n[3]);
    // tiles -2 and -3 (staged updates): the other kernels walk the default strips
    const int w = (tile == 0 || tile == -2 || tile == -3) ? default_strip(n) : tile;
    o.strip = w > 0 ? (uint32_t)w : 0u;
    o.div_w = make_fastdiv(w > 0 ? (uint32_t)w : 1u);
    // row ranges per column: tile_y > 0 as given (it divides Ny; the caller
    // checked), 0 = whole columns; plain order has none
    const int s = (w > 0 && tile_y > 0) ? tile_y : 1;
    o.ysplit = (uint32_t)s;
    o.seg = o.cols / o.ysplit;
    o.div_seg = make_fastdiv(o.seg);
    o.div_ys = make_fastdiv(o.ysplit);
    return o;
}

__host__ inline Geom make_geom(const int32_t n[4], int tile, int tile_y = 0)
{
    Geom g = {};
    for (int d = 0; d < 4; ++d)
        g.n[d] = n[d];
    g.nxh = (uint32_t)n[0] / 2u;
    const uint64_t vol = (uint64_t)n[0] * n[1] * n[2] * n[3];
    g.half = (uint32_t)(vol / 2);
    g.vs = (uint32_t)((uint64_t)n[0] * n[1] * n[2]);
    g.div_nx = make_fastdiv((uint32_t)n[0]);
    g.div_nxh = make_fastdiv(g.nxh);
    g.div_ny = make_fastdiv((uint32_t)n[1]);
    g.div_nz = make_fastdiv((uint32_t)n[2]);
    g.ord = make_block_order(n, tile, tile_y);
    return g;
}

struct Site {
    int32_t c[4];  // x, y, z, t
    uint32_t site; // linear site index
};

// Coordinates of the cb-th site of the given parity.
__host__ __device__ __forceinline__ Site site_of_cb(const Geom &g, uint32_t cb, int parity)
{
    const uint32_t row = fdiv(cb, g.div_nxh);
    const uint32_t xh = cb - row * g.nxh;
    const uint32_t zt = fdiv(row, g.div_ny);
    const uint32_t y = row - zt * (uint32_t)g.n[1];
    const uint32_t t = fdiv(zt, g.div_nz);
    const uint32_t z = zt - t * (uint32_t)g.n[2];
    const uint32_t x = 2u * xh + ((y + z + t + (uint32_t)parity) & 1u);
    Site s;
    s.c[0] = (int32_t)x;
    s.c[1] = (int32_t)y;
    s.c[2] = (int32_t)z;
    s.c[3] = (int32_t)t;
    s.site = x + (uint32_t)g.n[0] * row;
    return s;
}

__host__ __device__ __forceinline__ uint32_t cb_of(const Geom &g, int32_t x, int32_t y, int32_t z, int32_t t)
{
    return ((uint32_t)x >> 1) +
           g.nxh * ((uint32_t)y + (uint32_t)g.n[1] * ((uint32_t)z + (uint32_t)g.n[2] * (uint32_t)t));
}

__host__ __device__ __forceinline__ int32_t wrap_add(int32_t c, int32_t s, int32_t n)
{
    c += s;
    c = (c >= n) ? c - n : c;
    return (c < 0) ? c + n : c;
}

// cb index of the site displaced by (d0,d1,d2,d3) in {-1,0,1}.
__host__ __device__ __forceinline__ uint32_t cb_shift(const Geom &g, const int32_t c[4], int32_t d0, int32_t d1,
                                             int32_t d2, int32_t d3)
{
    return cb_of(g, wrap_add(c[0], d0, g.n[0]), wrap_add(c[1], d1, g.n[1]),
                 wrap_add(c[2], d2, g.n[2]), wrap_add(c[3], d3, g.n[3]));
}

// ---------------------------------------------------------------------------
// Link planes: plane q = 2 mu + parity, V/2 links each, consecutive planes
// (FP64: sub-planes) `stride` 16-byte elements apart.
//
// FP64 sub-planes of V/2 >= 2^18 elements (4 MB and more) are skewed: the
// stride is V/2 + kPlaneSkew, 256 KB + 128 B beyond the plane.  When V/2 is
// a multiple of 2^14, unskewed sub-planes put the same cb of all 16 of them
// at addresses that differ by multiples of 256 KB, and the updates of one
// block read nearby cb in most of them, so those lines compete for the same
// L2 sets.
// At 64^4 the skew cuts the heat bath's reads beyond L2 from 1.56x to 1.25x
// the compulsory bytes (overrelaxation 1.34x to 1.17x) and its class from
// 476 to 455 us.  FP32 planes (8 of them) gain nothing and stay unskewed.
// ---------------------------------------------------------------------------
constexpr uint32_t kPlaneSkew = 16392u;
constexpr uint32_t kPlaneSkewMinHalf = 1u << 18;

__host__ __device__ __forceinline__ uint32_t plane_stride(uint32_t half, bool f64)
{
    return (f64 && half >= kPlaneSkewMinHalf) ? half + kPlaneSkew : half;
}

typedef float V4f __attribute__((ext_vector_type(4)));
typedef double V2d __attribute__((ext_vector_type(2)));

template <class T>
struct Links;

template <>
struct Links<float> {
    float4 *p;
    uint32_t stride; // elements between plane starts
    __device__ __forceinline__ Quat<float> ld(int mu, int par, uint32_t cb) const
    {
        const float4 v = p[(size_t)(2 * mu + par) * stride + cb];
        return {v.x, v.y, v.z, v.w};
    }
    // Stores are non-temporal: an updated link is not read again by the
    // same launch, so it should not displace the neighbourhood from L2.
    __device__ __forceinline__ void st(int mu, int par, uint32_t cb, const Quat<float> &q) const
    {
        const V4f v = {q.w, q.x, q.y, q.z};
        __builtin_nontemporal_store(v, reinterpret_cast<V4f *>(p + (size_t)(2 * mu + par) * stride + cb));
    }
    // Non-temporal load, for a link read once by its own update.
    __device__ __forceinline__ Quat<float> ld_nt(int mu, int par, uint32_t cb) const
    {
        const V4f v = __builtin_nontemporal_load(reinterpret_cast<const V4f *>(p + (size_t)(2 * mu + par) * stride + cb));
        return {v.x, v.y, v.z, v.w};
    }
    // by byte offset within the plane (< 2^32)
    __device__ __forceinline__ Quat<float> ldb(int mu, int par, uint32_t boff) const
    {
        const char *base = reinterpret_cast<const char *>(p + (size_t)(2 * mu + par) * stride);
        const float4 v = *reinterpret_cast<const float4 *>(base + boff);
        return {v.x, v.y, v.z, v.w};
    }
    __device__ __forceinline__ Quat<float> ldb_nt(int mu, int par, uint32_t boff) const
    {
        const char *base = reinterpret_cast<const char *>(p + (size_t)(2 * mu + par) * stride);
        const V4f v = __builtin_nontemporal_load(reinterpret_cast<const V4f *>(base + boff));
        return {v.x, v.y, v.z, v.w};
    }
    __device__ __forceinline__ void stb(int mu, int par, uint32_t boff, const Quat<float> &q) const
    {
        char *base = reinterpret_cast<char *>(p + (size_t)(2 * mu + par) * stride);
        const V4f v = {q.w, q.x, q.y, q.z};
        __builtin_nontemporal_store(v, reinterpret_cast<V4f *>(base + boff));
    }
};

template <>
struct Links<double> {
    double2 *p;
    uint32_t stride; // elements between sub-plane starts
    __device__ __forceinline__ Quat<double> ld(int mu, int par, uint32_t cb) const
    {
        const size_t q = (size_t)(2 * mu + par);
        const double2 a = p[(2 * q) * stride + cb];
        const double2 b = p[(2 * q + 1) * stride + cb];
        return {a.x, a.y, b.x, b.y};
    }
    __device__ __forceinline__ void st(int mu, int par, uint32_t cb, const Quat<double> &v) const
    {
        const size_t q = (size_t)(2 * mu + par);
        const V2d a = {v.w, v.x}, b = {v.y, v.z};
        __builtin_nontemporal_store(a, reinterpret_cast<V2d *>(p + (2 * q) * stride + cb));
        __builtin_nontemporal_store(b, reinterpret_cast<V2d *>(p + (2 * q + 1) * stride + cb));
    }
    __device__ __forceinline__ Quat<double> ld_nt(int mu, int par, uint32_t cb) const
    {
        const size_t q = (size_t)(2 * mu + par);
        const V2d a = __builtin_nontemporal_load(reinterpret_cast<const V2d *>(p + (2 * q) * stride + cb));
        const V2d b = __builtin_nontemporal_load(reinterpret_cast<const V2d *>(p + (2 * q + 1) * stride + cb));
        return {a.x, a.y, b.x, b.y};
    }
    // by byte offset within the sub-planes (< 2^32)
    __device__ __forceinline__ Quat<double> ldb(int mu, int par, uint32_t boff) const
    {
        const size_t q = (size_t)(2 * mu + par);
        const char *ba = reinterpret_cast<const char *>(p + (2 * q) * stride);
        const char *bb = reinterpret_cast<const char *>(p + (2 * q + 1) * stride);
        const double2 a = *reinterpret_cast<const double2 *>(ba + boff);
        const double2 b = *reinterpret_cast<const double2 *>(bb + boff);
        return {a.x, a.y, b.x, b.y};
    }
    __device__ __forceinline__ Quat<double> ldb_nt(int mu, int par, uint32_t boff) const
    {
        const size_t q = (size_t)(2 * mu + par);
        const char *ba = reinterpret_cast<const char *>(p + (2 * q) * stride);
        const char *bb = reinterpret_cast<const char *>(p + (2 * q + 1) * stride);
        const V2d a = __builtin_nontemporal_load(reinterpret_cast<const V2d *>(ba + boff));
        const V2d b = __builtin_nontemporal_load(reinterpret_cast<const V2d *>(bb + boff));
        return {a.x, a.y, b.x, b.y};
    }
    __device__ __forceinline__ void stb(int mu, int par, uint32_t boff, const Quat<double> &v) const
    {
        const size_t q = (size_t)(2 * mu + par);
        char *ba = reinterpret_cast<char *>(p + (2 * q) * stride);
        char *bb = reinterpret_cast<char *>(p + (2 * q + 1) * stride);
        const V2d a = {v.w, v.x}, b = {v.y, v.z};
        __builtin_nontemporal_store(a, reinterpret_cast<V2d *>(ba + boff));
        __builtin_nontemporal_store(b, reinterpret_cast<V2d *>(bb + boff));
    }
};

// Normalisation on write: FP32 links are projected back onto the unit
// sphere; FP64 links are stored as computed.
template <class T>
__device__ __forceinline__ Quat<T> unitize(const Quat<T> &q)
{
    return q;
}
template <>
__device__ __forceinline__ Quat<float> unitize<float>(const Quat<float> &q)
{
    const float s = rsqrtf(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
    return {q.w * s, q.x * s, q.y * s, q.z * s};
}

// Counter arithmetic of the persistent sweep's grid-wide barrier: block b of
// a grid of G blocks adds barrier_increment(b, G) to the counter word (the G
// additions of one barrier sum to 2^31), and a block that read `old` from
// its own addition has passed the barrier once bit 31 of the word differs.
__host__ __device__ __forceinline__ uint32_t barrier_increment(uint32_t b, uint32_t g)
{
    return b == 0u ? 0x80000000u - (g - 1u) : 1u;
}
__host__ __device__ __forceinline__ bool barrier_passed(uint32_t now, uint32_t old)
{
    return ((now ^ old) & 0x80000000u) != 0u;
}

// XCD-aware block order: consecutive blocks are dispatched round-robin over
// the 8 XCDs, each with its own L2; renumber so that each XCD works through
// one contiguous range of tiles (neighbouring tiles share halo links).
__host__ __device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks)
{
    const uint32_t q = nblocks >> 3, r = nblocks & 7u;
    const uint32_t xcd = b & 7u, k = b >> 3;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// cb index of the i-th site of the walk.
__host__ __device__ __forceinline__ uint32_t walk_cb(uint32_t i, const BlockOrder &o)
{
    if (o.strip == 0)
        return i;
    const uint32_t j = fdiv(i, o.div_seg);   // range of the walk
    const uint32_t off = i - j * o.seg;
    const uint32_t q = fdiv(j, o.div_w);
    const uint32_t zz = j - q * o.strip;
    const uint32_t r = fdiv(q, o.div_nt);
    const uint32_t t = q - r * o.div_nt.d;
    const uint32_t s = fdiv(r, o.div_ys);    // strip
    const uint32_t yr = r - s * o.ysplit;    // row range within the strip
    const uint32_t z = s * o.strip + zz;
    return yr * o.seg + off + o.cols * (z + o.nz * t);
}

// ---------------------------------------------------------------------------
// Addressing of a site's neighbours.  Two policies give the same indices:
//
// CbAddr: from the site's coordinates (cb_shift), for any geometry.
//
// ColAddr: when the walk's unit (a column of C = Nx Ny / 2 cb indices, or a
// row range of it) is a multiple of 64, the 64 sites of a wave lie in one
// (z,t) column, so z, t and everything derived from them
// are wave-uniform (scalar registers) and only the in-plane position varies
// per lane.  A neighbour's index is then the sum of an x part and a y part
// (per lane) and a z part and a t part (scalar), each precomputed for the
// shifts 0, +1, -1.  Offsets are kept in bytes: with V/2 <= 2^28 a plane's
// byte offsets fit 32 bits, so every load is a scalar plane base plus one
// 32-bit lane offset (one add per load instead of the coordinate arithmetic).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int shift_slot(int d)
{
    return d == 0 ? 0 : (d > 0 ? 1 : 2);
}

struct CbAddr {
    Site s;
    uint32_t cb;
    const Geom *g;
    __host__ __device__ __forceinline__ uint32_t at(int32_t d0, int32_t d1, int32_t d2, int32_t d3) const
    {
        if (d0 == 0 && d1 == 0 && d2 == 0 && d3 == 0)
            return cb;
        return cb_shift(*g, s.c, d0, d1, d2, d3);
    }
    template <class T>
    __device__ __forceinline__ Quat<T> ld(const Links<T> &U, int mu, int par, uint32_t idx) const
    {
        return U.ld(mu, par, idx);
    }
    template <class T>
    __device__ __forceinline__ Quat<T> ld_nt(const Links<T> &U, int mu, int par, uint32_t idx) const
    {
        return U.ld_nt(mu, par, idx);
    }
    template <class T>
    __device__ __forceinline__ void st(const Links<T> &U, int mu, int par, uint32_t idx, const Quat<T> &q) const
    {
        U.st(mu, par, idx, q);
    }
    __host__ __device__ __forceinline__ uint32_t site() const
    {
        return s.site;
    }
};

struct ColAddr {
    uint32_t xb[3]; // lane: 16 * (x' >> 1) for x' = x, x+1, x-1 (mod Nx)
    uint32_t yb[3]; // lane: 16 * (Nx/2) * y' for y' = y, y+1, y-1 (mod Ny)
    uint32_t zb[3]; // wave: 16 * C * z' for z' = z, z+1, z-1 (mod Nz)
    uint32_t tb[3]; // wave: 16 * C * Nz * t' for t' = t, t+1, t-1 (mod Nt)
    uint32_t xodd;  // lane: x & 1
    __host__ __device__ __forceinline__ uint32_t at(int32_t d0, int32_t d1, int32_t d2, int32_t d3) const
    {
        return xb[shift_slot(d0)] + yb[shift_slot(d1)] + (zb[shift_slot(d2)] + tb[shift_slot(d3)]);
    }
    template <class T>
    __device__ __forceinline__ Quat<T> ld(const Links<T> &U, int mu, int par, uint32_t boff) const
    {
        return U.ldb(mu, par, boff);
    }
    template <class T>
    __device__ __forceinline__ Quat<T> ld_nt(const Links<T> &U, int mu, int par, uint32_t boff) const
    {
        return U.ldb_nt(mu, par, boff);
    }
    template <class T>
    __device__ __forceinline__ void st(const Links<T> &U, int mu, int par, uint32_t boff, const Quat<T> &q) const
    {
        U.stb(mu, par, boff, q);
    }
    __host__ __device__ __forceinline__ uint32_t site() const
    {
        return 2u * ((xb[0] + yb[0] + zb[0] + tb[0]) >> 4) + xodd;
    }
};

// Whether a lattice and walk qualify for ColAddr (host side; the launchers
// pick it): a wave's 64 walk indices must lie in one column (one row range
// in strip mode), and byte offsets within a plane must fit 32 bits.
__host__ inline bool col_addressing_ok(const Geom &g)
{
    const uint32_t unit = g.ord.strip == 0 ? g.ord.cols : g.ord.seg;
    return unit % 64u == 0 && g.half <= (1u << 28);
}

// ColAddr of walk index i0 + lane of class `par`, where i0 (a multiple of 64)
// is the wave's first index; the caller guarantees that the lattice
// qualifies and that i0 < V/2 (then so are all 64 indices: V/2 is a
// multiple of the walk's unit, hence of 64).
__host__ __device__ __forceinline__ ColAddr col_addr_at(const Geom &g, uint32_t i0, uint32_t lane, int par)
{
    const BlockOrder &o = g.ord;
    uint32_t z, t, off0; // off0: the wave's first position in the (x,y) plane, in cb units
    if (o.strip == 0) {
        const uint32_t j = fdiv(i0, o.div_cols); // column (wave-uniform)
        t = fdiv(j, g.div_nz);
        z = j - t * (uint32_t)g.n[2];
        off0 = i0 - j * o.cols;
    } else {
        const uint32_t j = fdiv(i0, o.div_seg); // row range of the walk (wave-uniform)
        const uint32_t q = fdiv(j, o.div_w);
        const uint32_t zz = j - q * o.strip;
        const uint32_t r = fdiv(q, o.div_nt);
        t = q - r * o.div_nt.d;
        const uint32_t sidx = fdiv(r, o.div_ys);
        z = sidx * o.strip + zz;
        off0 = (r - sidx * o.ysplit) * o.seg + (i0 - j * o.seg);
    }
    const uint32_t ny = (uint32_t)g.n[1], nz = (uint32_t)g.n[2], nt = (uint32_t)g.n[3];
    const uint32_t cz = 16u * o.cols, ct = cz * nz;
    ColAddr a;
    a.zb[0] = cz * z;
    a.zb[1] = cz * (z + 1u == nz ? 0u : z + 1u);
    a.zb[2] = cz * (z == 0u ? nz - 1u : z - 1u);
    a.tb[0] = ct * t;
    a.tb[1] = ct * (t + 1u == nt ? 0u : t + 1u);
    a.tb[2] = ct * (t == 0u ? nt - 1u : t - 1u);
    const uint32_t off = off0 + lane; // position in the (x,y) plane, in cb units
    const uint32_t y = fdiv(off, g.div_nxh);
    const uint32_t xh = off - y * g.nxh;
    a.xodd = (y + z + t + (uint32_t)par) & 1u;
    const uint32_t rb = 16u * g.nxh;
    a.yb[0] = rb * y;
    a.yb[1] = rb * (y + 1u == ny ? 0u : y + 1u);
    a.yb[2] = rb * (y == 0u ? ny - 1u : y - 1u);
    a.xb[0] = 16u * xh;
    a.xb[1] = a.xodd ? (xh + 1u == g.nxh ? 0u : 16u * (xh + 1u)) : 16u * xh;
    a.xb[2] = a.xodd ? 16u * xh : (xh == 0u ? 16u * (g.nxh - 1u) : 16u * (xh - 1u));
    return a;
}

// The same for walk index i held by a lane of a wave (lane = i & 63): the
// wave's first index is made scalar so that z, t and the column offsets live
// in scalar registers.
__device__ __forceinline__ ColAddr col_addr(const Geom &g, uint32_t i, int par)
{
    const uint32_t lane = i & 63u;
    return col_addr_at(g, __builtin_amdgcn_readfirstlane(i - lane), lane, par);
}

// ---------------------------------------------------------------------------
// Staple sum of U_mu(x) (x of parity `par`):
//   V = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
//                    + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
// so that the link's local action is -(beta/2) Tr(U_mu(x) V).  The order of
// the products and sums is the same for both addressing policies.
// ---------------------------------------------------------------------------
// The sum of the two staple products of plane (nu, MU), nu < MU: the half
// trace is linear, so its half trace with U_MU(x) is the sum of the two
// plaquettes of that plane containing the link.  Recorded when the update
// also measures the plaquette.
template <class T>
struct PlaneTerms {
    Quat<T> s[3];
};

template <class T, int MU, bool TERMS, class A>
__device__ __forceinline__ Quat<T> staple_impl(const Links<T> &U, const A &ad, int par, PlaneTerms<T> *terms)
{
    const int opp = par ^ 1;
    const int32_t m0 = (MU == 0), m1 = (MU == 1), m2 = (MU == 2), m3 = (MU == 3);
    const uint32_t i_xp = ad.at(m0, m1, m2, m3);
    const uint32_t i_x = ad.at(0, 0, 0, 0);
    Quat<T> V = {0, 0, 0, 0};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU)
            continue;
        const int32_t e0 = (nu == 0), e1 = (nu == 1), e2 = (nu == 2), e3 = (nu == 3);
        const uint32_t i_xpn = ad.at(e0, e1, e2, e3);
        const uint32_t i_xmn = ad.at(-e0, -e1, -e2, -e3);
        const uint32_t i_xpmn = ad.at(m0 - e0, m1 - e1, m2 - e2, m3 - e3);
        // upper staple
        const Quat<T> a = ad.ld(U, nu, opp, i_xp);
        const Quat<T> b = ad.ld(U, MU, opp, i_xpn);
        const Quat<T> c = ad.ld(U, nu, par, i_x);
        const Quat<T> su = qmul_nd(qmul_nd(a, b), c);
        qacc(V, su);
        // lower staple
        const Quat<T> d = ad.ld(U, nu, par, i_xpmn);
        const Quat<T> e = ad.ld(U, MU, opp, i_xmn);
        const Quat<T> f = ad.ld(U, nu, opp, i_xmn);
        const Quat<T> sl = qmul(qmul_dd(d, e), f);
        qacc(V, sl);
        if constexpr (TERMS) {
            if (nu < MU)
                terms->s[nu] = {su.w + sl.w, su.x + sl.x, su.y + sl.y, su.z + sl.z};
        }
    }
    return V;
}

// The staple in two steps: load its 18 links, then form it.  Used where
// independent work (the heat bath's random numbers) is placed between the
// two, while the loads are in flight.  Same products and sums, in the same
// order, as staple_impl.
template <class T, int MU, class A>
__device__ __forceinline__ void staple_load(const Links<T> &U, const A &ad, int par, Quat<T> (&L)[4][6])
{
    const int opp = par ^ 1;
    const int32_t m0 = (MU == 0), m1 = (MU == 1), m2 = (MU == 2), m3 = (MU == 3);
    const uint32_t i_xp = ad.at(m0, m1, m2, m3);
    const uint32_t i_x = ad.at(0, 0, 0, 0);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU)
            continue;
        const int32_t e0 = (nu == 0), e1 = (nu == 1), e2 = (nu == 2), e3 = (nu == 3);
        const uint32_t i_xpn = ad.at(e0, e1, e2, e3);
        const uint32_t i_xmn = ad.at(-e0, -e1, -e2, -e3);
        const uint32_t i_xpmn = ad.at(m0 - e0, m1 - e1, m2 - e2, m3 - e3);
        L[nu][0] = ad.ld(U, nu, opp, i_xp);
        L[nu][1] = ad.ld(U, MU, opp, i_xpn);
        L[nu][2] = ad.ld(U, nu, par, i_x);
        L[nu][3] = ad.ld(U, nu, par, i_xpmn);
        L[nu][4] = ad.ld(U, MU, opp, i_xmn);
        L[nu][5] = ad.ld(U, nu, opp, i_xmn);
    }
}

template <class T, int MU, bool TERMS>
__device__ __forceinline__ Quat<T> staple_compute(const Quat<T> (&L)[4][6], PlaneTerms<T> *terms)
{
    Quat<T> V = {0, 0, 0, 0};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU)
            continue;
        const Quat<T> su = qmul_nd(qmul_nd(L[nu][0], L[nu][1]), L[nu][2]);
        qacc(V, su);
        const Quat<T> sl = qmul(qmul_dd(L[nu][3], L[nu][4]), L[nu][5]);
        qacc(V, sl);
        if constexpr (TERMS) {
            if (nu < MU)
                terms->s[nu] = {su.w + sl.w, su.x + sl.x, su.y + sl.y, su.z + sl.z};
        }
    }
    return V;
}

template <class T, int MU, class A>
__device__ __forceinline__ Quat<T> staple(const Links<T> &U, const A &ad, int par)
{
    return staple_impl<T, MU, false>(U, ad, par, nullptr);
}

// Overrelaxation of one link from its staple V: U -> Vhat^+ U^+ Vhat^+
// (FP32 links renormalised).  Returns false, leaving `un` unset, when the
// link is kept (V = 0, or V not finite: then the flag is raised).  Every
// overrelaxation kernel forms the new link here.
template <class T>
__device__ __forceinline__ bool overrelax_reflect(const Quat<T> &V, const Quat<T> &u, uint32_t *flags, Quat<T> &un)
{
    const T k2 = V.w * V.w + V.x * V.x + V.y * V.y + V.z * V.z;
    const T k = sqrt(k2);
    if (!isfinite(k)) {
        atomicOr(flags, kFlagNonFinite);
        return false;
    }
    if (k == T(0))
        return false;
    const T inv = T(1) / k;
    const Quat<T> Vh = {V.w * inv, V.x * inv, V.y * inv, V.z * inv};
    const Quat<T> w = qmul(qmul(Vh, u), Vh);
    un = unitize(Quat<T>{w.w, -w.x, -w.y, -w.z});
    return true;
}

// (1/2) Tr(U W) for unit quaternions: the scalar part of the product.
template <class T>
__device__ __forceinline__ T half_trace(const Quat<T> &u, const Quat<T> &w)
{
    return u.w * w.w - u.x * w.x - u.y * w.y - u.z * w.z;
}

// Index of plane (nu, mu), nu < mu, in the order 01, 02, 03, 12, 13, 23.
__host__ __device__ constexpr int plane_index(int nu, int mu)
{
    return nu * (7 - nu) / 2 + (mu - nu - 1);
}

// The staple from a site's coordinates (any geometry).
template <class T, int MU>
__device__ __forceinline__ Quat<T> staple(const Links<T> &U, const Geom &g, const Site &s, uint32_t cb, int par)
{
    CbAddr ad;
    ad.s = s;
    ad.cb = cb;
    ad.g = &g;
    return staple<T, MU>(U, ad, par);
}

// Residency cap of the overrelaxation kernel on single lattices.  At the 7
// blocks per CU its registers allow, the blocks in flight on an XCD touch
// more links than its 4 MB L2 holds and neighbours are evicted between uses;
// 3 blocks per CU (12 waves) is the fastest for one large lattice (64^4
// class, FP32: 214.5 us at 3, 217.7 at 4, 246 at 2, ~227 uncapped; FP64:
// 471 / 475 / 490 / 521 us; 96^4 FP32: 1215 us at 3, 1220 at 4), and so
// it is for every single lattice measured down to 2^18 links per class
// (64^3 x 8: 24.1 against 27.3 us uncapped; 32^4 and 48^3 x 6: 1.5%).
// Below 2^17 links a class has at most two blocks per CU and the cap
// changes nothing.  The batched kernel over many lattices stays uncapped:
// there the cap costs more latency hiding than it saves (the 16-lattice
// scan, 0.1-2 M sites each: 12% slower at 4 blocks per CU, 21% at 3).  A
// waves-per-EU attribute cannot express the cap: that bounds the
// compiler's register budget, not the residency, and with the 67-82 VGPRs
// the FP32 kernel needs the hardware would still place 6 waves per SIMD.
// The cap is a static LDS reservation the kernel never touches:
// kOrBlocksPerCu blocks of it fit the CU's kLdsPerCu bytes (gfx950: 160 KB),
// one more does not.  (Requested as dynamic LDS of the same size at launch,
// it held the kernel lower than the cap: FP64 class 556 us against 487 us
// at a cap of 4.)  The launcher checks once per device, with the occupancy
// query, that the capped kernel runs exactly kOrBlocksPerCu blocks per CU,
// and launches the uncapped one where it does not.
constexpr int kOrBlocksPerCu = 3;
constexpr int kLdsPerCu = 160 * 1024;
constexpr int kOrResidencyLds = kLdsPerCu / kOrBlocksPerCu - 4 * 1024;
static_assert(kOrBlocksPerCu * kOrResidencyLds <= kLdsPerCu &&
                  (kOrBlocksPerCu + 1) * kOrResidencyLds > kLdsPerCu,
              "the reservation must admit exactly kOrBlocksPerCu blocks per CU");

__host__ inline bool residency_cap_pays(const Geom &g)
{
    return g.half >= (1u << 17);
}

// Lattices of a batch whose overrelaxation classes run as launches of their
// own, lattice by lattice, rather than inside the batched launches.  All
// classes of one such lattice run back to back, so its links stay in the
// 256 MB Infinity Cache between them (a 64^3 x 8 FP32 lattice holds
// 134 MB), where one launch per class over all lattices streams every
// lattice through it; and a lattice alone takes the residency cap, which
// slows the batched kernel (the 16-lattice scan: 21% at 3 blocks per CU).
// The scan's five 64^3 x 8 lattices, 4 sweeps: 4.60 ms batched, 4.85 ms as
// own launches class by class across the lattices, 3.91 ms lattice by
// lattice.  From 2^19 links per class (2048 blocks, 8 per CU), where a
// class is long enough to amortise its own launch.  (The heat bath stays
// batched: lattice by lattice it made the scan 1.5% slower.)
constexpr uint32_t kBatchOwnMinHalf = 1u << 19;

__host__ inline bool batch_own_launch(uint64_t volume)
{
    return volume / 2 >= kBatchOwnMinHalf;
}

__device__ __forceinline__ void reserve_lds_for_residency()
{
    __shared__ volatile char reservation[kOrResidencyLds];
    if (threadIdx.x == kBlock) // never true: keeps the reservation allocated
        reservation[0] = 0;
}

// ---------------------------------------------------------------------------
// Deterministic reductions: a fixed-order wave64 sum (DPP lane moves and
// scalar read-out), then the block's waves through LDS in a fixed order.
// ---------------------------------------------------------------------------
// A DPP lane move of a double within rows of 16 lanes (two 32-bit moves;
// every source lane of the controls used below is valid).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_double(double v, int lane)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave (all lanes active), returned in every
// lane, in a fixed order: pairs, quads, half rows and rows by DPP moves
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror),
// then the four row sums read out as scalars.  No LDS traffic.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_double<0xB1>(v);
    v += dpp_double<0x4E>(v);
    v += dpp_double<0x141>(v);
    v += dpp_double<0x140>(v);
    return (readlane_double(v, 0) + readlane_double(v, 16)) + (readlane_double(v, 32) + readlane_double(v, 48));
}

// Sum NV values over the block; thread 0 returns the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[NV])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        v[j] = wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j)
            lds[wave][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w)
                s += lds[w][j];
            v[j] = s;
        }
    }
}

} // namespace su2

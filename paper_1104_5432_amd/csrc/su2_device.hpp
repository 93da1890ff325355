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
constexpr uint32_t kMaxAttempts = 4096u;

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

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    return (__umulhi(n, f.m) + n) >> f.l;
}

// Order in which the threads of one checkerboard class walk its V/2 sites.
// A block takes 256 consecutive indices i of the walk; hardware blocks are
// renumbered (xcd_tile) so that each XCD takes one contiguous range of the
// walk.  In strip mode the walk visits (z,t) columns (C = Nx*Ny/2 cb indices
// each) strip by strip of W z-values, t-major inside a strip: the +-t halo
// of a column is W columns behind in the walk, still in the XCD's L2,
// instead of a whole t-slice behind.  Mode 0 walks plain cb order.  Every
// walk is a bijection onto the class, so results do not depend on it.
struct BlockOrder {
    uint32_t strip;  // 0 = plain cb order, else the strip width W (divides Nz)
    uint32_t cols;   // C
    uint32_t nz;     // Nz
    FastDiv div_cols, div_w, div_nt;
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
    uint32_t unused;
};

struct Site {
    int32_t c[4];  // x, y, z, t
    uint32_t site; // linear site index
};

// Coordinates of the cb-th site of the given parity.
__device__ __forceinline__ Site site_of_cb(const Geom &g, uint32_t cb, int parity)
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

__device__ __forceinline__ uint32_t cb_of(const Geom &g, int32_t x, int32_t y, int32_t z, int32_t t)
{
    return ((uint32_t)x >> 1) +
           g.nxh * ((uint32_t)y + (uint32_t)g.n[1] * ((uint32_t)z + (uint32_t)g.n[2] * (uint32_t)t));
}

__device__ __forceinline__ int32_t wrap_add(int32_t c, int32_t s, int32_t n)
{
    c += s;
    c = (c >= n) ? c - n : c;
    return (c < 0) ? c + n : c;
}

// cb index of the site displaced by (d0,d1,d2,d3) in {-1,0,1}.
__device__ __forceinline__ uint32_t cb_shift(const Geom &g, const int32_t c[4], int32_t d0, int32_t d1,
                                             int32_t d2, int32_t d3)
{
    return cb_of(g, wrap_add(c[0], d0, g.n[0]), wrap_add(c[1], d1, g.n[1]),
                 wrap_add(c[2], d2, g.n[2]), wrap_add(c[3], d3, g.n[3]));
}

// ---------------------------------------------------------------------------
// Link planes: plane q = 2 mu + parity, V/2 links each.
// ---------------------------------------------------------------------------
template <class T>
struct Links;

template <>
struct Links<float> {
    float4 *p;
    uint32_t half;
    __device__ __forceinline__ Quat<float> ld(int mu, int par, uint32_t cb) const
    {
        const float4 v = p[(size_t)(2 * mu + par) * half + cb];
        return {v.x, v.y, v.z, v.w};
    }
    __device__ __forceinline__ void st(int mu, int par, uint32_t cb, const Quat<float> &q) const
    {
        p[(size_t)(2 * mu + par) * half + cb] = make_float4(q.w, q.x, q.y, q.z);
    }
};

template <>
struct Links<double> {
    double2 *p;
    uint32_t half;
    __device__ __forceinline__ Quat<double> ld(int mu, int par, uint32_t cb) const
    {
        const size_t q = (size_t)(2 * mu + par);
        const double2 a = p[(2 * q) * half + cb];
        const double2 b = p[(2 * q + 1) * half + cb];
        return {a.x, a.y, b.x, b.y};
    }
    __device__ __forceinline__ void st(int mu, int par, uint32_t cb, const Quat<double> &v) const
    {
        const size_t q = (size_t)(2 * mu + par);
        p[(2 * q) * half + cb] = make_double2(v.w, v.x);
        p[(2 * q + 1) * half + cb] = make_double2(v.y, v.z);
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

// XCD-aware block order: consecutive blocks are dispatched round-robin over
// the 8 XCDs, each with its own L2; renumber so that each XCD works through
// one contiguous range of tiles (neighbouring tiles share halo links).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks)
{
    const uint32_t q = nblocks >> 3, r = nblocks & 7u;
    const uint32_t xcd = b & 7u, k = b >> 3;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// cb index of the i-th site of the walk.
__device__ __forceinline__ uint32_t walk_cb(uint32_t i, const BlockOrder &o)
{
    if (o.strip == 0)
        return i;
    const uint32_t j = fdiv(i, o.div_cols);
    const uint32_t off = i - j * o.cols;
    const uint32_t q = fdiv(j, o.div_w);
    const uint32_t zz = j - q * o.strip;
    const uint32_t s = fdiv(q, o.div_nt);
    const uint32_t t = q - s * o.div_nt.d;
    const uint32_t z = s * o.strip + zz;
    return off + o.cols * (z + o.nz * t);
}

// ---------------------------------------------------------------------------
// Staple sum of U_mu(x) (x of parity `par`, checkerboard index cb):
//   V = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
//                    + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
// so that the link's local action is -(beta/2) Tr(U_mu(x) V).
// ---------------------------------------------------------------------------
template <class T, int MU>
__device__ __forceinline__ Quat<T> staple(const Links<T> &U, const Geom &g, const Site &s, uint32_t cb,
                                          int par)
{
    const int opp = par ^ 1;
    const uint32_t cb_xp = cb_shift(g, s.c, MU == 0, MU == 1, MU == 2, MU == 3);
    Quat<T> V = {0, 0, 0, 0};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU)
            continue;
        const int32_t e0 = (nu == 0), e1 = (nu == 1), e2 = (nu == 2), e3 = (nu == 3);
        const int32_t m0 = (MU == 0), m1 = (MU == 1), m2 = (MU == 2), m3 = (MU == 3);
        const uint32_t cb_xpn = cb_shift(g, s.c, e0, e1, e2, e3);
        const uint32_t cb_xmn = cb_shift(g, s.c, -e0, -e1, -e2, -e3);
        const uint32_t cb_xpmn = cb_shift(g, s.c, m0 - e0, m1 - e1, m2 - e2, m3 - e3);
        // upper staple
        const Quat<T> a = U.ld(nu, opp, cb_xp);
        const Quat<T> b = U.ld(MU, opp, cb_xpn);
        const Quat<T> c = U.ld(nu, par, cb);
        qacc(V, qmul_nd(qmul_nd(a, b), c));
        // lower staple
        const Quat<T> d = U.ld(nu, par, cb_xpmn);
        const Quat<T> e = U.ld(MU, opp, cb_xmn);
        const Quat<T> f = U.ld(nu, opp, cb_xmn);
        qacc(V, qmul(qmul_dd(d, e), f));
    }
    return V;
}

} // namespace su2

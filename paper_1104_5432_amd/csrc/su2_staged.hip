// su2_staged.hip -- the update kernels with the staple neighbourhood of a
// slab staged in LDS (overrelaxation, with one or two threads per site, and
// heat bath; the slab plan and index arithmetic are in su2_staged.hpp).
// A block walks its slab slice by slice; for each slice it writes the
// links it loaded one or two slices earlier into LDS, issues the loads of
// a later slice (its share of the neighbourhood and, for overrelaxation,
// each site's own link) into registers and then forms every staple of the
// slice from LDS.  Each link of the class's neighbourhood is read from
// memory once per slab (the halo rows once more by the neighbouring slab)
// in contiguous 128-bit accesses along x: ~10 loads per update instead of
// 19.  The staple is formed with the products and sums of staple_impl, in
// its order, and the heat bath samples with the code of su2_heatbath.hpp,
// so the new links are bitwise those of the global-memory kernels.
#include "su2_device.hpp"
#include "su2_heatbath.hpp"
#include "su2_launch.hpp"
#include "su2_staged.hpp"

#include <mutex>

namespace su2 {

template <class T>
struct alignas(4 * sizeof(T)) LdsLink {
    T w, x, y, z;
};

template <class T>
__device__ __forceinline__ Quat<T> from_lds(const LdsLink<T> &l)
{
    return {l.w, l.x, l.y, l.z};
}

// Load links i = threadIdx.x, + blockDim.x, ... < total of arrays `which`
// (arrays 0-2 of slice sl_s, array 3 of slice sl_m) straight into LDS.
template <class T, int MU>
__device__ __forceinline__ void stage_direct(const Links<T> &U, const Geom &g, const StagePlan &p, LdsLink<T> *lds,
                                             uint32_t y0, uint32_t b0, int32_t s0, uint32_t which, int32_t sl_s,
                                             int32_t sl_m, int opp)
{
    const uint32_t total = load_count<MU>(p, which);
    for (uint32_t i = threadIdx.x; i < total; i += blockDim.x) {
        LoadItem it;
        if (load_item<MU>(g, p, y0, b0, s0, which, sl_s, sl_m, opp, i, it)) {
            const Quat<T> q = U.ld(it.dir, it.parity, it.cb);
            lds[it.lds] = {q.w, q.x, q.y, q.z};
        }
    }
}

// The staple of the site at slab-relative (a, b) of slice sl, parity par,
// from the LDS copies: the products and sums of staple_impl, in its order.
// rowbase[k] = staple_row_base(k, a, b) of the thread's site; xhv[0..2] the
// checkerboard x of the site displaced by -1, 0, +1 in x.  Everything else
// in an element's index is uniform over the block (scalar).
template <class T, int MU>
__device__ __forceinline__ Quat<T> staged_staple(const StagePlan &p, const LdsLink<T> *lds, int32_t s0, int32_t sl,
                                                 const uint32_t (&rowbase)[4], const uint32_t (&xhv)[3], int par)
{
    using R = Roles<MU>;
    using Ar = Arrays<MU>;
    auto link = [&](int d, int32_t ex, int32_t ea, int32_t eb, int32_t es) -> Quat<T> {
        const int k = Ar::array_of(d);
        const int q = par ^ ((ex + ea + eb + es) & 1);
        const uint32_t off = staple_shift(p, k, staple_slotq<MU>(k, sl + es, s0, q), ea, eb);
        return from_lds(lds[rowbase[k] + off + xhv[ex + 1]]);
    };
    constexpr int32_t mx = R::slot(MU) == 0, ma = R::slot(MU) == 1, mb = R::slot(MU) == 2, ms = R::slot(MU) == 3;
    Quat<T> V = {0, 0, 0, 0};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU)
            continue;
        const int sn = R::slot(nu);
        const int32_t ex = sn == 0, ea = sn == 1, eb = sn == 2, es = sn == 3;
        // upper staple U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        const Quat<T> la = link(nu, mx, ma, mb, ms);
        const Quat<T> lb = link(MU, ex, ea, eb, es);
        const Quat<T> lc = link(nu, 0, 0, 0, 0);
        const Quat<T> su = qmul_nd(qmul_nd(la, lb), lc);
        qacc(V, su);
        // lower staple U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        const Quat<T> ld = link(nu, mx - ex, ma - ea, mb - eb, ms - es);
        const Quat<T> le = link(MU, -ex, -ea, -eb, -es);
        const Quat<T> lf = link(nu, -ex, -ea, -eb, -es);
        const Quat<T> lo = qmul(qmul_dd(ld, le), lf);
        qacc(V, lo);
    }
    return V;
}

// Terms FIRST .. FIRST + 2 of the staple's six (upper and lower of each
// nu != MU in increasing nu: the order staged_staple adds them in), with
// its products.
template <class T, int MU, int FIRST>
__device__ __forceinline__ void staged_terms(const StagePlan &p, const LdsLink<T> *lds, int32_t s0, int32_t sl,
                                             const uint32_t (&rowbase)[4], const uint32_t (&xhv)[3], int par,
                                             Quat<T> (&out)[3])
{
    using R = Roles<MU>;
    using Ar = Arrays<MU>;
    auto link = [&](int d, int32_t ex, int32_t ea, int32_t eb, int32_t es) -> Quat<T> {
        const int k = Ar::array_of(d);
        const int q = par ^ ((ex + ea + eb + es) & 1);
        const uint32_t off = staple_shift(p, k, staple_slotq<MU>(k, sl + es, s0, q), ea, eb);
        return from_lds(lds[rowbase[k] + off + xhv[ex + 1]]);
    };
    constexpr int32_t mx = R::slot(MU) == 0, ma = R::slot(MU) == 1, mb = R::slot(MU) == 2, ms = R::slot(MU) == 3;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == MU)
            continue;
        const int j = nu < MU ? nu : nu - 1; // position of nu among the three
        const int sn = R::slot(nu);
        const int32_t ex = sn == 0, ea = sn == 1, eb = sn == 2, es = sn == 3;
        if (2 * j >= FIRST && 2 * j < FIRST + 3) {
            const Quat<T> la = link(nu, mx, ma, mb, ms);
            const Quat<T> lb = link(MU, ex, ea, eb, es);
            const Quat<T> lc = link(nu, 0, 0, 0, 0);
            out[2 * j - FIRST] = qmul_nd(qmul_nd(la, lb), lc);
        }
        if (2 * j + 1 >= FIRST && 2 * j + 1 < FIRST + 3) {
            const Quat<T> ld = link(nu, mx - ex, ma - ea, mb - eb, ms - es);
            const Quat<T> le = link(MU, -ex, -ea, -eb, -es);
            const Quat<T> lf = link(nu, -ex, -ea, -eb, -es);
            out[2 * j + 1 - FIRST] = qmul(qmul_dd(ld, le), lf);
        }
    }
}

// Two threads per site: the slab walk and LDS ring of overrelax_staged_kernel
// below with 2 x sites threads, so that twice as many waves (4 per SIMD at
// 512 sites) hide the memory latency of the slice being loaded.  The first
// `sites` threads form staple terms 0-2 of their site, the second `sites`
// threads terms 3-5, which they hand over through LDS (xch, after the
// ring, term-major so that consecutive lanes touch consecutive links); the
// first adds them in the same order, so the new link is bitwise
// that of the one-thread kernel.  All threads share the loads of the next
// slice; the first ones also hold their site's own link.
template <class T, int MU>
__global__ __launch_bounds__(kStagedPairThreads) void overrelax_staged2_kernel(Links<T> U, Geom g, StagePlan p,
                                                                               int par, uint32_t *flags)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    LdsLink<T> *lds = reinterpret_cast<LdsLink<T> *>(lds_raw);
    LdsLink<T> *xch = reinterpret_cast<LdsLink<T> *>(lds_raw + p.lds_bytes);
    const int opp = par ^ 1;

    const uint32_t j = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t ia = j % p.na, ib = (j / p.na) % p.nb, is = j / (p.na * p.nb);
    const uint32_t y0 = ia * p.A, b0 = ib * p.B;
    const int32_t s0 = (int32_t)(is * p.S);
    const uint32_t nx = (uint32_t)g.n[0];
    const int32_t nsl = g.n[Roles<MU>::s];

    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 1u, s0 - 1, 0, opp);
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 8u, 0, s0 - 1, opp);
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 8u, 0, s0, opp);

    // the thread's site (blockDim.x = 2 x sites) and half of its staple
    const uint32_t sites = p.A * p.B * p.nxh;
    const bool second = threadIdx.x >= sites; // wave-uniform: sites is a multiple of 64
    const uint32_t site_i = second ? threadIdx.x - sites : threadIdx.x;
    const uint32_t xh = site_i % p.nxh, row = site_i / p.nxh;
    const int32_t a = (int32_t)(row % p.A), b = (int32_t)(row / p.A);
    const uint32_t yb = y0 + (uint32_t)a + b0 + (uint32_t)b;
    const uint32_t own_cb0 = xh + p.nxh * global_row_base<MU>(g, y0, b0, a, b);
    uint32_t rowbase[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        rowbase[k] = staple_row_base<MU>(p, k, a, b);

    constexpr int kPre = kStagedPairPrefetch;
    LoadBase lb[kPre];
#pragma unroll
    for (int r = 0; r < kPre; ++r) {
        const uint32_t i = threadIdx.x + (uint32_t)r * blockDim.x;
        if (!(i < p.n_fresh && load_base<MU>(g, p, y0, b0, opp, i, lb[r])))
            lb[r].info = 0xffffffffu;
    }
    constexpr int kDepth = 2;
    Quat<T> pre[kDepth][kPre];
    Quat<T> pre_own[kDepth];
    auto prefetch = [&](int32_t sl, Quat<T>(&buf)[kPre], Quat<T> &own_out) {
        const SliceTerms t = slice_terms<MU>(g, p, s0, sl);
        if (!second)
            own_out = U.ld_nt(MU, par, own_cb0 + t.cb_s);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            if (lb[r].info != 0xffffffffu) {
                uint32_t cb, li;
                load_at(lb[r], t, cb, li);
                const int plane = (int)(lb[r].info & 0xffu);
                buf[r] = U.ld(plane >> 1, plane & 1, cb);
            }
        }
    };
    const int32_t s_end = s0 + (int32_t)p.S;
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
        pre_own[d] = {1, 0, 0, 0};
        if (s0 + d < s_end)
            prefetch(s0 + d, pre[d], pre_own[d]);
    }

    auto slice = [&](int32_t sl, int d) {
        const SliceTerms t = slice_terms<MU>(g, p, s0, sl);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            if (lb[r].info != 0xffffffffu) {
                uint32_t cb, li;
                load_at(lb[r], t, cb, li);
                lds[li] = {pre[d][r].w, pre[d][r].x, pre[d][r].y, pre[d][r].z};
            }
        }
        const Quat<T> own = pre_own[d];
        __syncthreads();
        if (sl + kDepth < s_end)
            prefetch(sl + kDepth, pre[d], pre_own[d]);
        const uint32_t sc = (uint32_t)(sl < nsl ? sl : sl - nsl);
        const uint32_t xs = 2u * xh + ((yb + sc + (uint32_t)par) & 1u);
        const uint32_t xhv[3] = {shifted_xh(xs, -1, nx), xh, shifted_xh(xs, 1, nx)};
        Quat<T> term[3];
        if (second) {
            staged_terms<T, MU, 3>(p, lds, s0, sl, rowbase, xhv, par, term);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                xch[(uint32_t)k * sites + site_i] = {term[k].w, term[k].x, term[k].y, term[k].z};
        } else {
            staged_terms<T, MU, 0>(p, lds, s0, sl, rowbase, xhv, par, term);
        }
        __syncthreads();
        if (!second) {
            Quat<T> V = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < 3; ++k)
                qacc(V, term[k]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                qacc(V, from_lds(xch[(uint32_t)k * sites + site_i]));
            Quat<T> un;
            if (overrelax_reflect(V, own, flags, un))
                U.st(MU, par, own_cb0 + t.cb_s, un);
        }
    };
    for (int32_t sl = s0; sl < s_end; sl += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d)
            if (sl + d < s_end)
                slice(sl + d, d);
    }
}

// One class (MU, par) of overrelaxation, slab by slab.  Grid: one block per
// slab (na x nb x ns), kStagedThreads threads, p.lds_bytes of dynamic LDS.
template <class T, int MU>
__global__ __launch_bounds__(kStagedThreads) void overrelax_staged_kernel(Links<T> U, Geom g, StagePlan p, int par,
                                                                          uint32_t *flags)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    LdsLink<T> *lds = reinterpret_cast<LdsLink<T> *>(lds_raw);
    const int opp = par ^ 1;

    // the block's slab (XCD-aware: each XCD takes neighbouring slabs)
    const uint32_t j = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t ia = j % p.na, ib = (j / p.na) % p.nb, is = j / (p.na * p.nb);
    const uint32_t y0 = ia * p.A, b0 = ib * p.B;
    const int32_t s0 = (int32_t)(is * p.S);
    const uint32_t nx = (uint32_t)g.n[0];
    const int32_t nsl = g.n[Roles<MU>::s];

    // prologue: the s-direction links of slice s0 - 1, the mu-links of
    // slices s0 - 1 and s0
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 1u, s0 - 1, 0, opp);
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 8u, 0, s0 - 1, opp);
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 8u, 0, s0, opp);

    // the thread's site in every slice (sites <= threads)
    const uint32_t sites = p.A * p.B * p.nxh;
    const bool active = threadIdx.x < sites;
    const uint32_t xh = threadIdx.x % p.nxh, row = threadIdx.x / p.nxh;
    const int32_t a = (int32_t)(row % p.A), b = (int32_t)(row / p.A);
    const uint32_t yb = y0 + (uint32_t)a + b0 + (uint32_t)b; // y + b of the site
    const uint32_t own_cb0 = xh + p.nxh * global_row_base<MU>(g, y0, b0, a, b);
    uint32_t rowbase[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        rowbase[k] = staple_row_base<MU>(p, k, a, b);

    // the thread's share of each slice's loads (arrays 0-2 of slice sl,
    // array 3 of sl + 1), decoded once; the next slice's share and own link
    // are held in registers
    constexpr int kPre = staged_prefetch(sizeof(T) * 4);
    LoadBase lb[kPre];
#pragma unroll
    for (int r = 0; r < kPre; ++r) {
        const uint32_t i = threadIdx.x + (uint32_t)r * kStagedThreads;
        if (!(i < p.n_fresh && load_base<MU>(g, p, y0, b0, opp, i, lb[r])))
            lb[r].info = 0xffffffffu;
    }
    // Two register buffers, so that a slice's loads are issued two slices
    // before the slice is written to LDS (FP32; FP64 keeps one, its links
    // taking twice the registers).
    constexpr int kDepth = sizeof(T) == 4 ? 2 : 1;
    Quat<T> pre[kDepth][kPre];
    Quat<T> pre_own[kDepth];
    auto prefetch = [&](int32_t sl, Quat<T>(&buf)[kPre], Quat<T> &own_out) {
        const SliceTerms t = slice_terms<MU>(g, p, s0, sl);
        if (active)
            own_out = U.ld_nt(MU, par, own_cb0 + t.cb_s);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            if (lb[r].info != 0xffffffffu) {
                uint32_t cb, li;
                load_at(lb[r], t, cb, li);
                const int plane = (int)(lb[r].info & 0xffu);
                buf[r] = U.ld(plane >> 1, plane & 1, cb);
            }
        }
    };
    const int32_t s_end = s0 + (int32_t)p.S;
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
        pre_own[d] = {1, 0, 0, 0};
        if (s0 + d < s_end)
            prefetch(s0 + d, pre[d], pre_own[d]);
    }

    // slice sl from buffer d: write its share to LDS, issue the loads of
    // slice sl + kDepth into the same buffer, update the slice
    auto slice = [&](int32_t sl, int d) {
        const SliceTerms t = slice_terms<MU>(g, p, s0, sl);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            if (lb[r].info != 0xffffffffu) {
                uint32_t cb, li;
                load_at(lb[r], t, cb, li);
                lds[li] = {pre[d][r].w, pre[d][r].x, pre[d][r].y, pre[d][r].z};
            }
        }
        const Quat<T> own = pre_own[d];
        __syncthreads();
        if (sl + kDepth < s_end)
            prefetch(sl + kDepth, pre[d], pre_own[d]);
        if (active) {
            // x of the site from its row's parity offset, and its neighbours'
            const uint32_t sc = (uint32_t)(sl < nsl ? sl : sl - nsl);
            const uint32_t xs = 2u * xh + ((yb + sc + (uint32_t)par) & 1u);
            const uint32_t xhv[3] = {shifted_xh(xs, -1, nx), xh, shifted_xh(xs, 1, nx)};
            const Quat<T> V = staged_staple<T, MU>(p, lds, s0, sl, rowbase, xhv, par);
            Quat<T> un;
            if (overrelax_reflect(V, own, flags, un))
                U.st(MU, par, own_cb0 + t.cb_s, un);
        }
        __syncthreads();
    };
    for (int32_t sl = s0; sl < s_end; sl += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d)
            if (sl + d < s_end)
                slice(sl + d, d);
    }
}

// One class (MU, par) of the heat bath, slab by slab: the slab walk, LDS
// ring and register prefetch of the overrelaxation kernel above (without
// the own link, which the heat bath does not read), and per slice the
// sampling of su2_heatbath.hpp with the block's rejected lanes compacted
// across all its threads.  The staple, the random words (keyed by the
// site) and the sampling are those of the global-memory kernel, so the new
// links are bitwise its links.
template <class T, int MU>
__global__ __launch_bounds__(kStagedThreads) void heatbath_staged_kernel(Links<T> U, Geom g, StagePlan p, int par,
                                                                         double beta, uint32_t k0, uint32_t k1,
                                                                         uint32_t c1, uint32_t sweep,
                                                                         const uint32_t *d_sweep, uint32_t *flags)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    LdsLink<T> *lds = reinterpret_cast<LdsLink<T> *>(lds_raw);
    __shared__ HbSharedT<kStagedThreads> sh;
    const int opp = par ^ 1;
    const uint32_t sw = d_sweep ? *d_sweep : sweep;

    const uint32_t j = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t ia = j % p.na, ib = (j / p.na) % p.nb, is = j / (p.na * p.nb);
    const uint32_t y0 = ia * p.A, b0 = ib * p.B;
    const int32_t s0 = (int32_t)(is * p.S);
    const uint32_t nx = (uint32_t)g.n[0];
    const int32_t nsl = g.n[Roles<MU>::s];

    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 1u, s0 - 1, 0, opp);
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 8u, 0, s0 - 1, opp);
    stage_direct<T, MU>(U, g, p, lds, y0, b0, s0, 8u, 0, s0, opp);

    const uint32_t sites = p.A * p.B * p.nxh;
    const bool active = threadIdx.x < sites;
    const uint32_t xh = threadIdx.x % p.nxh, row = threadIdx.x / p.nxh;
    const int32_t a = (int32_t)(row % p.A), b = (int32_t)(row / p.A);
    const uint32_t yb = y0 + (uint32_t)a + b0 + (uint32_t)b;
    const uint32_t own_cb0 = xh + p.nxh * global_row_base<MU>(g, y0, b0, a, b);
    uint32_t rowbase[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        rowbase[k] = staple_row_base<MU>(p, k, a, b);

    constexpr int kPre = staged_prefetch(sizeof(T) * 4);
    LoadBase lb[kPre];
#pragma unroll
    for (int r = 0; r < kPre; ++r) {
        const uint32_t i = threadIdx.x + (uint32_t)r * kStagedThreads;
        if (!(i < p.n_fresh && load_base<MU>(g, p, y0, b0, opp, i, lb[r])))
            lb[r].info = 0xffffffffu;
    }
    // one slice of loads ahead: the sampler needs the registers a second
    // buffer would take (with two, the FP32 kernel spills)
    constexpr int kDepth = 1;
    Quat<T> pre[kDepth][kPre];
    auto prefetch = [&](int32_t sl, Quat<T>(&buf)[kPre]) {
        const SliceTerms t = slice_terms<MU>(g, p, s0, sl);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            if (lb[r].info != 0xffffffffu) {
                uint32_t cb, li;
                load_at(lb[r], t, cb, li);
                const int plane = (int)(lb[r].info & 0xffu);
                buf[r] = U.ld(plane >> 1, plane & 1, cb);
            }
        }
    };
    const int32_t s_end = s0 + (int32_t)p.S;
#pragma unroll
    for (int d = 0; d < kDepth; ++d)
        if (s0 + d < s_end)
            prefetch(s0 + d, pre[d]);

    auto slice = [&](int32_t sl, int d) {
        const SliceTerms t = slice_terms<MU>(g, p, s0, sl);
#pragma unroll
        for (int r = 0; r < kPre; ++r) {
            if (lb[r].info != 0xffffffffu) {
                uint32_t cb, li;
                load_at(lb[r], t, cb, li);
                lds[li] = {pre[d][r].w, pre[d][r].x, pre[d][r].y, pre[d][r].z};
            }
        }
        __syncthreads();
        if (sl + kDepth < s_end)
            prefetch(sl + kDepth, pre[d]);
        Quat<T> Vh = {1, 0, 0, 0};
        double alpha = 0.0;
        bool need = false;
        uint32_t site = 0;
        U32x4 r0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0};
        const uint32_t cb = own_cb0 + t.cb_s;
        if (active) {
            const uint32_t sc = (uint32_t)(sl < nsl ? sl : sl - nsl);
            const uint32_t xs = 2u * xh + ((yb + sc + (uint32_t)par) & 1u);
            const uint32_t xhv[3] = {shifted_xh(xs, -1, nx), xh, shifted_xh(xs, 1, nx)};
            const Quat<T> V = staged_staple<T, MU>(p, lds, s0, sl, rowbase, xhv, par);
            site = 2u * cb + (xs & 1u);
            need = hb_staple_law<T>(V, beta, flags, Vh, alpha);
            r0 = philox(site, c1, sw, 0u, k0, k1);
            r1 = philox(site, c1, sw, 1u, k0, k1);
        }
        double x0 = 0.0, xlen = 0.0;
        if (hb_sample<T, kStagedThreads>(need, alpha, site, r0, r1, c1, sw, k0, k1, flags, sh, x0, xlen)) {
            const Quat<T> X = Direction<T>::make(x0, xlen, philox(site, c1, sw, 2u, k0, k1));
            U.st(MU, par, cb, unitize(qmul_nd(X, Vh)));
        }
        __syncthreads();
    };
    for (int32_t sl = s0; sl < s_end; sl += kDepth) {
#pragma unroll
        for (int d = 0; d < kDepth; ++d)
            if (sl + d < s_end)
                slice(sl + d, d);
    }
}

// ---------------------------------------------------------------------------
// Launcher.
// ---------------------------------------------------------------------------
// Dynamic LDS a block may take on the current device (read once per device).
static uint32_t lds_per_block_limit()
{
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static int cached[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return 0;
    std::lock_guard<std::mutex> hold(lock);
    if (cached[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = -1;
        cached[dev] = v;
    }
    return cached[dev] > 0 ? (uint32_t)cached[dev] : 0u;
}

// static_lds: the kernel's own LDS besides the ring (the heat bath's
// compaction state).
template <int MU>
static bool plan_for(const LaunchArgs &a, uint32_t static_lds, StagePlan &p)
{
    const uint32_t link_bytes = a.prec == kF32 ? 16u : 32u;
    const uint32_t device_limit = lds_per_block_limit();
    if (device_limit <= static_lds)
        return false;
    const uint32_t limit = device_limit - static_lds;
    // one slab per CU if the lattice allows it, else as many as it allows
    for (uint32_t min_blocks : {256u, 64u, 1u})
        if (make_stage_plan<MU>(a.n, link_bytes, limit, min_blocks, p))
            return true;
    return false;
}

template <class T, int MU>
static bool launch_staged_or(const LaunchArgs &a, int par, hipStream_t st)
{
    Links<T> U;
    U.p = reinterpret_cast<decltype(U.p)>(a.links);
    U.stride = plane_stride((uint32_t)(a.volume / 2), sizeof(T) == 8);
    const Geom g = make_geom(a.n, 0, 0);
    // FP32: two threads per site where the ring and the hand-over area fit
    // (the latter sized for the largest slab, 512 sites x 3 terms).  FP64
    // keeps one thread per site: its ring leaves no room for the hand-over
    // at the benchmarked sizes, and its loads would not fit 4 waves' registers.
    if constexpr (sizeof(T) == 4) {
        const uint32_t xch_max = 3u * 512u * (uint32_t)sizeof(LdsLink<T>);
        StagePlan q;
        if (plan_for<MU>(a, xch_max, q)) {
            const uint32_t sites = q.A * q.B * q.nxh;
            if (2u * sites <= (uint32_t)kStagedPairThreads && q.n_fresh <= 2u * sites * kStagedPairPrefetch) {
                const uint32_t lds_bytes = q.lds_bytes + 3u * sites * (uint32_t)sizeof(LdsLink<T>);
                overrelax_staged2_kernel<T, MU><<<q.na * q.nb * q.ns, 2u * sites, lds_bytes, st>>>(U, g, q, par,
                                                                                                    a.flags);
                return true;
            }
        }
    }
    StagePlan p;
    if (!plan_for<MU>(a, 0u, p))
        return false;
    overrelax_staged_kernel<T, MU><<<p.na * p.nb * p.ns, kStagedThreads, p.lds_bytes, st>>>(U, g, p, par, a.flags);
    return true;
}

template <class T>
static bool launch_staged_or_t(const LaunchArgs &a, int mu, int par, hipStream_t st)
{
    switch (mu) {
    case 0: return launch_staged_or<T, 0>(a, par, st);
    case 1: return launch_staged_or<T, 1>(a, par, st);
    case 2: return launch_staged_or<T, 2>(a, par, st);
    default: return launch_staged_or<T, 3>(a, par, st);
    }
}

template <class T, int MU>
static bool launch_staged_hb(const LaunchArgs &a, int par, double beta, uint64_t seed, uint32_t sweep,
                             const uint32_t *d_sweep, hipStream_t st)
{
    StagePlan p;
    if (!plan_for<MU>(a, (uint32_t)sizeof(HbSharedT<kStagedThreads>), p))
        return false;
    Links<T> U;
    U.p = reinterpret_cast<decltype(U.p)>(a.links);
    U.stride = plane_stride((uint32_t)(a.volume / 2), sizeof(T) == 8);
    const Geom g = make_geom(a.n, 0, 0);
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const uint32_t c1 = (uint32_t)MU + 4u * 1u + 16u * (uint32_t)a.lattice_id;
    heatbath_staged_kernel<T, MU><<<p.na * p.nb * p.ns, kStagedThreads, p.lds_bytes, st>>>(
        U, g, p, par, beta, k0, k1, c1, sweep, d_sweep, a.flags);
    return true;
}

template <class T>
static bool launch_staged_hb_t(const LaunchArgs &a, int mu, int par, double beta, uint64_t seed, uint32_t sweep,
                               const uint32_t *d_sweep, hipStream_t st)
{
    switch (mu) {
    case 0: return launch_staged_hb<T, 0>(a, par, beta, seed, sweep, d_sweep, st);
    case 1: return launch_staged_hb<T, 1>(a, par, beta, seed, sweep, d_sweep, st);
    case 2: return launch_staged_hb<T, 2>(a, par, beta, seed, sweep, d_sweep, st);
    default: return launch_staged_hb<T, 3>(a, par, beta, seed, sweep, d_sweep, st);
    }
}

bool launch_heatbath_staged(const LaunchArgs &a, double beta, uint64_t seed, uint32_t sweep, const uint32_t *d_sweep,
                            int mu, int par, hipStream_t st)
{
    return a.prec == kF32 ? launch_staged_hb_t<float>(a, mu, par, beta, seed, sweep, d_sweep, st)
                          : launch_staged_hb_t<double>(a, mu, par, beta, seed, sweep, d_sweep, st);
}

bool launch_overrelax_staged(const LaunchArgs &a, int mu, int par, hipStream_t st)
{
    return a.prec == kF32 ? launch_staged_or_t<float>(a, mu, par, st) : launch_staged_or_t<double>(a, mu, par, st);
}

} // namespace su2

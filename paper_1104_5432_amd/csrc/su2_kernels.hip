// su2_kernels.hip -- gfx950 update kernels of the SU(2) library (starts,
// heat bath, overrelaxation, single and batched) and their launchers.  One
// thread per link of a checkerboard class (mu, parity): the links of one
// class never appear in each other's staples, so a class is updated in one
// launch without synchronisation.
#include "su2_device.hpp"
#include "su2_heatbath.hpp"
#include "su2_launch.hpp"

#include <cstring>
#include <mutex>
#include <type_traits>

namespace su2 {

// Heat bath for one class (the sampling in su2_heatbath.hpp): one thread per
// link; the block compacts its rejected lanes for the retries.
// Plaquette of the configuration a sweep leaves, from its last classes: in
// class (MU, odd) every link of the plaquettes of planes (nu, MU), nu < MU,
// is final, and each of those plaquettes holds exactly one odd MU-link, so
// classes (1,odd), (2,odd), (3,odd) of the last sweep count all six planes
// once.  Each thread takes (1/2)Tr of the new link with the recorded sum of
// the two staple products of each such plane (FP64 from the half trace on,
// as in the plaquette kernel) and the block writes one partial per plane.
template <class T, int MU>
__device__ __forceinline__ void plaquette_partials(const Quat<T> &u, const PlaneTerms<T> &terms, bool valid,
                                                   double *partials)
{
    constexpr int NP = MU > 0 ? MU : 1;
    __shared__ double lds[kBlock / 64][NP];
    double acc[NP];
#pragma unroll
    for (int nu = 0; nu < NP; ++nu)
        acc[nu] = valid ? (double)half_trace(u, terms.s[nu]) : 0.0;
    block_sum<NP>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int nu = 0; nu < NP; ++nu)
            partials[(size_t)plane_index(nu, MU) * gridDim.x + blockIdx.x] = acc[nu];
}

template <class T, int MU, bool COL, bool PLAQ = false>
__device__ __forceinline__ void heatbath_body(const Links<T> &U, const Geom &g, int par, double beta,
                                              uint32_t k0, uint32_t k1, uint32_t c1, uint32_t sweep,
                                              uint32_t *flags, uint32_t b, uint32_t nblocks, HbShared &sh,
                                              double *plaq_partials = nullptr)
{
    const uint32_t i = xcd_tile(b, nblocks) * kBlock + threadIdx.x;
    const bool valid = i < g.half;

    uint32_t own = 0, site = 0; // own: byte offset (COL) or cb index of the link
    Quat<T> Vh = {1, 0, 0, 0};
    double alpha = 0.0;
    bool need = false;
    PlaneTerms<T> terms;
    // Random words of attempt 0 (counters 0, 1) and of the direction
    // (counter 2): they do not depend on the staple, so for FP32 links with
    // column addressing they are drawn between issuing the staple's loads
    // and using them, while the loads are in flight (64^4 class: 213.5 ->
    // 208.7 us).  FP64 keeps the staple's interleaved loads and draws in the
    // order they are used: holding all 18 links would take 179 VGPRs and
    // halve its occupancy, and drawing the words while only the first
    // plane's six links are in flight (125 VGPRs, as now) made the 64^4
    // class slower, 466 against 455 us.
    U32x4 r0 = {0, 0, 0, 0}, r1 = {0, 0, 0, 0}, rdir = {0, 0, 0, 0};
    if (valid) {
        Quat<T> V;
        if constexpr (COL) {
            const ColAddr ad = col_addr(g, i, par);
            own = ad.at(0, 0, 0, 0);
            site = ad.site();
            if constexpr (std::is_same<T, float>::value) {
                Quat<T> L[4][6];
                staple_load<T, MU>(U, ad, par, L);
                __builtin_amdgcn_sched_barrier(0);
                r0 = philox(site, c1, sweep, 0u, k0, k1);
                r1 = philox(site, c1, sweep, 1u, k0, k1);
                rdir = philox(site, c1, sweep, 2u, k0, k1);
                __builtin_amdgcn_sched_barrier(0);
                V = staple_compute<T, MU, PLAQ>(L, &terms);
            } else {
                V = staple_impl<T, MU, PLAQ>(U, ad, par, &terms);
                r0 = philox(site, c1, sweep, 0u, k0, k1);
                r1 = philox(site, c1, sweep, 1u, k0, k1);
            }
        } else {
            own = walk_cb(i, g.ord);
            CbAddr ad;
            ad.s = site_of_cb(g, own, par);
            ad.cb = own;
            ad.g = &g;
            site = ad.s.site;
            V = staple_impl<T, MU, PLAQ>(U, ad, par, &terms);
            r0 = philox(site, c1, sweep, 0u, k0, k1);
            r1 = philox(site, c1, sweep, 1u, k0, k1);
        }
        need = hb_staple_law<T>(V, beta, flags, Vh, alpha);
    }
    double x0 = 0.0, xlen = 0.0;
    const bool ok = hb_sample<T, kBlock>(need, alpha, site, r0, r1, c1, sweep, k0, k1, flags, sh, x0, xlen);
    Quat<T> Un = {1, 0, 0, 0};
    if (ok) {
        if constexpr (!(COL && std::is_same<T, float>::value))
            rdir = philox(site, c1, sweep, 2u, k0, k1);
        const Quat<T> X = Direction<T>::make(x0, xlen, rdir);
        Un = unitize(qmul_nd(X, Vh));
        if constexpr (COL)
            U.stb(MU, par, own, Un);
        else
            U.st(MU, par, own, Un);
    }
    if constexpr (PLAQ && MU > 0) {
        if (valid && !ok) // the link was kept
            Un = COL ? U.ldb(MU, par, own) : U.ld(MU, par, own);
        plaquette_partials<T, MU>(Un, terms, valid, plaq_partials);
    }
}

// ---------------------------------------------------------------------------
// Overrelaxation for one class: U -> Vhat^+ U^+ Vhat^+ = (Vhat U Vhat)^+.
// ---------------------------------------------------------------------------
template <class T, int MU, bool PLAQ, class A>
__device__ __forceinline__ Quat<T> overrelax_link(const Links<T> &U, const A &ad, int par, uint32_t *flags,
                                                  PlaneTerms<T> *terms)
{
    // The link being replaced is read by this update only (non-temporal).
    // FP32: its load is issued before the staple's loads; left to the
    // scheduler it is sunk to its use after the staple algebra, which
    // exposes a second memory round trip per wave (64^4 class: 218.5 ->
    // 216.0 us).  FP64 keeps the sunk load: issued first, the FP64 class
    // took 4.5% longer (485 -> 507 us) and fetched 6% more bytes beyond L2
    // (with skewed sub-planes and 3 blocks per CU: 473 -> 481 us).
    const uint32_t own = ad.at(0, 0, 0, 0);
    Quat<T> u;
    if constexpr (std::is_same<T, float>::value) {
        u = ad.ld_nt(U, MU, par, own);
        __builtin_amdgcn_sched_barrier(0);
    }
    const Quat<T> V = staple_impl<T, MU, PLAQ>(U, ad, par, terms);
    if constexpr (!std::is_same<T, float>::value)
        u = ad.ld_nt(U, MU, par, own);
    Quat<T> un;
    if (!overrelax_reflect(V, u, flags, un))
        return u;
    ad.st(U, MU, par, own, un);
    return un;
}

template <class T, int MU, bool COL, bool PLAQ = false>
__device__ __forceinline__ void overrelax_body(const Links<T> &U, const Geom &g, int par, uint32_t *flags,
                                               uint32_t b, uint32_t nblocks, double *plaq_partials = nullptr)
{
    const uint32_t i = xcd_tile(b, nblocks) * kBlock + threadIdx.x;
    const bool valid = i < g.half;
    if constexpr (!PLAQ) {
        if (!valid)
            return;
    }
    PlaneTerms<T> terms;
    Quat<T> un = {1, 0, 0, 0};
    if (valid) {
        if constexpr (COL) {
            un = overrelax_link<T, MU, PLAQ>(U, col_addr(g, i, par), par, flags, &terms);
        } else {
            CbAddr ad;
            ad.cb = walk_cb(i, g.ord);
            ad.s = site_of_cb(g, ad.cb, par);
            ad.g = &g;
            un = overrelax_link<T, MU, PLAQ>(U, ad, par, flags, &terms);
        }
    }
    if constexpr (PLAQ && MU > 0)
        plaquette_partials<T, MU>(un, terms, valid, plaq_partials);
}

// ---------------------------------------------------------------------------
// Kernels: one lattice, or a batch of lattices in one launch.  A batch is a
// device table of BatchEntry (geometry, links, beta, lattice id, flags and
// the lattice's range of blocks, a multiple of 8 so that every lattice keeps
// its XCD-aligned walk); a block looks its lattice up in the table.
// The heat-bath sweep index is read from device memory when `d_sweep` is
// given, so a captured graph can be replayed sweep after sweep.
// ---------------------------------------------------------------------------
template <class T, int MU, bool COL, bool PLAQ>
__global__ __launch_bounds__(kBlock) void heatbath_kernel(Links<T> U, Geom g, int par, double beta,
                                                           uint32_t k0, uint32_t k1, uint32_t c1,
                                                           uint32_t sweep, const uint32_t *d_sweep,
                                                           uint32_t *flags, double *plaq_partials)
{
    __shared__ HbShared sh;
    const uint32_t sw = d_sweep ? *d_sweep : sweep;
    heatbath_body<T, MU, COL, PLAQ>(U, g, par, beta, k0, k1, c1, sw, flags, blockIdx.x, gridDim.x, sh,
                                    plaq_partials);
}

template <class T, int MU, bool COL, bool CAP, bool PLAQ>
__global__ __launch_bounds__(kBlock) void overrelax_kernel(Links<T> U, Geom g, int par, uint32_t *flags,
                                                            double *plaq_partials)
{
    if constexpr (CAP)
        reserve_lds_for_residency();
    overrelax_body<T, MU, COL, PLAQ>(U, g, par, flags, blockIdx.x, gridDim.x, plaq_partials);
}

// The lattice of block b of a batched grid: the entries' first blocks
// (block0 over all lattices, sub_block0 over those without launches of
// their own, where such a lattice has an empty range starting where the
// next lattice's does) never decrease, so it is the last entry whose first
// block is <= b.  One round of independent loads for up to 64 lattices
// instead of a chain of dependent ones (which, exposed at low residency,
// cost more than the update).
template <uint32_t BatchEntry::*FIRST>
__device__ __forceinline__ const BatchEntry &find_entry(const BatchEntry *tab, int count, uint32_t b)
{
    return tab[find_entry_index<FIRST>(tab, count, b)];
}

// Block `rel` (0 .. e.nblocks - 1) of the lattice's heat-bath class.
template <class T, int MU>
__device__ __forceinline__ void heatbath_item(const BatchEntry &e, int par, uint32_t k0, uint32_t k1, uint32_t sw,
                                              uint32_t rel, HbShared &sh)
{
    Links<T> U;
    U.p = reinterpret_cast<decltype(U.p)>(e.links);
    U.stride = plane_stride(e.g.half, sizeof(T) == 8);
    const uint32_t c1 = (uint32_t)MU + 4u * 1u + e.lid16;
    if (e.col)
        heatbath_body<T, MU, true>(U, e.g, par, e.beta, k0, k1, c1, sw, e.flags, rel, e.nblocks, sh);
    else
        heatbath_body<T, MU, false>(U, e.g, par, e.beta, k0, k1, c1, sw, e.flags, rel, e.nblocks, sh);
}

// Block `rel` (0 .. e.nblocks - 1) of the lattice's overrelaxation class.
template <class T, int MU>
__device__ __forceinline__ void overrelax_item(const BatchEntry &e, int par, uint32_t rel)
{
    Links<T> U;
    U.p = reinterpret_cast<decltype(U.p)>(e.links);
    U.stride = plane_stride(e.g.half, sizeof(T) == 8);
    if (e.col)
        overrelax_body<T, MU, true>(U, e.g, par, e.flags, rel, e.nblocks);
    else
        overrelax_body<T, MU, false>(U, e.g, par, e.flags, rel, e.nblocks);
}

// A heat-bath class of every lattice of the batch (the grid of block0
// ranges).  Unlike the overrelaxation it gains nothing from launches of its
// own per large lattice (the scan: 1.5% slower that way).
template <class T, int MU>
__global__ __launch_bounds__(kBlock) void heatbath_batch_kernel(const BatchEntry *tab, int count, int par,
                                                                 uint32_t k0, uint32_t k1, uint32_t sweep,
                                                                 const uint32_t *d_sweep)
{
    __shared__ HbShared sh;
    const uint32_t sw = d_sweep ? *d_sweep : sweep;
    const BatchEntry &e = find_entry<&BatchEntry::block0>(tab, count, blockIdx.x);
    heatbath_item<T, MU>(e, par, k0, k1, sw, blockIdx.x - e.block0, sh);
}

// An overrelaxation class of the batch's lattices without launches of
// their own (those take the single-lattice kernel with its residency cap).
template <class T, int MU>
__global__ __launch_bounds__(kBlock) void overrelax_batch_kernel(const BatchEntry *tab, int count, int par)
{
    const BatchEntry &e = find_entry<&BatchEntry::sub_block0>(tab, count, blockIdx.x);
    overrelax_item<T, MU>(e, par, blockIdx.x - e.sub_block0);
}

// ---------------------------------------------------------------------------
// Persistent batched sweep: one launch runs the eight heat-bath classes and
// then n_or overrelaxation sweeps (8 classes each) of every lattice of a
// batch.  The grid holds at most the blocks the device keeps resident at
// once, a multiple of 8; block b takes the items b, b + G, b + 2G, ... of a
// class, an item being one block of the batched class launch (the same
// lattice, walk position and arithmetic, so the same links bit for bit).
// As G is a multiple of 8, block b (dispatched to XCD b mod 8) only takes
// items of that XCD's range of each lattice's walk.  Classes are separated
// by a grid-wide barrier.
//
// The barrier counts arrivals in one word: every block adds 1 except block
// 0, which adds 2^31 - (G - 1), so the G arrivals of a barrier sum to 2^31:
// bit 31 flips exactly when the last block arrives and bits 0-30 return to
// 0.  A block waits until bit 31 differs from the value its own addition
// returned (no barrier can complete again before every block has arrived
// there, so a late reader cannot miss a flip).  The addition is a release
// and the wait ends with an acquire, both at device scope, after a block
// barrier: every store of every block before the barrier is visible to
// every load after it, across XCDs.  The wait is bounded: after spin_limit
// polls the block sets kFlagSync in every lattice's flags and goes on, so
// every block still ends (the links are then unreliable); each block still
// adds once per barrier, so bits 0-30 of the word end the launch at 0
// either way (bit 31, the phase, flips once per barrier).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void grid_barrier(uint32_t *word, uint32_t spin_limit, const BatchEntry *tab, int count)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t inc = barrier_increment(blockIdx.x, gridDim.x);
        const uint32_t old = __hip_atomic_fetch_add(word, inc, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t polls = 0;
        bool flipped = false;
        while (!(flipped = barrier_passed(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), old)) &&
               ++polls < spin_limit)
            __builtin_amdgcn_s_sleep(4);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!flipped)
            for (int j = 0; j < count; ++j)
                atomicOr(tab[j].flags, kFlagSync);
    }
    __syncthreads();
}

// The items b, b + G, ... of one class of the persistent sweep.
template <class T, int MU, bool HB>
__device__ __forceinline__ void batch_class_items(const BatchEntry *tab, int count, uint32_t total, int par,
                                                  uint32_t k0, uint32_t k1, uint32_t sw, HbShared &sh)
{
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        const BatchEntry &e = find_entry<&BatchEntry::block0>(tab, count, item);
        if constexpr (HB)
            heatbath_item<T, MU>(e, par, k0, k1, sw, item - e.block0, sh);
        else
            overrelax_item<T, MU>(e, par, item - e.block0);
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void batch_sweep_kernel(const BatchEntry *tab, int count, uint32_t total,
                                                             uint32_t k0, uint32_t k1, uint32_t sweep,
                                                             const uint32_t *d_sweep, int n_or, uint32_t *sync,
                                                             uint32_t spin_limit)
{
    __shared__ HbShared sh;
    const uint32_t sw = d_sweep ? *d_sweep : sweep;
    const int classes = 8 * (1 + n_or);
    for (int c = 0; c < classes; ++c) {
        const int mu = (c & 7) >> 1, par = c & 1;
        switch ((c < 8 ? 0 : 4) + mu) {
        case 0: batch_class_items<T, 0, true>(tab, count, total, par, k0, k1, sw, sh); break;
        case 1: batch_class_items<T, 1, true>(tab, count, total, par, k0, k1, sw, sh); break;
        case 2: batch_class_items<T, 2, true>(tab, count, total, par, k0, k1, sw, sh); break;
        case 3: batch_class_items<T, 3, true>(tab, count, total, par, k0, k1, sw, sh); break;
        case 4: batch_class_items<T, 0, false>(tab, count, total, par, k0, k1, sw, sh); break;
        case 5: batch_class_items<T, 1, false>(tab, count, total, par, k0, k1, sw, sh); break;
        case 6: batch_class_items<T, 2, false>(tab, count, total, par, k0, k1, sw, sh); break;
        default: batch_class_items<T, 3, false>(tab, count, total, par, k0, k1, sw, sh); break;
        }
        if (c + 1 < classes)
            grid_barrier(sync, spin_limit, tab, count);
    }
}

__global__ void sweep_advance_kernel(uint32_t *d_sweep)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *d_sweep += 1u;
}

// ---------------------------------------------------------------------------
// Starts.  Hot: four Box-Muller normals from two Philox calls (counter
// (site, mu + 16*lattice_id, 0, 0/1)), normalised; always computed in FP64.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void init_kernel(Links<T> U, Geom g, int hot, uint32_t k0, uint32_t k1,
                                                       uint32_t lid16, uint32_t *flags)
{
    const uint32_t cb = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *flags = 0u;
    if (cb >= g.half)
        return;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        const Site s = site_of_cb(g, cb, par);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            Quat<double> q = {1.0, 0.0, 0.0, 0.0};
            if (hot) {
                const uint32_t c1 = (uint32_t)mu + lid16;
                double u1, u2, u3, u4;
                Draw<double>::two(philox(s.site, c1, 0u, 0u, k0, k1), u1, u2);
                Draw<double>::two(philox(s.site, c1, 0u, 1u, k0, k1), u3, u4);
                const double ra = sqrt(-2.0 * log(u1));
                const double rb = sqrt(-2.0 * log(u3));
                double sa, ca, sb, cbv;
                sincos((2.0 * kPi) * u2, &sa, &ca);
                sincos((2.0 * kPi) * u4, &sb, &cbv);
                const double g0 = ra * ca, g1 = ra * sa, g2 = rb * cbv, g3 = rb * sb;
                const double nrm = sqrt(g0 * g0 + g1 * g1 + g2 * g2 + g3 * g3);
                q = {g0 / nrm, g1 / nrm, g2 / nrm, g3 / nrm};
            }
            U.st(mu, par, cb, unitize(Quat<T>{(T)q.w, (T)q.x, (T)q.y, (T)q.z}));
        }
    }
}

__global__ void copy_flags_kernel(const uint32_t *flags, uint32_t *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dst = *flags;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <class T>
static Links<T> links_of(const LaunchArgs &a)
{
    Links<T> L;
    L.p = reinterpret_cast<decltype(L.p)>(a.links);
    L.stride = plane_stride((uint32_t)(a.volume / 2), sizeof(T) == 8);
    return L;
}

static uint32_t blocks_for(uint64_t n)
{
    return (uint32_t)((n + kBlock - 1) / kBlock);
}

uint32_t class_blocks(const LaunchArgs &a)
{
    return blocks_for(a.volume / 2);
}

uint64_t batch_entry_bytes()
{
    return sizeof(BatchEntry);
}

void fill_batch_entry(const LaunchArgs &a, const WorkLayout &w, double beta, const BatchOffsets &o, void *dst)
{
    BatchEntry e = {};
    e.g = make_geom(a.n, a.tile, a.tile_y);
    e.links = a.links;
    e.flags = a.flags;
    e.beta = beta;
    e.lid16 = 16u * (uint32_t)a.lattice_id;
    e.col = col_addressing_ok(e.g) ? 1u : 0u;
    e.block0 = o.block0;
    e.nblocks = o.nblocks;
    e.sub_block0 = o.sub_block0;
    e.lfield = reinterpret_cast<double *>(a.work + w.off_lfield);
    e.poly_part = reinterpret_cast<double *>(a.work + w.off_poly);
    e.corr_part = reinterpret_cast<double *>(a.work + w.off_corr);
    e.pblock0 = o.pblock0;
    e.pnblk = w.nblk_poly;
    e.cblock0 = o.cblock0;
    e.cnblk = w.nblk_corr;
    e.rmax = (uint32_t)w.rmax;
    e.ocol0 = o.ocol0;
    std::memcpy(dst, &e, sizeof e);
}

template <class T, bool COL, bool PLAQ>
static void launch_hb_mode(const Links<T> &U, const Geom &g, int mu, int par, double beta, uint32_t k0,
                           uint32_t k1, uint32_t c1, uint32_t sweep, const uint32_t *d_sweep, uint32_t *flags,
                           double *pp, hipStream_t st)
{
    const dim3 grid(blocks_for(g.half)), block(kBlock);
    switch (mu) {
    case 0: heatbath_kernel<T, 0, COL, false><<<grid, block, 0, st>>>(U, g, par, beta, k0, k1, c1, sweep, d_sweep, flags, pp); break;
    case 1: heatbath_kernel<T, 1, COL, PLAQ><<<grid, block, 0, st>>>(U, g, par, beta, k0, k1, c1, sweep, d_sweep, flags, pp); break;
    case 2: heatbath_kernel<T, 2, COL, PLAQ><<<grid, block, 0, st>>>(U, g, par, beta, k0, k1, c1, sweep, d_sweep, flags, pp); break;
    default: heatbath_kernel<T, 3, COL, PLAQ><<<grid, block, 0, st>>>(U, g, par, beta, k0, k1, c1, sweep, d_sweep, flags, pp); break;
    }
}

// plaq_partials != nullptr (class (mu >= 1, odd) of a lattice's last sweep):
// the class also writes its planes' plaquette partials.
template <class T>
static void launch_hb(const LaunchArgs &a, const Geom &g, int mu, int par, double beta, uint64_t seed,
                      uint32_t sweep, const uint32_t *d_sweep, double *plaq_partials, hipStream_t st)
{
    const Links<T> U = links_of<T>(a);
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const uint32_t c1 = (uint32_t)mu + 4u * 1u + 16u * (uint32_t)a.lattice_id;
    const bool col = col_addressing_ok(g), plaq = plaq_partials != nullptr;
    if (col && plaq)
        launch_hb_mode<T, true, true>(U, g, mu, par, beta, k0, k1, c1, sweep, d_sweep, a.flags, plaq_partials, st);
    else if (col)
        launch_hb_mode<T, true, false>(U, g, mu, par, beta, k0, k1, c1, sweep, d_sweep, a.flags, nullptr, st);
    else if (plaq)
        launch_hb_mode<T, false, true>(U, g, mu, par, beta, k0, k1, c1, sweep, d_sweep, a.flags, plaq_partials, st);
    else
        launch_hb_mode<T, false, false>(U, g, mu, par, beta, k0, k1, c1, sweep, d_sweep, a.flags, nullptr, st);
}

// Whether the capped overrelaxation kernel runs exactly kOrBlocksPerCu
// blocks per CU on the current device (occupancy query, once per device).
template <class T>
static bool or_cap_holds()
{
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static int cached[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return false;
    std::lock_guard<std::mutex> hold(lock);
    if (cached[dev] == 0) {
        int blocks = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &blocks, overrelax_kernel<T, 0, true, true, false>, kBlock, 0);
        cached[dev] = (e == hipSuccess && blocks == kOrBlocksPerCu) ? 1 : -1;
    }
    return cached[dev] > 0;
}

template <class T, bool COL, bool CAP, bool PLAQ>
static void launch_or_mode(const Links<T> &U, const Geom &g, int mu, int par, uint32_t *flags, double *pp,
                           hipStream_t st)
{
    const dim3 grid(blocks_for(g.half)), block(kBlock);
    switch (mu) {
    case 0: overrelax_kernel<T, 0, COL, CAP, false><<<grid, block, 0, st>>>(U, g, par, flags, pp); break;
    case 1: overrelax_kernel<T, 1, COL, CAP, PLAQ><<<grid, block, 0, st>>>(U, g, par, flags, pp); break;
    case 2: overrelax_kernel<T, 2, COL, CAP, PLAQ><<<grid, block, 0, st>>>(U, g, par, flags, pp); break;
    default: overrelax_kernel<T, 3, COL, CAP, PLAQ><<<grid, block, 0, st>>>(U, g, par, flags, pp); break;
    }
}

template <class T, bool COL, bool CAP>
static void launch_or_cap(const Links<T> &U, const Geom &g, int mu, int par, uint32_t *flags, double *pp,
                          hipStream_t st)
{
    if (pp)
        launch_or_mode<T, COL, CAP, true>(U, g, mu, par, flags, pp, st);
    else
        launch_or_mode<T, COL, CAP, false>(U, g, mu, par, flags, nullptr, st);
}

template <class T>
static void launch_or(const LaunchArgs &a, const Geom &g, int mu, int par, double *plaq_partials, hipStream_t st)
{
    const Links<T> U = links_of<T>(a);
    const bool cap = residency_cap_pays(g) && or_cap_holds<T>();
    if (col_addressing_ok(g)) {
        if (cap)
            launch_or_cap<T, true, true>(U, g, mu, par, a.flags, plaq_partials, st);
        else
            launch_or_cap<T, true, false>(U, g, mu, par, a.flags, plaq_partials, st);
    } else {
        if (cap)
            launch_or_cap<T, false, true>(U, g, mu, par, a.flags, plaq_partials, st);
        else
            launch_or_cap<T, false, false>(U, g, mu, par, a.flags, plaq_partials, st);
    }
}

void launch_init(const LaunchArgs &a, int hot, uint64_t seed, hipStream_t st)
{
    const Geom g = make_geom(a.n, a.tile, a.tile_y);
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const uint32_t lid16 = 16u * (uint32_t)a.lattice_id;
    const dim3 grid(blocks_for(g.half)), block(kBlock);
    if (a.prec == kF32)
        init_kernel<float><<<grid, block, 0, st>>>(links_of<float>(a), g, hot, k0, k1, lid16, a.flags);
    else
        init_kernel<double><<<grid, block, 0, st>>>(links_of<double>(a), g, hot, k0, k1, lid16, a.flags);
}

void launch_heatbath(const LaunchArgs &a, double beta, uint64_t seed, uint32_t sweep, const uint32_t *d_sweep,
                     int mu, int par, double *plaq_partials, hipStream_t st)
{
    // the staged kernel takes no plaquette; a class it cannot plan runs here
    if (a.tile == kTileStagedBoth && !plaq_partials &&
        launch_heatbath_staged(a, beta, seed, sweep, d_sweep, mu, par, st))
        return;
    const Geom g = make_geom(a.n, a.tile, a.tile_y);
    if (a.prec == kF32)
        launch_hb<float>(a, g, mu, par, beta, seed, sweep, d_sweep, plaq_partials, st);
    else
        launch_hb<double>(a, g, mu, par, beta, seed, sweep, d_sweep, plaq_partials, st);
}

void launch_overrelax(const LaunchArgs &a, int mu, int par, double *plaq_partials, hipStream_t st)
{
    // the staged kernel takes no plaquette; a class it cannot plan runs here
    if ((a.tile == kTileStaged || a.tile == kTileStagedBoth) && !plaq_partials &&
        launch_overrelax_staged(a, mu, par, st))
        return;
    const Geom g = make_geom(a.n, a.tile, a.tile_y);
    if (a.prec == kF32)
        launch_or<float>(a, g, mu, par, plaq_partials, st);
    else
        launch_or<double>(a, g, mu, par, plaq_partials, st);
}

template <class T>
static void launch_hb_batch(const BatchEntry *tab, int count, uint32_t total, int mu, int par, uint64_t seed,
                            uint32_t sweep, const uint32_t *d_sweep, hipStream_t st)
{
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const dim3 grid(total), block(kBlock);
    switch (mu) {
    case 0: heatbath_batch_kernel<T, 0><<<grid, block, 0, st>>>(tab, count, par, k0, k1, sweep, d_sweep); break;
    case 1: heatbath_batch_kernel<T, 1><<<grid, block, 0, st>>>(tab, count, par, k0, k1, sweep, d_sweep); break;
    case 2: heatbath_batch_kernel<T, 2><<<grid, block, 0, st>>>(tab, count, par, k0, k1, sweep, d_sweep); break;
    default: heatbath_batch_kernel<T, 3><<<grid, block, 0, st>>>(tab, count, par, k0, k1, sweep, d_sweep); break;
    }
}

template <class T>
static void launch_or_batch(const BatchEntry *tab, int count, uint32_t total, int mu, int par, hipStream_t st)
{
    const dim3 grid(total), block(kBlock);
    switch (mu) {
    case 0: overrelax_batch_kernel<T, 0><<<grid, block, 0, st>>>(tab, count, par); break;
    case 1: overrelax_batch_kernel<T, 1><<<grid, block, 0, st>>>(tab, count, par); break;
    case 2: overrelax_batch_kernel<T, 2><<<grid, block, 0, st>>>(tab, count, par); break;
    default: overrelax_batch_kernel<T, 3><<<grid, block, 0, st>>>(tab, count, par); break;
    }
}

void launch_heatbath_batch(const void *d_table, int count, int prec, uint32_t total_blocks, int mu, int par,
                           uint64_t seed, uint32_t sweep, const uint32_t *d_sweep, hipStream_t st)
{
    const BatchEntry *tab = static_cast<const BatchEntry *>(d_table);
    if (prec == kF32)
        launch_hb_batch<float>(tab, count, total_blocks, mu, par, seed, sweep, d_sweep, st);
    else
        launch_hb_batch<double>(tab, count, total_blocks, mu, par, seed, sweep, d_sweep, st);
}

void launch_overrelax_batch(const void *d_table, int count, int prec, uint32_t total_blocks, int mu, int par,
                            hipStream_t st)
{
    const BatchEntry *tab = static_cast<const BatchEntry *>(d_table);
    if (prec == kF32)
        launch_or_batch<float>(tab, count, total_blocks, mu, par, st);
    else
        launch_or_batch<double>(tab, count, total_blocks, mu, par, st);
}

// Blocks of batch_sweep_kernel<T> the current device holds at once (the
// occupancy query times the CU count, once per device), rounded down to a
// multiple of 8; 0 if it cannot be resident.
template <class T>
static uint32_t batch_sweep_resident()
{
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static int64_t cached[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return 0;
    std::lock_guard<std::mutex> hold(lock);
    if (cached[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_sweep_kernel<T>, kBlock, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            per_cu = cus = 0;
        const int64_t n = ((int64_t)per_cu * cus) & ~int64_t(7);
        cached[dev] = n > 0 ? n : -1;
    }
    return cached[dev] > 0 ? (uint32_t)cached[dev] : 0u;
}

template <class T>
static bool launch_batch_sweep_t(const BatchEntry *tab, int count, uint32_t total, uint64_t seed, uint32_t sweep,
                                 const uint32_t *d_sweep, int n_or, uint32_t *d_sync, uint32_t spin_limit,
                                 hipStream_t st)
{
    const uint32_t resident = batch_sweep_resident<T>();
    if (resident == 0)
        return false;
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const uint32_t grid = total < resident ? total : resident; // both multiples of 8
    batch_sweep_kernel<T><<<dim3(grid), dim3(kBlock), 0, st>>>(tab, count, total, k0, k1, sweep, d_sweep, n_or,
                                                               d_sync, spin_limit);
    return true;
}

bool launch_batch_sweep(const void *d_table, int count, int prec, uint32_t total_blocks, uint64_t seed,
                        uint32_t sweep, const uint32_t *d_sweep, int n_or, uint32_t *d_sync, uint32_t spin_limit,
                        hipStream_t st)
{
    const BatchEntry *tab = static_cast<const BatchEntry *>(d_table);
    if (prec == kF32)
        return launch_batch_sweep_t<float>(tab, count, total_blocks, seed, sweep, d_sweep, n_or, d_sync, spin_limit,
                                           st);
    return launch_batch_sweep_t<double>(tab, count, total_blocks, seed, sweep, d_sweep, n_or, d_sync, spin_limit,
                                        st);
}

void launch_sweep_advance(uint32_t *d_sweep, hipStream_t st)
{
    sweep_advance_kernel<<<1, 64, 0, st>>>(d_sweep);
}

void launch_get_flags(const LaunchArgs &a, uint32_t *d_flags, hipStream_t st)
{
    copy_flags_kernel<<<1, 64, 0, st>>>(a.flags, d_flags);
}

} // namespace su2

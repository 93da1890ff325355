// su2_observables.hip -- gfx950 kernels of the measured observables: the
// mean plaquette (per plane), the Polyakov loop and its on-axis correlator.
// All sums are FP64 and deterministic: fixed-order wave64 sums, an LDS
// tree, one partial per block (stored column by column) and a fixed-order
// final pass.
#include "su2_device.hpp"
#include "su2_launch.hpp"

#include <mutex>

namespace su2 {

template <class T>
static Links<T> links_of(const LaunchArgs &a)
{
    Links<T> L;
    L.p = reinterpret_cast<decltype(L.p)>(a.links);
    L.stride = plane_stride((uint32_t)(a.volume / 2), sizeof(T) == 8);
    return L;
}

// Plaquettes: every site x sums (1/2) Tr of its six plaquettes
// U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+, mu < nu, in FP64.  A thread
// takes one cb index and both parities; blocks walk the lattice in the
// same order as the update kernels; one partial per block.
template <class T, class A>
__device__ __forceinline__ void plaquette_site(const Links<T> &U, const A &ad, int par, double (&acc)[6])
{
    const int opp = par ^ 1;
    const uint32_t own = ad.at(0, 0, 0, 0);
    Quat<T> u[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
        u[mu] = ad.ld(U, mu, par, own);
    const uint32_t ip[4] = {ad.at(1, 0, 0, 0), ad.at(0, 1, 0, 0), ad.at(0, 0, 1, 0), ad.at(0, 0, 0, 1)};
    int p = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int nu = mu + 1; nu < 4; ++nu) {
            const Quat<T> a = qmul(u[mu], ad.ld(U, nu, opp, ip[mu]));
            const Quat<T> b = qmul(u[nu], ad.ld(U, mu, opp, ip[nu]));
            acc[p++] += (double)qdot(a, b);
        }
}

template <class T, bool COL>
__global__ __launch_bounds__(kBlock) void plaquette_kernel(Links<T> U, Geom g, double *partials)
{
    __shared__ double lds[kBlock / 64][6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const uint32_t i = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < g.half) {
        if constexpr (COL) {
#pragma unroll
            for (int par = 0; par < 2; ++par)
                plaquette_site(U, col_addr(g, i, par), par, acc);
        } else {
            CbAddr ad;
            ad.cb = walk_cb(i, g.ord);
            ad.g = &g;
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                ad.s = site_of_cb(g, ad.cb, par);
                plaquette_site(U, ad, par, acc);
            }
        }
    }
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 6; ++j)
            partials[(size_t)j * gridDim.x + blockIdx.x] = acc[j];
}

// Plaquettes and Polyakov loop in one pass: a thread takes one spatial site
// and walks t = 0..Nt-1.  At each t it loads the site's four links and the
// nine links at x+e_x, x+e_y, x+e_z that the spatial plaquettes (01, 02, 12)
// and the temporal ones need; the temporal plaquettes (mu, 3) of slice t-1
// take U_mu(x + e_t) from the links just loaded for slice t (slice 0's links
// close the last slice), and the Polyakov line multiplies U_3(x,t) in t
// order.  13 loads per site instead of 16, every link read once as its own.
// Partials per block, column by column: the six planes, sum L, sum |L|.
template <class T>
__global__ __launch_bounds__(kBlock) void measure_kernel(Links<T> U, Geom g, double *Lfield, double *partials)
{
    __shared__ double lds[kBlock / 64][8];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint32_t sp = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (sp < g.vs) {
        const uint32_t nx = (uint32_t)g.n[0], ny = (uint32_t)g.n[1], nz = (uint32_t)g.n[2];
        const uint32_t yz = fdiv(sp, g.div_nx);
        const uint32_t x = sp - yz * nx;
        const uint32_t z = fdiv(yz, g.div_ny);
        const uint32_t y = yz - z * ny;
        // spatial site indices of the three forward neighbours
        const uint32_t sx = (x + 1u == nx ? 0u : x + 1u) + nx * yz;
        const uint32_t sy = x + nx * ((y + 1u == ny ? 0u : y + 1u) + ny * z);
        const uint32_t sz = x + nx * (y + ny * (z + 1u == nz ? 0u : z + 1u));
        const uint32_t par0 = (x + y + z) & 1u;
        Quat<T> first[3], prev[4], prev3[3];
        Quat<T> P = {1, 0, 0, 0};
        for (uint32_t t = 0; t < (uint32_t)g.n[3]; ++t) {
            const uint32_t base = g.vs * t;
            const int par = (int)((par0 + t) & 1u), opp = par ^ 1;
            const uint32_t cb = (base + sp) >> 1, cbx = (base + sx) >> 1, cby = (base + sy) >> 1,
                           cbz = (base + sz) >> 1;
            Quat<T> u[4];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                u[mu] = U.ld(mu, par, cb);
            const Quat<T> x1 = U.ld(1, opp, cbx), x2 = U.ld(2, opp, cbx), x3 = U.ld(3, opp, cbx);
            const Quat<T> y0 = U.ld(0, opp, cby), y2 = U.ld(2, opp, cby), y3 = U.ld(3, opp, cby);
            const Quat<T> z0 = U.ld(0, opp, cbz), z1 = U.ld(1, opp, cbz), z3 = U.ld(3, opp, cbz);
            acc[0] += (double)qdot(qmul(u[0], x1), qmul(u[1], y0)); // 01
            acc[1] += (double)qdot(qmul(u[0], x2), qmul(u[2], z0)); // 02
            acc[3] += (double)qdot(qmul(u[1], y2), qmul(u[2], z1)); // 12
            if (t == 0) {
#pragma unroll
                for (int mu = 0; mu < 3; ++mu)
                    first[mu] = u[mu];
            } else {
                acc[2] += (double)qdot(qmul(prev[0], prev3[0]), qmul(prev[3], u[0])); // 03 at t-1
                acc[4] += (double)qdot(qmul(prev[1], prev3[1]), qmul(prev[3], u[1])); // 13
                acc[5] += (double)qdot(qmul(prev[2], prev3[2]), qmul(prev[3], u[2])); // 23
            }
            P = qmul(P, u[3]);
#pragma unroll
            for (int mu = 0; mu < 4; ++mu)
                prev[mu] = u[mu];
            prev3[0] = x3;
            prev3[1] = y3;
            prev3[2] = z3;
        }
        acc[2] += (double)qdot(qmul(prev[0], prev3[0]), qmul(prev[3], first[0]));
        acc[4] += (double)qdot(qmul(prev[1], prev3[1]), qmul(prev[3], first[1]));
        acc[5] += (double)qdot(qmul(prev[2], prev3[2]), qmul(prev[3], first[2]));
        const double L = (double)P.w;
        Lfield[sp] = L;
        acc[6] = L;
        acc[7] = fabs(L);
    }
    block_sum<8>(acc, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            partials[(size_t)j * gridDim.x + blockIdx.x] = acc[j];
}

// Polyakov loop at each spatial site: ordered product of the Nt temporal
// links.  Block b of nb (grid-stride over the spatial sites) writes its
// partial sums of L and |L| to partials[b] and partials[nb + b].
template <class T>
__device__ __forceinline__ void polyakov_body(const Links<T> &U, const Geom &g, double *Lfield, double *partials,
                                              uint32_t b, uint32_t nb)
{
    __shared__ double lds[kBlock / 64][2];
    double acc[2] = {0, 0};
    for (uint32_t sp = b * kBlock + threadIdx.x; sp < g.vs; sp += nb * kBlock) {
        const uint32_t yz = fdiv(sp, g.div_nx);
        const uint32_t x = sp - yz * (uint32_t)g.n[0];
        const uint32_t z = fdiv(yz, g.div_ny);
        const uint32_t y = yz - z * (uint32_t)g.n[1];
        Quat<T> P = {1, 0, 0, 0};
        for (int t = 0; t < g.n[3]; ++t) {
            const uint32_t site = sp + g.vs * (uint32_t)t;
            const int par = (int)((x + y + z + (uint32_t)t) & 1u);
            P = qmul(P, U.ld(3, par, site >> 1));
        }
        const double L = (double)P.w;
        Lfield[sp] = L;
        acc[0] += L;
        acc[1] += fabs(L);
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        partials[b] = acc[0];
        partials[(size_t)nb + b] = acc[1];
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void polyakov_kernel(Links<T> U, Geom g, double *Lfield, double *partials)
{
    polyakov_body<T>(U, g, Lfield, partials, blockIdx.x, gridDim.x);
}

// On-axis Polyakov correlator: for the separations r0 .. r0+kCorrGroup-1
// that do not exceed rmax, sum_x L(x)(L(x+r e_x) + L(x+r e_y) + L(x+r e_z));
// block b of nb writes its partial for r to partials[(r-1) nb + b]
// (column r-1).  Each site's L(x) is loaded once for the whole group.
__device__ __forceinline__ void polycorr_body(const double *Lfield, const Geom &g, double *partials, uint32_t r0,
                                              uint32_t rmax, uint32_t b, uint32_t nb)
{
    __shared__ double lds[kBlock / 64][kCorrGroup];
    const uint32_t nx = (uint32_t)g.n[0], ny = (uint32_t)g.n[1], nz = (uint32_t)g.n[2];
    const uint32_t nr = rmax - r0 + 1u < kCorrGroup ? rmax - r0 + 1u : kCorrGroup;
    double acc[kCorrGroup];
#pragma unroll
    for (uint32_t j = 0; j < kCorrGroup; ++j)
        acc[j] = 0.0;
    for (uint32_t sp = b * kBlock + threadIdx.x; sp < g.vs; sp += nb * kBlock) {
        const uint32_t yz = fdiv(sp, g.div_nx);
        const uint32_t x = sp - yz * nx;
        const uint32_t z = fdiv(yz, g.div_ny);
        const uint32_t y = yz - z * ny;
        const double L = Lfield[sp];
#pragma unroll
        for (uint32_t j = 0; j < kCorrGroup; ++j) {
            if (j < nr) {
                const uint32_t r = r0 + j; // r <= min(Nx,Ny,Nz)/2: one wrap at most
                const uint32_t xr = x + r, yr = y + r, zr = z + r;
                const uint32_t xs = xr >= nx ? xr - nx : xr;
                const uint32_t ys = yr >= ny ? yr - ny : yr;
                const uint32_t zs = zr >= nz ? zr - nz : zr;
                acc[j] += L * (Lfield[xs + nx * (y + ny * z)] + Lfield[x + nx * (ys + ny * z)] +
                               Lfield[x + nx * (y + ny * zs)]);
            }
        }
    }
    block_sum<kCorrGroup>(acc, lds);
    if (threadIdx.x == 0)
        for (uint32_t j = 0; j < nr; ++j)
            partials[(size_t)(r0 + j - 1u) * nb + b] = acc[j];
}

// Separation group blockIdx.y: r0 = kCorrGroup * blockIdx.y + 1.
__global__ __launch_bounds__(kBlock) void polycorr_kernel(const double *Lfield, Geom g, double *partials,
                                                           uint32_t rmax)
{
    polycorr_body(Lfield, g, partials, kCorrGroup * blockIdx.y + 1u, rmax, blockIdx.x, gridDim.x);
}

// *out = scale * sum_b col[b], b < nblk, in a fixed order (one block).
__device__ __forceinline__ void colsum_body(const double *col, uint32_t nblk, double scale, double *out)
{
    __shared__ double lds[kBlock / 64][1];
    double acc[1] = {0.0};
    // Eight loads are issued before their (in-order) sums; one load per
    // iteration made the loop a chain of dependent global-memory latencies.
    uint32_t b = threadIdx.x;
    for (; b + 7u * kBlock < nblk; b += 8u * kBlock) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = col[b + (uint32_t)u * kBlock];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            acc[0] += v[u];
    }
    for (; b < nblk; b += kBlock)
        acc[0] += col[b];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0)
        *out = acc[0] * scale;
}

// out[c] = scale * sum_b partials[c*nblk + b] (partials stored column by
// column, so the reads are contiguous), one block per column c.
__global__ __launch_bounds__(kBlock) void colsum_kernel(const double *partials, uint32_t nblk, double scale,
                                                         double *out)
{
    colsum_body(partials + (size_t)blockIdx.x * nblk, nblk, scale, out + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Polyakov loop and correlator of every lattice of a batch, three launches
// in all.  Each lattice keeps the block counts, partial layout and summation
// order of its single-lattice launches, so its results are bitwise those of
// su2_polyakov; a block finds its lattice from the table's ranges.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void polyakov_batch_kernel(const BatchEntry *tab, int count)
{
    const BatchEntry &e = tab[find_entry_index<&BatchEntry::pblock0>(tab, count, blockIdx.x)];
    Links<T> U;
    U.p = reinterpret_cast<decltype(U.p)>(e.links);
    U.stride = plane_stride(e.g.half, sizeof(T) == 8);
    polyakov_body<T>(U, e.g, e.lfield, e.poly_part, blockIdx.x - e.pblock0, e.pnblk);
}

// A lattice's corr_groups(rmax) * cnblk blocks: separation group local / cnblk.
__global__ __launch_bounds__(kBlock) void polycorr_batch_kernel(const BatchEntry *tab, int count)
{
    const BatchEntry &e = tab[find_entry_index<&BatchEntry::cblock0>(tab, count, blockIdx.x)];
    const uint32_t local = blockIdx.x - e.cblock0;
    const uint32_t grp = local / e.cnblk;
    polycorr_body(e.lfield, e.g, e.corr_part, kCorrGroup * grp + 1u, e.rmax, local - grp * e.cnblk, e.cnblk);
}

// One block per output: lattice j's columns 0, 1 (mean L, mean |L|) go to
// d_poly[2j], d_poly[2j+1]; with the correlator, its columns 2 + (r-1) go to
// d_corr[j * corr_stride + r - 1].
__global__ __launch_bounds__(kBlock) void polysum_batch_kernel(const BatchEntry *tab, int count, double *d_poly,
                                                                double *d_corr, uint32_t corr_stride)
{
    int j;
    uint32_t c;
    if (d_corr) {
        j = find_entry_index<&BatchEntry::ocol0>(tab, count, blockIdx.x);
        c = blockIdx.x - tab[j].ocol0;
    } else {
        j = (int)(blockIdx.x >> 1);
        c = blockIdx.x & 1u;
    }
    const BatchEntry &e = tab[j];
    if (c < 2u)
        colsum_body(e.poly_part + (size_t)c * e.pnblk, e.pnblk, 1.0 / (double)e.g.vs, d_poly + 2 * j + c);
    else
        colsum_body(e.corr_part + (size_t)(c - 2u) * e.cnblk, e.cnblk, 1.0 / (3.0 * (double)e.g.vs),
                    d_corr + (size_t)j * corr_stride + (c - 2u));
}

// d_out[0] = mean of the six plane averages d_out[1..6].
__global__ void plaq_total_kernel(double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        out[0] = (out[1] + out[2] + out[3] + out[4] + out[5] + out[6]) / 6.0;
}

// colsum_kernel over the six planes and plaq_total_kernel in one block: each
// thread adds its partials of a plane in the same order as colsum_body, the
// block sum and the final mean are the same expressions, so the results are
// bitwise those of the two launches.  Used for short columns, where the
// second launch costs more than one block reading all six.
__global__ __launch_bounds__(kBlock) void plaq_finish_kernel(const double *partials, uint32_t nblk, double scale,
                                                             double *out)
{
    __shared__ double lds[kBlock / 64][6];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    uint32_t b = threadIdx.x;
    for (; b + 7u * kBlock < nblk; b += 8u * kBlock) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double *col = partials + (size_t)j * nblk;
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = col[b + (uint32_t)u * kBlock];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                acc[j] += v[u];
        }
    }
    for (; b < nblk; b += kBlock)
#pragma unroll
        for (int j = 0; j < 6; ++j)
            acc[j] += partials[(size_t)j * nblk + b];
    block_sum<6>(acc, lds);
    if (threadIdx.x == 0) {
        // the two-launch path rounds each scaled plane before the mean
#pragma clang fp contract(off)
        double p[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            p[j] = acc[j] * scale;
            out[1 + j] = p[j];
        }
        out[0] = (p[0] + p[1] + p[2] + p[3] + p[4] + p[5]) / 6.0;
    }
}

// Columns up to this many partials are finished by plaq_finish_kernel.
constexpr uint32_t kFinishOneBlock = 2048;

static void launch_plaquette_finish(const double *partials, uint32_t nblk, double scale, double *d_out,
                                    hipStream_t st)
{
    if (nblk <= kFinishOneBlock) {
        plaq_finish_kernel<<<1, kBlock, 0, st>>>(partials, nblk, scale, d_out);
    } else {
        colsum_kernel<<<6, kBlock, 0, st>>>(partials, nblk, scale, d_out + 1);
        plaq_total_kernel<<<1, 64, 0, st>>>(d_out);
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
// The plane partials a measured sweep left in the plaquette region (one per
// block of the class grid and plane) summed into d_out[0..6].
void launch_plaquette_sum(const LaunchArgs &a, const WorkLayout &w, double *d_out, hipStream_t st)
{
    double *partials = reinterpret_cast<double *>(a.work + w.off_plaq);
    launch_plaquette_finish(partials, w.nblk_plaq, 1.0 / (double)a.volume, d_out, st);
}

// The plaquette pass with its block partials (6 planes x nblk) in `partials`.
static void launch_plaquette_into(const LaunchArgs &a, uint32_t nblk, double *partials, double *d_out,
                                  hipStream_t st)
{
    // The lattice's strip width, but whole columns: with row ranges the
    // plaquette kernel (two sites per thread) fetched 1.5x more.
    const Geom g = make_geom(a.n, a.tile, 1);
    const bool col = col_addressing_ok(g);
    if (a.prec == kF32) {
        if (col)
            plaquette_kernel<float, true><<<nblk, kBlock, 0, st>>>(links_of<float>(a), g, partials);
        else
            plaquette_kernel<float, false><<<nblk, kBlock, 0, st>>>(links_of<float>(a), g, partials);
    } else {
        if (col)
            plaquette_kernel<double, true><<<nblk, kBlock, 0, st>>>(links_of<double>(a), g, partials);
        else
            plaquette_kernel<double, false><<<nblk, kBlock, 0, st>>>(links_of<double>(a), g, partials);
    }
    launch_plaquette_finish(partials, nblk, 1.0 / (double)a.volume, d_out, st);
}

void launch_plaquette(const LaunchArgs &a, const WorkLayout &w, double *d_out, hipStream_t st)
{
    launch_plaquette_into(a, w.nblk_plaq, reinterpret_cast<double *>(a.work + w.off_plaq), d_out, st);
}

// ---------------------------------------------------------------------------
// The plaquette without a caller's workspace: the block partials go to a
// file-scope device array instead.  Each GPU holds its own copy of the array
// (8 MiB, for as long as the process lives); its address on a device comes
// from hipGetSymbolAddress, once per device, and is the only form in which
// host code hands the array to a kernel.  Every call on one GPU overwrites
// the same array (each block writes its own partials before the finishing
// kernel reads them, so nothing needs clearing between calls), hence calls
// that overlap in time on one GPU race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[6u * kNoAllocPlaqBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
double *g_scratch_addr[kMaxDevices] = {};
} // namespace

// Address of the scratch array on the current device (looked up on the
// first call per device).  Returns hipSuccess or the HIP error.
static hipError_t scratch_on_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> hold(g_scratch_lock);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

hipError_t launch_plaquette_noalloc(const LaunchArgs &a, double *d_out, hipStream_t st)
{
    const uint32_t nblk = plaquette_blocks(a.volume);
    if (nblk > kNoAllocPlaqBlocks)
        return hipErrorInvalidValue; // the caller checked the size first
    double *partials = nullptr;
    const hipError_t e = scratch_on_current_device(&partials);
    if (e != hipSuccess)
        return e;
    launch_plaquette_into(a, nblk, partials, d_out, st);
    return hipSuccess;
}

void launch_polyakov(const LaunchArgs &a, const WorkLayout &w, double *d_out, double *d_corr, hipStream_t st)
{
    const Geom g = make_geom(a.n, a.tile, a.tile_y);
    double *Lf = reinterpret_cast<double *>(a.work + w.off_lfield);
    double *pp = reinterpret_cast<double *>(a.work + w.off_poly);
    if (a.prec == kF32)
        polyakov_kernel<float><<<w.nblk_poly, kBlock, 0, st>>>(links_of<float>(a), g, Lf, pp);
    else
        polyakov_kernel<double><<<w.nblk_poly, kBlock, 0, st>>>(links_of<double>(a), g, Lf, pp);
    colsum_kernel<<<2, kBlock, 0, st>>>(pp, w.nblk_poly, 1.0 / (double)g.vs, d_out);
    if (d_corr && w.rmax > 0) {
        double *cp = reinterpret_cast<double *>(a.work + w.off_corr);
        polycorr_kernel<<<dim3(w.nblk_corr, corr_groups(w.rmax)), kBlock, 0, st>>>(Lf, g, cp, (uint32_t)w.rmax);
        colsum_kernel<<<w.rmax, kBlock, 0, st>>>(cp, w.nblk_corr, 1.0 / (3.0 * (double)g.vs), d_corr);
    }
}

void launch_polyakov_batch(const void *d_table, int count, int prec, const BatchPolyGrid &grid, double *d_poly,
                           double *d_corr, uint32_t corr_stride, hipStream_t st)
{
    const BatchEntry *tab = static_cast<const BatchEntry *>(d_table);
    if (prec == kF32)
        polyakov_batch_kernel<float><<<grid.poly_blocks, kBlock, 0, st>>>(tab, count);
    else
        polyakov_batch_kernel<double><<<grid.poly_blocks, kBlock, 0, st>>>(tab, count);
    if (d_corr)
        polycorr_batch_kernel<<<grid.corr_blocks, kBlock, 0, st>>>(tab, count);
    const uint32_t outs = d_corr ? grid.columns : 2u * (uint32_t)count;
    polysum_batch_kernel<<<outs, kBlock, 0, st>>>(tab, count, d_poly, d_corr, corr_stride);
}

void launch_measure(const LaunchArgs &a, const WorkLayout &w, double *d_plaq, double *d_poly, double *d_corr,
                    hipStream_t st)
{
    const Geom g = make_geom(a.n, a.tile, a.tile_y);
    double *Lf = reinterpret_cast<double *>(a.work + w.off_lfield);
    double *pm = reinterpret_cast<double *>(a.work + w.off_meas);
    if (a.prec == kF32)
        measure_kernel<float><<<w.nblk_meas, kBlock, 0, st>>>(links_of<float>(a), g, Lf, pm);
    else
        measure_kernel<double><<<w.nblk_meas, kBlock, 0, st>>>(links_of<double>(a), g, Lf, pm);
    launch_plaquette_finish(pm, w.nblk_meas, 1.0 / (double)a.volume, d_plaq, st);
    colsum_kernel<<<2, kBlock, 0, st>>>(pm + (size_t)6 * w.nblk_meas, w.nblk_meas, 1.0 / (double)g.vs, d_poly);
    if (d_corr && w.rmax > 0) {
        double *cp = reinterpret_cast<double *>(a.work + w.off_corr);
        polycorr_kernel<<<dim3(w.nblk_corr, corr_groups(w.rmax)), kBlock, 0, st>>>(Lf, g, cp, (uint32_t)w.rmax);
        colsum_kernel<<<w.rmax, kBlock, 0, st>>>(cp, w.nblk_corr, 1.0 / (3.0 * (double)g.vs), d_corr);
    }
}

} // namespace su2

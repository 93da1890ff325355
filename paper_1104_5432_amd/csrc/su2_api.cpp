// su2_api.cpp -- the C ABI declared in include/su2.h: argument checks (all
// before any HIP call), workspace layout, launch sequencing, error codes.
#include "su2.h"
#include "su2_device.hpp"
#include "su2_launch.hpp"
#include "su2_learned.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>

namespace {

thread_local char g_last_error[256] = "";

int fail(int code, const char *msg)
{
    std::snprintf(g_last_error, sizeof g_last_error, "%s", msg);
    return code;
}

bool dims_ok(const int32_t n[4])
{
    if (!n)
        return false;
    uint64_t vol = 1;
    for (int d = 0; d < 4; ++d) {
        if (n[d] < 2 || (n[d] & 1))
            return false;
        vol *= (uint64_t)n[d];
        if (vol >= (1ull << 32))
            return false;
    }
    return true;
}

bool prec_ok(int32_t p)
{
    return p == SU2_F64 || p == SU2_F32;
}

bool aligned(const void *p, uintptr_t a)
{
    return ((uintptr_t)p % a) == 0;
}

uint64_t plane_stride_of(const int32_t n[4], int32_t prec)
{
    const uint64_t vol = (uint64_t)n[0] * n[1] * n[2] * n[3];
    return su2::plane_stride((uint32_t)(vol / 2), prec == SU2_F64);
}

// 8 planes (F32) or 16 sub-planes (F64) of plane_stride_of 16-byte elements
uint64_t links_bytes_of(const int32_t n[4], int32_t prec)
{
    return plane_stride_of(n, prec) * (prec == SU2_F32 ? 8u : 16u) * 16u;
}

// Checks of a lattice descriptor's extents, precision, id, walk and links;
// fills *out (without a workspace).
int check_lattice_links(const su2_lattice_t *lat, su2::LaunchArgs *out)
{
    if (!lat)
        return fail(SU2_EINVAL, "lattice descriptor is NULL");
    if (!prec_ok(lat->prec))
        return fail(SU2_EINVAL, "precision must be SU2_F64 or SU2_F32");
    if (!dims_ok(lat->n))
        return fail(SU2_EDIMS, "extents must be even, >= 2, with volume < 2^32");
    if (lat->lattice_id < 0 || lat->lattice_id >= (1 << 27))
        return fail(SU2_EINVAL, "lattice_id must be in [0, 2^27)");
    if (lat->tile > 0 && (lat->tile > lat->n[2] || lat->n[2] % lat->tile != 0))
        return fail(SU2_EINVAL, "a positive tile (strip width) must divide Nz");
    if (lat->tile < -3)
        return fail(SU2_EINVAL, "tile must be -3, -2, -1, 0 or a divisor of Nz");
    if (lat->tile_y < 0 || (lat->tile_y > 0 && (lat->tile_y > lat->n[1] || lat->n[1] % lat->tile_y != 0)))
        return fail(SU2_EINVAL, "tile_y must be 0 or a divisor of Ny");
    if (!lat->links)
        return fail(SU2_EINVAL, "links must be a non-NULL device pointer");
    if (!aligned(lat->links, 16))
        return fail(SU2_EALIGN, "links must be 16-byte aligned");
    out->n[0] = lat->n[0];
    out->n[1] = lat->n[1];
    out->n[2] = lat->n[2];
    out->n[3] = lat->n[3];
    out->prec = lat->prec;
    out->lattice_id = lat->lattice_id;
    out->tile = lat->tile;
    out->tile_y = lat->tile_y;
    out->volume = (uint64_t)lat->n[0] * lat->n[1] * lat->n[2] * lat->n[3];
    out->links = lat->links;
    out->work = nullptr;
    out->flags = nullptr;
    return SU2_OK;
}

// Common checks of a lattice descriptor, its workspace included.
int check_lattice(const su2_lattice_t *lat, su2::LaunchArgs *out, su2::WorkLayout *wl)
{
    int rc = check_lattice_links(lat, out);
    if (rc)
        return rc;
    if (!lat->work)
        return fail(SU2_EINVAL, "work must be a non-NULL device pointer");
    if (!aligned(lat->work, 16))
        return fail(SU2_EALIGN, "work must be 16-byte aligned");
    const su2::WorkLayout w = su2::work_layout(lat->n);
    if (lat->work_bytes < w.total)
        return fail(SU2_EWORK, "work_bytes is smaller than su2_workspace_bytes()");
    {
        const uintptr_t l0 = (uintptr_t)lat->links, l1 = l0 + links_bytes_of(lat->n, lat->prec);
        const uintptr_t w0 = (uintptr_t)lat->work, w1 = w0 + w.total;
        if (l0 < w1 && w0 < l1)
            return fail(SU2_EINVAL, "links and work must not overlap");
    }
    out->work = static_cast<char *>(lat->work);
    out->flags = reinterpret_cast<uint32_t *>(lat->work);
    if (wl)
        *wl = w;
    return SU2_OK;
}

int check_class(int32_t mu, int32_t parity)
{
    if (mu < 0 || mu > 3 || (parity != 0 && parity != 1))
        return fail(SU2_EINVAL, "mu must be 0..3 and parity 0 or 1");
    return SU2_OK;
}

int check_beta(double beta)
{
    if (!std::isfinite(beta) || beta < 0.0)
        return fail(SU2_EINVAL, "beta must be finite and >= 0");
    return SU2_OK;
}

int launched()
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::snprintf(g_last_error, sizeof g_last_error, "HIP: %s", hipGetErrorString(e));
        return SU2_EHIP;
    }
    return SU2_OK;
}

uint64_t round256(uint64_t b)
{
    return (b + 255) & ~uint64_t(255);
}

constexpr int kMaxBatch = 4096;
constexpr int kMaxBatchOr = 64; // overrelaxation sweeps of one persistent batched call
// Polls of a persistent sweep's barrier wait before it gives up: each poll
// is a device-scope load (about a microsecond) and a short sleep, so a few
// tenths of a second, against a legitimate wait of one block's work (tens
// of microseconds).
constexpr uint32_t kDefaultSpinLimit = 1u << 18;

uint32_t round8(uint32_t b)
{
    return (b + 7u) & ~7u;
}

// Checks of a batch's descriptors; *total receives the blocks of one batched class launch.
int check_batch(const su2_lattice_t *lats, int32_t count, uint32_t *total)
{
    if (!lats)
        return fail(SU2_EINVAL, "lats must be a non-NULL host array");
    if (count < 1 || count > kMaxBatch)
        return fail(SU2_EINVAL, "count must be in [1, 4096]");
    uint64_t sum = 0;
    for (int j = 0; j < count; ++j) {
        su2::LaunchArgs a;
        const int rc = check_lattice(&lats[j], &a, nullptr);
        if (rc)
            return rc;
        if (lats[j].prec != lats[0].prec)
            return fail(SU2_EINVAL, "all lattices of a batch must have the same precision");
        sum += round8(su2::class_blocks(a));
    }
    if (sum >= (1ull << 31))
        return fail(SU2_EDIMS, "a batch must have fewer than 2^31 blocks per class");
    // Distinct lattices: one launch updates every lattice's class at once, so
    // shared links would race, a shared workspace would mix two lattices'
    // flags and partials, and a repeated lattice id would repeat a random
    // stream.
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    std::vector<int32_t> ids;
    spans.reserve(2 * (size_t)count);
    ids.reserve((size_t)count);
    for (int j = 0; j < count; ++j) {
        const uintptr_t l0 = (uintptr_t)lats[j].links, w0 = (uintptr_t)lats[j].work;
        spans.emplace_back(l0, l0 + links_bytes_of(lats[j].n, lats[j].prec));
        spans.emplace_back(w0, w0 + su2::work_layout(lats[j].n).total);
        ids.push_back(lats[j].lattice_id);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k].first < spans[k - 1].second)
            return fail(SU2_EINVAL, "the lattices of a batch must not share or overlap links or work");
    std::sort(ids.begin(), ids.end());
    if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
        return fail(SU2_EINVAL, "the lattices of a batch must have distinct lattice ids");
    if (total)
        *total = (uint32_t)sum;
    return SU2_OK;
}

} // namespace

namespace su2 {

WorkLayout work_layout(const int32_t n[4])
{
    const uint64_t vol = (uint64_t)n[0] * n[1] * n[2] * n[3];
    const uint64_t vs = (uint64_t)n[0] * n[1] * n[2];
    int ns = n[0] < n[1] ? n[0] : n[1];
    ns = ns < n[2] ? ns : n[2];
    WorkLayout w;
    w.rmax = ns / 2;
    auto blocks = [](uint64_t items, uint64_t cap) {
        uint64_t b = (items + 255) / 256;
        return (uint32_t)(b < cap ? (b > 0 ? b : 1) : cap);
    };
    // one block per 256 cb indices: also the grid of an update class
    // (class_blocks), whose blocks write here when a last sweep takes the
    // plaquette, so the two must stay equal
    w.nblk_plaq = su2::plaquette_blocks(vol);
    w.nblk_poly = blocks(vs, 2048);
    w.nblk_corr = blocks(vs, 1024);
    uint64_t off = 256; // flags word
    w.off_plaq = off;
    off += round256((uint64_t)w.nblk_plaq * 6 * sizeof(double));
    w.off_poly = off;
    off += round256((uint64_t)w.nblk_poly * 2 * sizeof(double));
    w.off_corr = off;
    off += round256((uint64_t)w.nblk_corr * (uint64_t)(w.rmax > 0 ? w.rmax : 1) * sizeof(double));
    w.off_lfield = off;
    off += round256(vs * sizeof(double));
    w.nblk_meas = (uint32_t)((vs + 255) / 256); // one block per 256 spatial sites
    w.off_meas = off;
    off += round256((uint64_t)w.nblk_meas * 8 * sizeof(double));
    w.total = off;
    return w;
}

} // namespace su2

extern "C" {

uint64_t su2_links_bytes(const int32_t n[4], int32_t prec)
{
    if (!dims_ok(n) || !prec_ok(prec))
        return 0;
    return links_bytes_of(n, prec);
}

uint64_t su2_plane_stride(const int32_t n[4], int32_t prec)
{
    if (!dims_ok(n) || !prec_ok(prec))
        return 0;
    return plane_stride_of(n, prec);
}

uint64_t su2_workspace_bytes(const int32_t n[4], int32_t prec)
{
    if (!dims_ok(n) || !prec_ok(prec))
        return 0;
    return su2::work_layout(n).total;
}

int su2_init_cold(const su2_lattice_t *lat, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (rc)
        return rc;
    su2::launch_init(a, 0, 0, (hipStream_t)stream);
    return launched();
}

int su2_init_hot(const su2_lattice_t *lat, uint64_t seed, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (rc)
        return rc;
    su2::launch_init(a, 1, seed, (hipStream_t)stream);
    return launched();
}

int su2_heatbath_halfsweep(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t sweep, int32_t mu,
                           int32_t parity, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (!rc)
        rc = check_beta(beta);
    if (!rc)
        rc = check_class(mu, parity);
    if (rc)
        return rc;
    su2::launch_heatbath(a, beta, seed, sweep, nullptr, mu, parity, nullptr, (hipStream_t)stream);
    return launched();
}

int su2_heatbath_sweep(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t sweep, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (!rc)
        rc = check_beta(beta);
    if (rc)
        return rc;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            su2::launch_heatbath(a, beta, seed, sweep, nullptr, mu, p, nullptr, (hipStream_t)stream);
    return launched();
}

int su2_overrelax_halfsweep(const su2_lattice_t *lat, int32_t mu, int32_t parity, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (!rc)
        rc = check_class(mu, parity);
    if (rc)
        return rc;
    su2::launch_overrelax(a, mu, parity, nullptr, (hipStream_t)stream);
    return launched();
}

int su2_overrelax(const su2_lattice_t *lat, int32_t n_sweeps, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (rc)
        return rc;
    if (n_sweeps < 0)
        return fail(SU2_EINVAL, "n_sweeps must be >= 0");
    for (int s = 0; s < n_sweeps; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                su2::launch_overrelax(a, mu, p, nullptr, (hipStream_t)stream);
    return launched();
}

namespace {

int check_plaq_out(const double *d_plaq)
{
    if (!d_plaq)
        return fail(SU2_EINVAL, "d_plaq must be a device pointer to 7 doubles");
    if (!aligned(d_plaq, 8))
        return fail(SU2_EALIGN, "d_plaq must be 8-byte aligned");
    return SU2_OK;
}

// The plaquette-partials region when class (mu, p) of the last sweep writes
// plane partials, else null.
double *plaq_region(const su2::LaunchArgs &a, const su2::WorkLayout &w, int mu, int p)
{
    return (p == 1 && mu >= 1) ? reinterpret_cast<double *>(a.work + w.off_plaq) : nullptr;
}

}

int su2_heatbath_sweep_measured(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t sweep,
                                double *d_plaq, void *stream)
{
    su2::LaunchArgs a;
    su2::WorkLayout w;
    int rc = check_lattice(lat, &a, &w);
    if (!rc)
        rc = check_beta(beta);
    if (!rc)
        rc = check_plaq_out(d_plaq);
    if (rc)
        return rc;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            su2::launch_heatbath(a, beta, seed, sweep, nullptr, mu, p, plaq_region(a, w, mu, p),
                                 (hipStream_t)stream);
    su2::launch_plaquette_sum(a, w, d_plaq, (hipStream_t)stream);
    return launched();
}

int su2_overrelax_measured(const su2_lattice_t *lat, int32_t n_sweeps, double *d_plaq, void *stream)
{
    su2::LaunchArgs a;
    su2::WorkLayout w;
    int rc = check_lattice(lat, &a, &w);
    if (!rc)
        rc = check_plaq_out(d_plaq);
    if (rc)
        return rc;
    if (n_sweeps < 0)
        return fail(SU2_EINVAL, "n_sweeps must be >= 0");
    if (n_sweeps == 0) {
        su2::launch_plaquette(a, w, d_plaq, (hipStream_t)stream);
        return launched();
    }
    for (int s = 0; s < n_sweeps; ++s)
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                su2::launch_overrelax(a, mu, p, s + 1 == n_sweeps ? plaq_region(a, w, mu, p) : nullptr,
                                      (hipStream_t)stream);
    su2::launch_plaquette_sum(a, w, d_plaq, (hipStream_t)stream);
    return launched();
}

int su2_plaquette(const su2_lattice_t *lat, double *d_out, void *stream)
{
    su2::LaunchArgs a;
    su2::WorkLayout w;
    int rc = check_lattice(lat, &a, &w);
    if (rc)
        return rc;
    if (!d_out)
        return fail(SU2_EINVAL, "d_out must be a device pointer to 7 doubles");
    if (!aligned(d_out, 8))
        return fail(SU2_EALIGN, "d_out must be 8-byte aligned");
    su2::launch_plaquette(a, w, d_out, (hipStream_t)stream);
    return launched();
}

int su2_plaquette_noalloc(const su2_lattice_t *lat, double *d_out, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice_links(lat, &a); // work and work_bytes are not used
    if (rc)
        return rc;
    if (su2::plaquette_blocks(a.volume) > su2::kNoAllocPlaqBlocks)
        return fail(SU2_EDIMS, "su2_plaquette_noalloc takes at most 44,739,072 sites per parity "
                               "(V/2 <= 256 x 174762)");
    if (!d_out)
        return fail(SU2_EINVAL, "d_out must be a device pointer to 7 doubles");
    if (!aligned(d_out, 8))
        return fail(SU2_EALIGN, "d_out must be 8-byte aligned");
    const hipError_t e = su2::launch_plaquette_noalloc(a, d_out, (hipStream_t)stream);
    if (e != hipSuccess) {
        std::snprintf(g_last_error, sizeof g_last_error, "HIP: %s", hipGetErrorString(e));
        return SU2_EHIP;
    }
    return launched();
}

int su2_polyakov(const su2_lattice_t *lat, double *d_out, double *d_corr, void *stream)
{
    su2::LaunchArgs a;
    su2::WorkLayout w;
    int rc = check_lattice(lat, &a, &w);
    if (rc)
        return rc;
    if (!d_out)
        return fail(SU2_EINVAL, "d_out must be a device pointer to 2 doubles");
    if (!aligned(d_out, 8) || (d_corr && !aligned(d_corr, 8)))
        return fail(SU2_EALIGN, "d_out and d_corr must be 8-byte aligned");
    su2::launch_polyakov(a, w, d_out, d_corr, (hipStream_t)stream);
    return launched();
}

int su2_measure(const su2_lattice_t *lat, double *d_plaq, double *d_poly, double *d_corr, void *stream)
{
    su2::LaunchArgs a;
    su2::WorkLayout w;
    int rc = check_lattice(lat, &a, &w);
    if (rc)
        return rc;
    if (!d_plaq || !d_poly)
        return fail(SU2_EINVAL, "d_plaq and d_poly must be device pointers to 7 and 2 doubles");
    if (!aligned(d_plaq, 8) || !aligned(d_poly, 8) || (d_corr && !aligned(d_corr, 8)))
        return fail(SU2_EALIGN, "d_plaq, d_poly and d_corr must be 8-byte aligned");
    su2::launch_measure(a, w, d_plaq, d_poly, d_corr, (hipStream_t)stream);
    return launched();
}

uint64_t su2_batch_table_bytes(int32_t count)
{
    if (count < 1 || count > kMaxBatch)
        return 0;
    return (uint64_t)count * su2::batch_entry_bytes();
}

int su2_batch_fill(const su2_lattice_t *lats, const double *betas, int32_t count, void *host_table,
                   uint64_t table_bytes)
{
    int rc = check_batch(lats, count, nullptr);
    if (rc)
        return rc;
    if (!betas || !host_table)
        return fail(SU2_EINVAL, "betas and host_table must be non-NULL host pointers");
    if (table_bytes < su2_batch_table_bytes(count))
        return fail(SU2_EWORK, "table_bytes is smaller than su2_batch_table_bytes()");
    for (int j = 0; j < count; ++j)
        if ((rc = check_beta(betas[j])))
            return rc;
    su2::BatchOffsets o = {};
    for (int j = 0; j < count; ++j) {
        su2::LaunchArgs a;
        su2::WorkLayout w;
        check_lattice(&lats[j], &a, &w);
        o.nblocks = round8(su2::class_blocks(a));
        su2::fill_batch_entry(a, w, betas[j], o, static_cast<char *>(host_table) + j * su2::batch_entry_bytes());
        o.block0 += o.nblocks;
        if (!su2::batch_own_launch(a.volume))
            o.sub_block0 += o.nblocks;
        o.pblock0 += w.nblk_poly;
        o.cblock0 += w.nblk_corr * su2::corr_groups(w.rmax);
        o.ocol0 += 2u + (uint32_t)w.rmax;
    }
    return SU2_OK;
}

int su2_batch_polyakov(const su2_lattice_t *lats, int32_t count, const void *d_table, double *d_poly,
                       double *d_corr, int32_t corr_stride, void *stream)
{
    int rc = check_batch(lats, count, nullptr);
    if (rc)
        return rc;
    if (!d_table || !aligned(d_table, 8))
        return fail(SU2_EINVAL, "d_table must be an 8-byte aligned device pointer");
    if (!d_poly)
        return fail(SU2_EINVAL, "d_poly must be a device pointer to 2*count doubles");
    if (!aligned(d_poly, 8) || (d_corr && !aligned(d_corr, 8)))
        return fail(SU2_EALIGN, "d_poly and d_corr must be 8-byte aligned");
    su2::BatchPolyGrid grid = {};
    int rmax = 0;
    for (int j = 0; j < count; ++j) {
        const su2::WorkLayout w = su2::work_layout(lats[j].n);
        grid.poly_blocks += w.nblk_poly;
        grid.corr_blocks += w.nblk_corr * su2::corr_groups(w.rmax);
        grid.columns += 2u + (uint32_t)w.rmax;
        rmax = w.rmax > rmax ? w.rmax : rmax;
    }
    if (d_corr && corr_stride < rmax)
        return fail(SU2_EINVAL, "corr_stride must be >= min(Nx,Ny,Nz)/2 of every lattice of the batch");
    su2::launch_polyakov_batch(d_table, count, lats[0].prec, grid, d_poly, d_corr, (uint32_t)corr_stride,
                               (hipStream_t)stream);
    return launched();
}

int su2_batch_heatbath_sweep(const su2_lattice_t *lats, int32_t count, const void *d_table, uint64_t seed,
                             uint32_t sweep, const uint32_t *d_sweep, void *stream)
{
    uint32_t total = 0;
    int rc = check_batch(lats, count, &total);
    if (rc)
        return rc;
    if (!d_table || !aligned(d_table, 8))
        return fail(SU2_EINVAL, "d_table must be an 8-byte aligned device pointer");
    if (d_sweep && !aligned(d_sweep, 4))
        return fail(SU2_EALIGN, "d_sweep must be 4-byte aligned");
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            su2::launch_heatbath_batch(d_table, count, lats[0].prec, total, mu, p, seed, sweep, d_sweep,
                                       (hipStream_t)stream);
    return launched();
}

int su2_batch_overrelax(const su2_lattice_t *lats, int32_t count, const void *d_table, int32_t n_sweeps,
                        void *stream)
{
    uint32_t total = 0;
    int rc = check_batch(lats, count, &total);
    if (rc)
        return rc;
    if (!d_table || !aligned(d_table, 8))
        return fail(SU2_EINVAL, "d_table must be an 8-byte aligned device pointer");
    if (n_sweeps < 0)
        return fail(SU2_EINVAL, "n_sweeps must be >= 0");
    // lattices with launches of their own (batch_own_launch), and the
    // batched grid of the others (the table's sub_block0 ranges)
    std::vector<su2::LaunchArgs> own;
    uint32_t batched = 0;
    for (int j = 0; j < count; ++j) {
        su2::LaunchArgs a;
        check_lattice(&lats[j], &a, nullptr);
        if (su2::batch_own_launch(a.volume))
            own.push_back(a);
        else
            batched += round8(su2::class_blocks(a));
    }
    // Lattice by lattice: all sweeps of one large lattice before the next
    // keep its links in the Infinity Cache between classes (the scan's five
    // 64^3 x 8 lattices, 4 sweeps: 3.9 ms this way, 4.85 ms class by class
    // across the lattices).  Lattices are independent, so only each
    // lattice's own class order matters.
    for (const su2::LaunchArgs &a : own)
        for (int s = 0; s < n_sweeps; ++s)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p)
                    su2::launch_overrelax(a, mu, p, nullptr, (hipStream_t)stream);
    if (batched)
        for (int s = 0; s < n_sweeps; ++s)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p)
                    su2::launch_overrelax_batch(d_table, count, lats[0].prec, batched, mu, p, (hipStream_t)stream);
    return launched();
}

int su2_batch_sweep(const su2_lattice_t *lats, int32_t count, const void *d_table, uint64_t seed, uint32_t sweep,
                    const uint32_t *d_sweep, int32_t n_or, uint32_t *d_sync, uint32_t spin_limit, void *stream)
{
    uint32_t total = 0;
    int rc = check_batch(lats, count, &total);
    if (rc)
        return rc;
    if (!d_table || !aligned(d_table, 8))
        return fail(SU2_EINVAL, "d_table must be an 8-byte aligned device pointer");
    if (d_sweep && !aligned(d_sweep, 4))
        return fail(SU2_EALIGN, "d_sweep must be 4-byte aligned");
    if (n_or < 0 || n_or > kMaxBatchOr)
        return fail(SU2_EINVAL, "n_or must be in [0, 64]");
    if (!d_sync)
        return fail(SU2_EINVAL, "d_sync must be a device pointer");
    if (!aligned(d_sync, 4))
        return fail(SU2_EALIGN, "d_sync must be 4-byte aligned");
    if (!su2::launch_batch_sweep(d_table, count, lats[0].prec, total, seed, sweep, d_sweep, n_or, d_sync,
                                 spin_limit ? spin_limit : kDefaultSpinLimit, (hipStream_t)stream))
        return fail(SU2_EHIP, "the persistent sweep kernel cannot be resident on this device");
    return launched();
}

int su2_sweep_advance(uint32_t *d_sweep, void *stream)
{
    if (!d_sweep)
        return fail(SU2_EINVAL, "d_sweep must be a device pointer");
    if (!aligned(d_sweep, 4))
        return fail(SU2_EALIGN, "d_sweep must be 4-byte aligned");
    su2::launch_sweep_advance(d_sweep, (hipStream_t)stream);
    return launched();
}

int32_t su2_lp_param_count(void)
{
    return su2::lp::param_count();
}

static bool lp_dims_ok(const int32_t n[4])
{
    return dims_ok(n) && n[0] % 8 == 0 && n[1] % 8 == 0 && n[2] % 8 == 0;
}

uint64_t su2_lp_workspace_bytes(const int32_t n[4])
{
    if (!lp_dims_ok(n))
        return 0;
    return su2::lp::work_layout(n).total;
}

static int check_lp(const su2_lattice_t *lat, su2::LaunchArgs *a)
{
    int rc = check_lattice(lat, a, nullptr);
    if (rc)
        return rc;
    if (!lp_dims_ok(lat->n))
        return fail(SU2_EDIMS, "the learned proposal needs Nx, Ny, Nz multiples of 8");
    return SU2_OK;
}

static int check_lpwork(const su2_lattice_t *lat, const float *d_params, const void *d_lpwork, uint64_t bytes)
{
    if (!d_params || !d_lpwork)
        return fail(SU2_EINVAL, "d_params and d_lpwork must be non-NULL device pointers");
    if (!aligned(d_params, 4) || !aligned(d_lpwork, 16))
        return fail(SU2_EALIGN, "d_params must be 4-byte and d_lpwork 16-byte aligned");
    if (bytes < su2::lp::work_layout(lat->n).total)
        return fail(SU2_EWORK, "lpwork_bytes is smaller than su2_lp_workspace_bytes()");
    return SU2_OK;
}

int su2_lp_forward(const su2_lattice_t *lat, const float *d_params, void *d_lpwork, uint64_t lpwork_bytes,
                   float *d_y, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lp(lat, &a);
    if (!rc)
        rc = check_lpwork(lat, d_params, d_lpwork, lpwork_bytes);
    if (rc)
        return rc;
    if (!d_y || !aligned(d_y, 4))
        return fail(SU2_EINVAL, "d_y must be a 4-byte aligned device pointer");
    su2::lp::launch_forward(a, d_params, static_cast<char *>(d_lpwork), d_y, (hipStream_t)stream);
    return launched();
}

int su2_lp_loss_grad(const su2_lattice_t *lat, double beta, const float *d_params, void *d_lpwork,
                     uint64_t lpwork_bytes, float *d_grad, double *d_loss, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lp(lat, &a);
    if (!rc)
        rc = check_lpwork(lat, d_params, d_lpwork, lpwork_bytes);
    if (!rc)
        rc = check_beta(beta);
    if (rc)
        return rc;
    if (!d_grad || !d_loss || !aligned(d_grad, 4) || !aligned(d_loss, 8))
        return fail(SU2_EINVAL, "d_grad and d_loss must be aligned device pointers");
    su2::lp::launch_loss_grad(a, beta, d_params, static_cast<char *>(d_lpwork), d_grad, d_loss,
                              (hipStream_t)stream);
    return launched();
}

int su2_lp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t count, int32_t step, float lr,
                float beta1, float beta2, float eps, void *stream)
{
    if (!d_params || !d_grad || !d_m || !d_v)
        return fail(SU2_EINVAL, "Adam needs four device arrays");
    if (count < 1 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(SU2_EINVAL, "bad Adam hyper-parameters (count >= 1, step >= 1, 0 <= beta < 1, eps > 0)");
    su2::lp::launch_adam(d_params, d_grad, d_m, d_v, (uint32_t)count, step, lr, beta1, beta2, eps,
                         (hipStream_t)stream);
    return launched();
}

int su2_lp_move(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t step, int32_t parity, int32_t colour,
                const float *d_y, uint32_t *d_accepted, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lp(lat, &a);
    if (!rc)
        rc = check_beta(beta);
    if (rc)
        return rc;
    if ((parity != 0 && parity != 1) || colour < 0 || colour > 7 || step >= (1u << 28))
        return fail(SU2_EINVAL, "parity 0/1, colour 0..7, step < 2^28");
    if (!d_y || !d_accepted || !aligned(d_y, 4) || !aligned(d_accepted, 4))
        return fail(SU2_EINVAL, "d_y and d_accepted must be aligned device pointers");
    su2::lp::launch_block_move(a, beta, seed, step, parity, colour, d_y, d_accepted, (hipStream_t)stream);
    return launched();
}

int su2_lp_sweep(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t step, const float *d_y,
                 uint32_t *d_accepted, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lp(lat, &a);
    if (!rc)
        rc = check_beta(beta);
    if (rc)
        return rc;
    if (step >= (1u << 28))
        return fail(SU2_EINVAL, "step < 2^28");
    if (!d_y || !d_accepted || !aligned(d_y, 4) || !aligned(d_accepted, 4))
        return fail(SU2_EINVAL, "d_y and d_accepted must be aligned device pointers");
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < 8; ++k)
            su2::lp::launch_block_move(a, beta, seed, step, p, k, d_y, d_accepted, (hipStream_t)stream);
    return launched();
}

int su2_get_flags(const su2_lattice_t *lat, uint32_t *d_flags, void *stream)
{
    su2::LaunchArgs a;
    int rc = check_lattice(lat, &a, nullptr);
    if (rc)
        return rc;
    if (!d_flags)
        return fail(SU2_EINVAL, "d_flags must be a device pointer");
    if (!aligned(d_flags, 4))
        return fail(SU2_EALIGN, "d_flags must be 4-byte aligned");
    su2::launch_get_flags(a, d_flags, (hipStream_t)stream);
    return launched();
}

const char *su2_strerror(int code)
{
    switch (code) {
    case SU2_OK: return "ok";
    case SU2_EINVAL: return "invalid argument";
    case SU2_EDIMS: return "invalid lattice extents";
    case SU2_EALIGN: return "misaligned pointer";
    case SU2_EWORK: return "workspace too small";
    case SU2_EHIP: return "HIP launch failed";
    default: return "unknown error";
    }
}

const char *su2_last_error(void)
{
    return g_last_error;
}

} // extern "C"

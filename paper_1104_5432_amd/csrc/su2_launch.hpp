// su2_launch.hpp -- internal interface between the C-ABI facade (argument
// checks, workspace layout) and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace su2 {

constexpr int kF64 = 0;
constexpr int kF32 = 1;

// Workspace layout: the flags word, then the reduction partials and the
// Polyakov-loop field, each region 256-byte aligned.
struct WorkLayout {
    uint64_t off_plaq, off_poly, off_corr, off_lfield, off_meas, total;
    uint32_t nblk_plaq, nblk_poly, nblk_corr, nblk_meas;
    int rmax;
};

struct LaunchArgs {
    int32_t n[4];
    int prec;
    int lattice_id;
    int tile;
    int tile_y;
    uint64_t volume;
    void *links;
    char *work;
    uint32_t *flags;
};

WorkLayout work_layout(const int32_t n[4]);

// Blocks of a class update and of the plaquette pass: one per 256 cb indices.
inline uint32_t plaquette_blocks(uint64_t volume)
{
    return (uint32_t)((volume / 2 + 255) / 256);
}

// The no-allocation plaquette's scratch holds the partials of at most this
// many blocks (6 planes each, 8 MiB in all): V/2 <= 256 x 174762, which
// takes in 96^4.
constexpr uint32_t kNoAllocPlaqBlocks = 174762;

// Separations of the Polyakov correlator taken by one block (one load of a
// site's L for the group); corr_groups(rmax) groups cover r = 1..rmax.
constexpr uint32_t kCorrGroup = 8;
__host__ __device__ inline uint32_t corr_groups(int rmax)
{
    return rmax > 0 ? ((uint32_t)rmax + kCorrGroup - 1u) / kCorrGroup : 0u;
}

uint32_t class_blocks(const LaunchArgs &a);
uint64_t batch_entry_bytes();
// A lattice's ranges in the batched grids: update blocks (block0, nblocks),
// Polyakov blocks (pblock0), correlator blocks (cblock0) and output columns
// of the batched Polyakov sums (ocol0); each the sum over earlier lattices.
struct BatchOffsets {
    uint32_t block0, nblocks, sub_block0, pblock0, cblock0, ocol0;
};
void fill_batch_entry(const LaunchArgs &a, const WorkLayout &w, double beta, const BatchOffsets &o, void *dst);
// Grid sizes of the batched Polyakov launches, from the same descriptors.
struct BatchPolyGrid {
    uint32_t poly_blocks, corr_blocks, columns; // columns with the correlator (2 + rmax per lattice)
};

void launch_init(const LaunchArgs &a, int hot, uint64_t seed, hipStream_t st);
// plaq_partials: null, or (classes (mu >= 1, odd) of a sweep that should
// leave the plaquette behind) the plaquette-partials region of the workspace.
void launch_heatbath(const LaunchArgs &a, double beta, uint64_t seed, uint32_t sweep, const uint32_t *d_sweep,
                     int mu, int par, double *plaq_partials, hipStream_t st);
void launch_heatbath_batch(const void *d_table, int count, int prec, uint32_t total_blocks, int mu, int par,
                           uint64_t seed, uint32_t sweep, const uint32_t *d_sweep, hipStream_t st);
void launch_overrelax_batch(const void *d_table, int count, int prec, uint32_t total_blocks, int mu, int par,
                            hipStream_t st);
// One persistent launch: the heat-bath sweep and n_or overrelaxation sweeps
// of every lattice of the batch, classes separated by a grid-wide barrier on
// *d_sync; false (nothing launched) if the kernel cannot be resident.
bool launch_batch_sweep(const void *d_table, int count, int prec, uint32_t total_blocks, uint64_t seed,
                        uint32_t sweep, const uint32_t *d_sweep, int n_or, uint32_t *d_sync, uint32_t spin_limit,
                        hipStream_t st);
void launch_sweep_advance(uint32_t *d_sweep, hipStream_t st);
void launch_overrelax(const LaunchArgs &a, int mu, int par, double *plaq_partials, hipStream_t st);
// Walk values (descriptor field `tile`) of the LDS-staged updates: with -2
// the overrelaxation classes whose lattice admits a slab plan run
// overrelax_staged_kernel, with -3 the heat-bath classes too
// (heatbath_staged_kernel); every other kernel walks the default strips.
constexpr int kTileStaged = -2;
constexpr int kTileStagedBoth = -3;
// The LDS-staged overrelaxation / heat bath of one class; false (nothing
// launched) if no slab plan fits the lattice on the current device.
bool launch_overrelax_staged(const LaunchArgs &a, int mu, int par, hipStream_t st);
bool launch_heatbath_staged(const LaunchArgs &a, double beta, uint64_t seed, uint32_t sweep, const uint32_t *d_sweep,
                            int mu, int par, hipStream_t st);
void launch_plaquette_sum(const LaunchArgs &a, const WorkLayout &w, double *d_out, hipStream_t st);
void launch_plaquette(const LaunchArgs &a, const WorkLayout &w, double *d_out, hipStream_t st);
// The plaquette pass with its partials in the library's static scratch
// (a.work is not used); the lattice must have at most kNoAllocPlaqBlocks
// plaquette blocks.  Returns the HIP error of the scratch lookup, if any.
hipError_t launch_plaquette_noalloc(const LaunchArgs &a, double *d_out, hipStream_t st);
void launch_polyakov(const LaunchArgs &a, const WorkLayout &w, double *d_out, double *d_corr, hipStream_t st);
// d_corr null: no correlator.
void launch_polyakov_batch(const void *d_table, int count, int prec, const BatchPolyGrid &grid, double *d_poly,
                           double *d_corr, uint32_t corr_stride, hipStream_t st);
void launch_measure(const LaunchArgs &a, const WorkLayout &w, double *d_plaq, double *d_poly, double *d_corr,
                    hipStream_t st);
void launch_get_flags(const LaunchArgs &a, uint32_t *d_flags, hipStream_t st);

} // namespace su2

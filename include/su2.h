/*
 * su2.h -- C ABI of libsu2.so: SU(2) lattice gauge configurations on one
 * AMD Instinct MI355X (gfx950) by checkerboard heat bath and
 * overrelaxation, with the per-sweep mean plaquette and Polyakov-loop
 * reductions.
 *
 * Method: Cardoso, Cardoso & Bicudo, "Finite temperature lattice QCD with
 * GPUs", Excited QCD 2011 -- Sec. 2.1 (random SU(2) start, heat-bath
 * iterations, mean plaquette at every iteration, single and double
 * precision) and Sec. 2.2 (Polyakov loop, eq. (1); Polyakov-loop
 * correlator, eq. (3)).  The paper leaves the sampler, representation and
 * random numbers unstated; this library uses the Kennedy-Pendleton (1985)
 * sampler for alpha = beta*|V| >= 2 and Creutz (1980) below, Creutz (1987)
 * overrelaxation and Philox4x32-10 (Salmon et al., SC'11).
 *
 * Conventions
 *  - Extents n[4] = (Nx, Ny, Nz, Nt); each must be even and >= 2 and the
 *    volume V = Nx*Ny*Nz*Nt must be below 2^32.
 *  - Site i = x + Nx*(y + Ny*(z + Nz*t)); parity (x+y+z+t) mod 2;
 *    checkerboard index cb = i/2 (a bijection within each parity).
 *  - A link U_mu(x) is the unit quaternion (a0,a1,a2,a3) of the SU(2)
 *    matrix a0 + i(a1 s1 + a2 s2 + a3 s3); mu = 0,1,2,3 = x,y,z,t.
 *  - Link layout in device memory (part of the ABI), plane q = 2*mu + parity,
 *    in 16-byte elements, with S = su2_plane_stride(n, prec):
 *      SU2_F32: float4 (a0,a1,a2,a3) at element q*S + cb;
 *      SU2_F64: double2 (a0,a1) at element (2q)*S + cb and
 *               double2 (a2,a3) at element (2q+1)*S + cb.
 *    S = V/2, except for SU2_F64 with V/2 >= 2^18, where S = V/2 + 16392:
 *    the sub-planes of large FP64 lattices are skewed by 256 KB + 128 B so
 *    that equal cb in different sub-planes do not share L2 sets.  The
 *    S - V/2 elements after each (sub-)plane are never read or written.
 *  - Random numbers: Philox4x32-10 with key (seed lo32, seed hi32) and
 *    counter (site i, mu + 4*kind + 16*lattice_id, sweep, 4*attempt + draw);
 *    kind 0 = hot start, 1 = heat bath.  A heat-bath sweep is therefore a
 *    pure function of (links, beta, seed, sweep, lattice_id).
 *  - Wilson action S = beta * sum_P (1 - (1/2) Tr U_P).
 *
 * Memory and streams
 *  - links and work are DEVICE pointers owned by the caller, 16-byte
 *    aligned, of at least su2_links_bytes() and su2_workspace_bytes()
 *    bytes, not overlapping (SU2_EINVAL otherwise).  The library never
 *    allocates, frees or synchronises.
 *  - stream is a hipStream_t (NULL = the null stream).  Every call only
 *    enqueues work on that stream; results written to device pointers are
 *    valid once that stream reaches them.
 *  - Calls on distinct lattices (distinct links/work) may run concurrently;
 *    calls on one lattice must be ordered by the caller (one stream).
 *
 * Errors
 *  - Every entry point returns SU2_OK (0) or a negative code.  All argument
 *    checks happen before any HIP call, so a rejected call has no effect.
 *    SU2_EHIP reports a failed launch; su2_last_error() then holds the HIP
 *    message (thread-local).
 *  - Device-side anomalies set sticky bits in a flags word in the workspace:
 *    SU2_FLAG_CAP (a sampler hit its attempt cap; the link was kept),
 *    SU2_FLAG_NONFINITE (a staple was not finite; the link was kept) and
 *    SU2_FLAG_SYNC (su2_batch_sweep: a barrier wait gave up).  Both starts
 *    clear it; su2_get_flags() copies it out.
 */
#ifndef SU2_H
#define SU2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SU2_F64 = 0, SU2_F32 = 1 };

enum {
    SU2_OK = 0,
    SU2_EINVAL = -1, /* null lattice/pointer, bad precision, beta < 0 or not finite, bad mu/parity/count */
    SU2_EDIMS = -2,  /* an extent odd or < 2, or V >= 2^32 */
    SU2_EALIGN = -3, /* links, work or an output pointer not suitably aligned */
    SU2_EWORK = -4,  /* work_bytes < su2_workspace_bytes() */
    SU2_EHIP = -5    /* a HIP launch failed */
};

#define SU2_FLAG_CAP 1u
#define SU2_FLAG_NONFINITE 2u
#define SU2_FLAG_SYNC 4u /* su2_batch_sweep: a grid-wide barrier wait gave up */
#define SU2_MAX_ATTEMPTS 4096

typedef struct su2_lattice {
    int32_t n[4];        /* (Nx, Ny, Nz, Nt) */
    int32_t prec;        /* SU2_F64 or SU2_F32 */
    int32_t lattice_id;  /* 0 .. 2^27-1; enters the random-number counter */
    int32_t tile;        /* order in which the threads of a class walk the
                            lattice (performance only, results do not depend
                            on it): 0 = default, W > 0 = (z,t) columns in
                            z-strips of width W (W must divide Nz), -1 =
                            plain checkerboard-index order, -2 = staged:
                            overrelaxation classes walk slabs whose staple
                            neighbourhood each block holds in LDS (where a
                            slab plan fits the lattice and the device's LDS;
                            not in a sweep that takes the plaquette), the
                            other kernels the default strips; -3 = staged
                            as -2 for the heat-bath classes too */
    int32_t tile_y;      /* in strip order (tile >= 0): the update kernels
                            walk each column as tile_y ranges of Ny/tile_y
                            rows (tile_y must divide Ny; 0 = default);
                            performance only */
    void *links;         /* device, >= su2_links_bytes(n, prec) */
    void *work;          /* device, >= su2_workspace_bytes(n, prec) */
    uint64_t work_bytes; /* size of work in bytes */
} su2_lattice_t;

/* Bytes of link storage: 8 planes (F32) or 16 sub-planes (F64) of
 * su2_plane_stride() 16-byte elements each (4 V links of 16 or 32 bytes,
 * plus the skew of large FP64 lattices).  Returns 0 if the extents or
 * precision are invalid. */
uint64_t su2_links_bytes(const int32_t n[4], int32_t prec);

/* S of the link layout: 16-byte elements from the start of one plane (F32)
 * or sub-plane (F64) to the next -- V/2, or V/2 + 16392 for SU2_F64 when
 * V/2 >= 2^18.  Returns 0 if the extents or precision are invalid. */
uint64_t su2_plane_stride(const int32_t n[4], int32_t prec);

/* Bytes of workspace: flags word, reduction partials, Polyakov-loop field.
 * Returns 0 if the extents or precision are invalid. */
uint64_t su2_workspace_bytes(const int32_t n[4], int32_t prec);

/* Cold start: every link = identity (Sec. 2.1 "initialization").  Clears
 * the flags word. */
int su2_init_cold(const su2_lattice_t *lat, void *stream);

/* Hot start (Sec. 2.1 "random SU(2) matrix initialization"): every link
 * Haar-random, from four Box-Muller normals normalised onto the unit
 * 3-sphere, computed in FP64 (F32 lattices store the rounded value,
 * renormalised in FP32).  Clears the flags word. */
int su2_init_hot(const su2_lattice_t *lat, uint64_t seed, void *stream);

/* One heat-bath sweep (Sec. 2.1 "heat bath method"): for mu = 0..3, for
 * parity 0 then 1, every link U_mu(x) of that class is replaced by a draw
 * from exp((beta/2) Tr(U V)) dU, V the sum of its six staples.  Eight
 * ordered launches on stream.  sweep is the random-number sweep index. */
int su2_heatbath_sweep(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t sweep,
                       void *stream);

/* One checkerboard class (mu, parity) of su2_heatbath_sweep. */
int su2_heatbath_halfsweep(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t sweep,
                           int32_t mu, int32_t parity, void *stream);

/* n_sweeps overrelaxation sweeps (same class order as the heat bath):
 * U -> Vhat^dagger U^dagger Vhat^dagger, Vhat = V/|V|; links with V = 0 are
 * kept.  Preserves the action, uses no random numbers.  F32 lattices are
 * renormalised on every write.  n_sweeps >= 0. */
int su2_overrelax(const su2_lattice_t *lat, int32_t n_sweeps, void *stream);

/* One checkerboard class (mu, parity) of su2_overrelax. */
int su2_overrelax_halfsweep(const su2_lattice_t *lat, int32_t mu, int32_t parity, void *stream);

/* Mean plaquette (Sec. 2.1 "mean average plaquette"): d_out (device,
 * 8-byte aligned, 7 doubles) receives [0] the average of (1/2) Tr U_P over
 * all 6V plaquettes and [1..6] the per-plane averages for the planes
 * (01, 02, 03, 12, 13, 23).  Half traces and all sums in FP64; the
 * reduction order is fixed, so the result is bitwise reproducible. */
int su2_plaquette(const su2_lattice_t *lat, double *d_out, void *stream);

/* su2_plaquette for callers that cannot allocate device memory or hand the
 * library a workspace (code under stream capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and the same d_out,
 * bitwise the same result, but the block partials go to a static 8 MiB
 * array of the library on the current device instead of lat->work, which
 * is not used (work and work_bytes may be NULL and 0).  No allocation, no
 * free.  Limit: V/2 <= 256 x 174762 = 44,739,072 sites per parity (96^4 fits);
 * larger lattices give SU2_EDIMS.  The current device must be the one that
 * holds the links, d_out and the stream.  Every call on one GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (different streams
 * or threads) race; calls ordered on one stream do not.  Errors: as
 * su2_plaquette except for the workspace; SU2_EHIP if the array's address
 * cannot be obtained. */
int su2_plaquette_noalloc(const su2_lattice_t *lat, double *d_out, void *stream);

/* Polyakov loop (Sec. 2.2, eq. (1)) L(x) = (1/2) Tr prod_{t=0}^{Nt-1}
 * U_t(x,t) at every spatial site.  d_out (device, 2 doubles) receives
 * [0] the spatial mean of L and [1] the spatial mean of |L|.  If d_corr is
 * not NULL it receives (device, R = min(Nx,Ny,Nz)/2 doubles) the on-axis
 * correlator of eq. (3), C(r) = (1/(3 Vs)) sum_x sum_i L(x) L(x + r e_i),
 * r = 1..R.  FP64 sums, fixed reduction order. */
int su2_polyakov(const su2_lattice_t *lat, double *d_out, double *d_corr, void *stream);

/* A heat-bath sweep (as su2_heatbath_sweep) that also leaves the mean
 * plaquette of the configuration it produces in d_plaq (device, 7 doubles,
 * as su2_plaquette's d_out; Sec. 2.1 measures it after every iteration).
 * No extra pass over the lattice: in class (mu, odd), mu >= 1, every link of
 * the plaquettes of planes (nu, mu), nu < mu, is final, and each such
 * plaquette holds exactly one odd mu-link, so the classes (1,odd), (2,odd),
 * (3,odd) take the half traces of their new links with the staple products
 * they already formed (FP64 from the half trace on; in FP32 the two
 * plaquettes of one plane through a link share one half trace of the summed
 * staple products).  The links are bitwise those of su2_heatbath_sweep; the
 * plaquette agrees with su2_plaquette to the summation order (FP64) or to
 * the rounding of FP32 products (FP32).  Uses the plaquette partials of the
 * lattice's workspace.  Errors: as su2_heatbath_sweep, plus SU2_EINVAL for a
 * NULL d_plaq and SU2_EALIGN for one not 8-byte aligned. */
int su2_heatbath_sweep_measured(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t sweep,
                                double *d_plaq, void *stream);

/* su2_overrelax with the mean plaquette of the final configuration left in
 * d_plaq, measured by the last sweep as in su2_heatbath_sweep_measured
 * (n_sweeps = 0: su2_plaquette of the current configuration).  Errors: as
 * su2_overrelax, plus those of d_plaq as in su2_heatbath_sweep_measured. */
int su2_overrelax_measured(const su2_lattice_t *lat, int32_t n_sweeps, double *d_plaq, void *stream);

/* Both measurements of a configuration in one pass over the links (Sec. 2.1
 * mean plaquette; Sec. 2.2 eqs. (1), (3)): d_plaq (device, 7 doubles) as
 * su2_plaquette's d_out, d_poly (device, 2 doubles) as su2_polyakov's d_out,
 * d_corr (optional) as su2_polyakov's.  Same quantities, FP64 sums in a
 * different fixed order (so the values agree with the separate calls to a
 * few ulp, not bitwise); each link is read once as its own site's link and
 * the temporal links once for both the plaquettes and the Polyakov lines. */
int su2_measure(const su2_lattice_t *lat, double *d_plaq, double *d_poly, double *d_corr, void *stream);

/* ---- Batches: many independent lattices per launch (a temperature scan) ----
 * A batch is count lattice descriptors of one precision, each with its own
 * extents, beta, lattice_id (distinct ids give independent random streams;
 * a lattice gives bit-identical links whether it is updated alone or in a
 * batch) and tile.  su2_batch_fill writes a table into HOST memory; the
 * caller copies it to device memory (8-byte aligned) and passes that copy as
 * d_table together with the same descriptors.  The table holds the link and
 * workspace pointers and betas: refill it when any of them changes. */

/* Bytes of the batch table for count lattices (0 if count < 1 or > 4096). */
uint64_t su2_batch_table_bytes(int32_t count);

/* Fill host_table for lats[0..count) with betas[0..count) (host arrays).
 * Checks every descriptor as the single-lattice calls do, one precision;
 * SU2_EINVAL if two lattices share or overlap links or work or repeat a
 * lattice_id (the batched calls check the same). */
int su2_batch_fill(const su2_lattice_t *lats, const double *betas, int32_t count, void *host_table,
                   uint64_t table_bytes);

/* One heat-bath sweep of every lattice of the batch (the per-lattice sweep of
 * su2_heatbath_sweep with that lattice's beta): eight launches, each updating
 * one class (mu, parity) of all lattices.  The sweep index is *d_sweep
 * (device, read when the launches run) if d_sweep is not NULL, else sweep;
 * with d_sweep and su2_sweep_advance a captured graph can be replayed. */
int su2_batch_heatbath_sweep(const su2_lattice_t *lats, int32_t count, const void *d_table, uint64_t seed,
                             uint32_t sweep, const uint32_t *d_sweep, void *stream);

/* n_sweeps overrelaxation sweeps of every lattice of the batch.  Per class
 * (mu, parity): one launch for the lattices of fewer than 2^20 sites, and
 * for each larger lattice the class launch of su2_overrelax (whose residency
 * cap the batched kernel cannot take), all on `stream`; every lattice's
 * links are bitwise those of su2_overrelax on it alone. */
int su2_batch_overrelax(const su2_lattice_t *lats, int32_t count, const void *d_table, int32_t n_sweeps,
                        void *stream);

/* The same as su2_batch_heatbath_sweep followed by su2_batch_overrelax with
 * n_or sweeps (Sec. 2.1 heat bath, then overrelaxation), bit for bit, in ONE
 * persistent launch: its grid is at most the blocks the device keeps
 * resident at once, each block takes the batched launches' blocks in turn,
 * and all blocks meet at a grid-wide barrier between classes (8 * (1 + n_or)
 * classes).  d_sync: device, one uint32, 4-byte aligned, the barrier's
 * counter: its low 31 bits must be 0 before the first call (zero it once)
 * and every call leaves them 0; bit 31 is the barrier's phase, flipped by
 * each barrier.  Calls that share a d_sync must not overlap, and nothing else should run
 * on the device meanwhile: the barrier needs every block of the grid
 * resident.  A barrier wait gives up after spin_limit polls (0: the default,
 * a few tenths of a second, against a normal wait of tens of microseconds) and sets
 * SU2_FLAG_SYNC in every lattice's flags word; the call still ends, with
 * unreliable links.  The sweep index is *d_sweep if d_sweep is not NULL (so a
 * captured graph of this one launch and su2_sweep_advance can be replayed),
 * else sweep.  Errors: those of su2_batch_heatbath_sweep; SU2_EINVAL for n_or
 * outside [0, 64] or a NULL d_sync; SU2_EALIGN for a misaligned d_sync;
 * SU2_EHIP if the kernel cannot be resident on the device. */
int su2_batch_sweep(const su2_lattice_t *lats, int32_t count, const void *d_table, uint64_t seed, uint32_t sweep,
                    const uint32_t *d_sweep, int32_t n_or, uint32_t *d_sync, uint32_t spin_limit, void *stream);

/* Polyakov loop and on-axis correlator (Sec. 2.2, eqs. (1) and (3)) of every
 * lattice of the batch, each exactly as su2_polyakov computes it (the same
 * block partials and summation order, so bitwise the same values), in three
 * launches for the whole batch.  d_poly: device, 2*count doubles, [2j] the
 * mean L and [2j+1] the mean |L| of lattice j.  d_corr: device,
 * count*corr_stride doubles, or NULL for no correlator; row j holds C(r),
 * r = 1..min(Nx,Ny,Nz)/2 of lattice j, and its entries beyond are left
 * untouched; corr_stride must be >= the largest min(Nx,Ny,Nz)/2 of the
 * batch.  Uses each lattice's workspace; lats and d_table as for the other
 * batched calls (the table of su2_batch_fill for these descriptors).
 * Errors: those of the descriptors as in su2_batch_fill; SU2_EINVAL for a
 * NULL or misaligned d_table, a NULL d_poly or a corr_stride too small;
 * SU2_EALIGN for d_poly or d_corr not 8-byte aligned. */
int su2_batch_polyakov(const su2_lattice_t *lats, int32_t count, const void *d_table, double *d_poly,
                       double *d_corr, int32_t corr_stride, void *stream);

/* *d_sweep += 1 on the device (d_sweep: device, one uint32). */
int su2_sweep_advance(uint32_t *d_sweep, void *stream);

/* ---- Learned block proposal --------------------------------------------
 * An exact Metropolis-Hastings move for the temporal link T(e) of a spatial
 * site e of every time slice, with the temporal links of e's six spatial
 * neighbours integrated out: the marginal of T(e) is prod_o Z(beta|V_o|),
 * Z(a) = 2 I1(a)/a, V_o the staple of neighbour o's temporal link.  T(e) is
 * proposed from q(T) ~ exp((1/2)Tr(T M)), M = sum_o c_o S_o, where S_o is
 * V_o without its term through e carried to e and c_o = beta r(a0) /
 * sqrt(|S_o|^2+1) exp(y_o) (r = I2/I1, a0 = beta sqrt(|S_o|^2+1)), y the
 * six outputs of the proposal network at e; after the accept/reject every
 * neighbour's temporal link is redrawn by heat bath.  Sites of one parity
 * and colour (x + 2y + 3z) mod 8 are updated together (they are >= 4
 * apart).  Random numbers: kind 2, counter (site, 3 + 8 + 16 lattice_id,
 * 16 step + 8 parity + colour, 4 attempt + draw), draw 3 the accept uniform.
 * Requires Nx, Ny, Nz multiples of 8.
 *
 * The network (62502 FP32 parameters, in the order given below) maps
 * gauge-invariant features --
 * the spatial plaquettes of slices t and t+1, no temporal link -- through
 * three periodic 3x3x3 convolutions (8->32->32->32, tanh; BF16 MFMA with
 * FP32 accumulation) and a linear head to y[site][6].  Parameter order:
 * W1[27][8][32] b1[32] W2[27][32][32] b2[32] W3[27][32][32] b3[32] V[6][32]
 * bv[6]; tap = (dz+1)*9 + (dy+1)*3 + (dx+1). */

#define SU2_LP_NPARAM 62502

int32_t su2_lp_param_count(void);

/* Bytes of the network workspace (device) for extents n; 0 if invalid. */
uint64_t su2_lp_workspace_bytes(const int32_t n[4]);

/* Network outputs for the lattice's current links: d_y (device, V*6 floats,
 * index site*6 + direction, directions -x,+x,-y,+y,-z,+z). */
int su2_lp_forward(const su2_lattice_t *lat, const float *d_params, void *d_lpwork, uint64_t lpwork_bytes,
                   float *d_y, void *stream);

/* Maximum-likelihood training signal on the lattice's current links: the
 * loss -mean_e log q(T(e) | M(e)) over every site and slice into d_loss
 * (device, one double) and its gradient into d_grad (device, param_count
 * floats, overwritten). */
int su2_lp_loss_grad(const su2_lattice_t *lat, double beta, const float *d_params, void *d_lpwork,
                     uint64_t lpwork_bytes, float *d_grad, double *d_loss, void *stream);

/* One Adam step on count parameters (step counts from 1). */
int su2_lp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t count, int32_t step, float lr,
                float beta1, float beta2, float eps, void *stream);

/* Block moves of one class (parity, colour) with network outputs d_y;
 * *d_accepted (device) is incremented once per accepted move. */
int su2_lp_move(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t step, int32_t parity, int32_t colour,
                const float *d_y, uint32_t *d_accepted, void *stream);

/* All 16 classes (parity 0 then 1, colours 0..7): one learned sweep. */
int su2_lp_sweep(const su2_lattice_t *lat, double beta, uint64_t seed, uint32_t step, const float *d_y,
                 uint32_t *d_accepted, void *stream);

/* Copy the sticky flags word to d_flags (device, one uint32). */
int su2_get_flags(const su2_lattice_t *lat, uint32_t *d_flags, void *stream);

/* Message for an error code (static string). */
const char *su2_strerror(int code);

/* Detail of the last error on the calling thread (static per thread). */
const char *su2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif

/*
 * su2_oracle.h -- plain FP64 CPU reference for SU(2) lattice gauge
 * configuration generation by checkerboard heat bath and overrelaxation,
 * with the mean plaquette and Polyakov-loop observables.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the test suite, the
 * smoke check and the benchmark's CPU baseline can compare the GPU library
 * against an independent, obviously correct implementation.  Nothing in the
 * product path links, loads or calls it.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * Method: Cardoso, Cardoso & Bicudo, "Finite temperature lattice QCD with
 * GPUs" (Excited QCD 2011): Sec. 2.1 (random SU(2) start, heat-bath
 * iterations, mean plaquette per iteration), Sec. 2.2 eq. (1) (Polyakov loop)
 * and eq. (3) (Polyakov-loop correlator).  The heat-bath samplers are
 * Creutz, Phys. Rev. D 21 (1980) 2308 and Kennedy & Pendleton, Phys. Lett.
 * B 156 (1985) 393; overrelaxation is Creutz, Phys. Rev. D 36 (1987) 515;
 * the random numbers are Philox4x32-10 of Salmon, Moraes, Dror & Shaw,
 * SC'11 (2011).  The paper itself leaves the representation, staple
 * orientation, update order and random-number layout unstated; the readings
 * taken are listed with each function in su2_oracle.c.
 *
 * Conventions shared by every function here:
 *  - extents n[4] = (Nx, Ny, Nz, Nt), each even and >= 2;
 *  - linear site i = x + Nx*(y + Ny*(z + Nz*t)), parity (x+y+z+t) mod 2;
 *  - canonical host layout U[i][mu][4] in double, mu = 0,1,2,3 = x,y,z,t;
 *  - a link is the unit quaternion (a0,a1,a2,a3) for the SU(2) matrix
 *    a0*1 + i*(a1*s1 + a2*s2 + a3*s3) (s_k the Pauli matrices);
 *  - Philox counter (c0,c1,c2,c3) = (site, mu + 4*kind + 16*lattice_id,
 *    sweep, 4*attempt + draw), key = (seed low 32 bits, seed high 32 bits);
 *    kind 0 = hot start, 1 = heat bath, 3 = random gauge transformation.
 *
 * Returned flag bits: 1 = rejection-loop attempt cap hit (link kept),
 *                     2 = non-finite staple (link kept).
 */
#ifndef SU2_ORACLE_H
#define SU2_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_FLAG_CAP 1u
#define OR_FLAG_NONFINITE 2u
#define OR_MAX_ATTEMPTS 4096

/* Random numbers. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u01_f64(uint32_t r_even, uint32_t r_odd);
float or_u01_f32(uint32_t r_even);

/* Quaternion algebra. */
void or_qmul(const double a[4], const double b[4], double out[4]);
void or_qdag(const double a[4], double out[4]);

/* Lattice geometry. */
int64_t or_volume(const int n[4]);
int64_t or_neighbor(const int n[4], int64_t site, int dir, int step);
int or_parity(const int n[4], int64_t site);

/* Staple sum of link (site, mu). */
void or_staple(const int n[4], const double *U, int64_t site, int mu, double V[4]);

/* Starts. */
void or_init_cold(const int n[4], double *U);
void or_init_hot(const int n[4], double *U, uint64_t seed, uint32_t lattice_id);

/* Updates; return the OR of the flag bits raised. */
uint32_t or_heatbath_halfsweep(const int n[4], double *U, double beta, uint64_t seed,
                               uint32_t sweep, int mu, int parity, uint32_t lattice_id);
uint32_t or_heatbath_sweep(const int n[4], double *U, double beta, uint64_t seed,
                           uint32_t sweep, uint32_t lattice_id);
/* The heat-bath half-sweep with single-precision links: U must hold values
 * representable in single precision and receives single-precision results;
 * the precisions of each step are listed in su2_oracle.c. */
uint32_t or_heatbath_halfsweep_f32(const int n[4], double *U, double beta, uint64_t seed,
                                   uint32_t sweep, int mu, int parity, uint32_t lattice_id);
uint32_t or_overrelax_halfsweep(const int n[4], double *U, int mu, int parity);
uint32_t or_overrelax_sweep(const int n[4], double *U);

/* Observables. */
double or_plaquette(const int n[4], const double *U, double planes[6]);
void or_polyakov_field(const int n[4], const double *U, double *L);
void or_polyakov(const int n[4], const double *U, double out[2]);
int or_polyakov_corr(const int n[4], const double *U, double *C);

/* Random gauge transformation U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger. */
void or_gauge_transform(const int n[4], double *U, uint64_t seed, uint32_t lattice_id);

/* Learned block proposal (reference): Bessel functions, the block pieces
 * S_o, the marginal log density of a block centre, the proposal's effective
 * staple, and the move itself (see su2_oracle.c). */
double or_bessel_ive(int n, double x);
double or_log_z(double a);
double or_bessel_ratio(double a);
int or_block_colour(int x, int y, int z);
void or_block_piece(const int n[4], const double *U, int64_t e, int dir, double S[4]);
double or_block_log_marginal(const int n[4], const double *U, int64_t e, double beta, const double T[4]);
void or_block_proposal(const int n[4], const double *U, int64_t e, double beta, const double y[6],
                       double M[4]);
uint32_t or_block_move(const int n[4], double *U, double beta, uint64_t seed, uint32_t step, int p, int k,
                       const double *y, uint32_t lattice_id, int64_t *accepted);
void or_block_pieces_all(const int n[4], const double *U, double *S);
uint32_t or_block_sweep(const int n[4], double *U, double beta, uint64_t seed, uint32_t step, const double *y,
                        uint32_t lattice_id, int64_t *accepted);

/* Number of OpenMP threads the oracle's parallel loops use. */
int or_num_threads(void);

#ifdef __cplusplus
}
#endif

#endif

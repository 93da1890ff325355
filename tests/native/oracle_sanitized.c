/*
 * Drives every entry point of the CPU oracle (oracle/su2_oracle.c) on small
 * lattices, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (run by tests/test_oracle_sanitized.py, host only).  Prints the results
 * it computes, one "name value" per line, so that the test can also compare
 * them with the regular build of the oracle.
 */
#include "su2_oracle.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static double *alloc_links(const int n[4])
{
    const int64_t v = or_volume(n);
    double *U = malloc((size_t)v * 16 * sizeof(double));
    if (!U) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return U;
}

static void chain(const char *tag, const int n[4], uint64_t seed, double beta)
{
    double *U = alloc_links(n);
    uint32_t flags = 0;
    or_init_hot(n, U, seed, 3);
    for (uint32_t s = 0; s < 3; ++s) {
        flags |= or_heatbath_sweep(n, U, beta, seed, s, 3);
        flags |= or_overrelax_sweep(n, U);
    }
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
            flags |= or_heatbath_halfsweep(n, U, beta, seed, 7, mu, p, 3);
            flags |= or_overrelax_halfsweep(n, U, mu, p);
        }
    double planes[6];
    const double P = or_plaquette(n, U, planes);
    double L[2];
    or_polyakov(n, U, L);
    const int nmin = n[0] < n[1] ? (n[0] < n[2] ? n[0] : n[2]) : (n[1] < n[2] ? n[1] : n[2]);
    double *C = calloc((size_t)(nmin / 2 + 1), sizeof(double));
    const int rmax = or_polyakov_corr(n, U, C);
    double *Lf = malloc((size_t)(or_volume(n) / n[3]) * sizeof(double));
    or_polyakov_field(n, U, Lf);
    or_gauge_transform(n, U, seed + 1, 3);
    double planes_g[6];
    const double Pg = or_plaquette(n, U, planes_g);
    printf("%s_flags %u\n", tag, flags);
    printf("%s_plaquette %.17g\n", tag, P);
    printf("%s_plaquette_gauge %.17g\n", tag, Pg);
    printf("%s_plane5 %.17g\n", tag, planes[5]);
    printf("%s_poly_mean %.17g\n", tag, L[0]);
    printf("%s_poly_abs %.17g\n", tag, L[1]);
    printf("%s_L0 %.17g\n", tag, Lf[0]);
    printf("%s_corr_last %.17g\n", tag, rmax > 0 ? C[rmax - 1] : 0.0);
    free(Lf);
    free(C);
    free(U);
}

/* The single-precision heat-bath step wants links representable in single
 * precision: round a hot start. */
static void chain_f32(const char *tag, const int n[4], uint64_t seed, double beta)
{
    double *U = alloc_links(n);
    uint32_t flags = 0;
    or_init_hot(n, U, seed, 0);
    const int64_t m = or_volume(n) * 16;
    for (int64_t k = 0; k < m; ++k)
        U[k] = (double)(float)U[k];
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            flags |= or_heatbath_halfsweep_f32(n, U, beta, seed, 1, mu, p, 0);
    double planes[6];
    printf("%s_flags %u\n", tag, flags);
    printf("%s_plaquette %.17g\n", tag, or_plaquette(n, U, planes));
    free(U);
}

static void block(const int n[4], uint64_t seed, double beta)
{
    double *U = alloc_links(n);
    const int64_t v = or_volume(n);
    double *y = malloc((size_t)v * 6 * sizeof(double));
    double *S = malloc((size_t)v * 6 * 4 * sizeof(double));
    for (int64_t k = 0; k < v * 6; ++k)
        y[k] = 0.01 * (double)(k % 7) - 0.03;
    or_init_hot(n, U, seed, 0);
    for (uint32_t s = 0; s < 2; ++s)
        or_heatbath_sweep(n, U, beta, seed, s, 0);
    double Sx[4], M[4];
    or_block_piece(n, U, 5, 2, Sx);
    or_block_proposal(n, U, 5, beta, y + 30, M);
    const double T[4] = {0.5, 0.5, 0.5, 0.5};
    const double lm = or_block_log_marginal(n, U, 5, beta, T);
    or_block_pieces_all(n, U, S);
    int64_t acc = 0;
    uint32_t flags = or_block_move(n, U, beta, seed, 0, 1, 3, y, 0, &acc);
    flags |= or_block_sweep(n, U, beta, seed, 1, y, 0, &acc);
    double planes[6];
    printf("block_flags %u\n", flags);
    printf("block_accepted %lld\n", (long long)acc);
    printf("block_piece %.17g\n", Sx[0]);
    printf("block_proposal %.17g\n", M[3]);
    printf("block_log_marginal %.17g\n", lm);
    printf("block_pieces_all %.17g\n", S[4 * 6 * 9 + 2]);
    printf("block_plaquette %.17g\n", or_plaquette(n, U, planes));
    printf("bessel %.17g %.17g %.17g\n", or_bessel_ive(1, 3.5), or_log_z(0.25), or_bessel_ratio(12.0));
    printf("colour %d\n", or_block_colour(3, 5, 7));
    free(S);
    free(y);
    free(U);
}

int main(void)
{
    const uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    printf("philox %u %u %u %u\n", r[0], r[1], r[2], r[3]);
    printf("u01 %.17g %.9g\n", or_u01_f64(0xffffffffu, 0xffffffffu), (double)or_u01_f32(0u));
    const double a[4] = {0.5, 0.5, -0.5, 0.5}, b[4] = {0.1, 0.7, 0.1, 0.7};
    double q[4], d[4];
    or_qmul(a, b, q);
    or_qdag(q, d);
    printf("qmul %.17g %.17g\n", q[0], d[3]);
    const int ragged[4] = {6, 4, 10, 8}, tiny[4] = {2, 2, 2, 2}, odd_t[4] = {4, 6, 2, 12};
    printf("neighbor %lld parity %d\n", (long long)or_neighbor(ragged, 0, 3, -1), or_parity(ragged, 7));
    double V[4];
    double *U = alloc_links(ragged);
    or_init_cold(ragged, U);
    or_staple(ragged, U, 11, 2, V);
    printf("cold_staple %.17g\n", V[0]);
    free(U);
    chain("ragged", ragged, 1234, 2.3);
    chain("tiny", tiny, 77, 0.4);
    chain("long_t", odd_t, 5, 6.0);
    chain_f32("f32", ragged, 99, 2.3);
    const int blk[4] = {8, 8, 8, 4};
    block(blk, 31, 2.3);
    return 0;
}

/*
 * su2_oracle.c -- plain FP64 CPU reference (TEST INFRASTRUCTURE ONLY; see
 * su2_oracle.h).  Deliberately simple: natural site order, coordinates
 * recomputed for every neighbour, no blocking, no fusion.  The only
 * parallelism is an OpenMP loop over the sites of one checkerboard class,
 * whose links are mutually independent, so the result does not depend on
 * the thread count.
 *
 * Pins (what fixes each function other than itself):
 *  - or_philox4x32_10: raw outputs against PyTorch's header-only host Philox
 *    engine (a separately written implementation of the same published
 *    generator), plus uniformity statistics;
 *  - or_u01_f64 / or_u01_f32: exhaustive edge values (closed form);
 *  - or_qmul / or_qdag: numpy complex 2x2 matrix products;
 *  - or_staple: brute-force change of the total Wilson action;
 *  - or_init_hot: Haar moments and the Haar density of a0 (KS);
 *  - heat bath: conditional law of one link (KS against the exact density,
 *    mean against a ratio of Bessel functions), probability-integral
 *    transform at equilibrium, strong- and weak-coupling limits;
 *  - heat bath with single-precision links: the same exact law (KS) and
 *    agreement with the double-precision step except where a decision
 *    flips between 23-bit and 52-bit arithmetic;
 *  - overrelaxation: action conservation and involution;
 *  - observables: cold start = 1, gauge invariance, Z2 centre symmetry.
 */
#include "su2_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double OR_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, Salmon et al. SC'11 (2011): ten rounds of two 32x32->64    */
/* multiplications with the round multipliers below, the key bumped by the  */
/* Weyl constants between rounds.                                            */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t next[4];
        next[0] = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        next[1] = (uint32_t)p1;
        next[2] = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        next[3] = (uint32_t)p0;
        memcpy(c, next, sizeof c);
    }
    memcpy(out, c, sizeof c);
}

/* Uniform in the open interval (0,1): the top 52 bits of the 64-bit word
 * (r_even, r_odd) plus one half, times 2^-52. */
double or_u01_f64(uint32_t r_even, uint32_t r_odd)
{
    uint64_t w = ((uint64_t)r_even << 32) | (uint64_t)r_odd;
    uint64_t m = w >> 12;
    return ((double)m + 0.5) * 0x1p-52;
}

/* Single-precision uniform from the top 23 bits of r_even, so that it is the
 * FP64 uniform of the same pair rounded to 23 bits. */
float or_u01_f32(uint32_t r_even)
{
    uint32_t m = r_even >> 9;
    return ((float)m + 0.5f) * 0x1p-23f;
}

/* Two FP64 uniforms from one Philox call at counter (site, c1, c2, c3). */
static void draw2(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                  double *ua, double *ub)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    *ua = or_u01_f64(r[0], r[1]);
    *ub = or_u01_f64(r[2], r[3]);
}

/* ------------------------------------------------------------------------ */
/* Quaternion form of SU(2): U = a0 + i a.sigma, so that                      */
/* (a0,a)(b0,b) = (a0 b0 - a.b, a0 b + b0 a - a x b), U^dagger = (a0, -a),  */
/* and half the trace of U is a0.                                            */
/* ------------------------------------------------------------------------ */
void or_qmul(const double a[4], const double b[4], double out[4])
{
    double r0 = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    double r1 = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    double r2 = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    double r3 = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
    out[0] = r0;
    out[1] = r1;
    out[2] = r2;
    out[3] = r3;
}

void or_qdag(const double a[4], double out[4])
{
    out[0] = a[0];
    out[1] = -a[1];
    out[2] = -a[2];
    out[3] = -a[3];
}

/* ------------------------------------------------------------------------ */
/* Geometry: periodic 4-D lattice, x fastest.                                */
/* ------------------------------------------------------------------------ */
int64_t or_volume(const int n[4])
{
    return (int64_t)n[0] * n[1] * n[2] * n[3];
}

static void coords(const int n[4], int64_t site, int c[4])
{
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(site % n[d]);
        site /= n[d];
    }
}

static int64_t site_of(const int n[4], const int c[4])
{
    return c[0] + (int64_t)n[0] * (c[1] + (int64_t)n[1] * (c[2] + (int64_t)n[2] * c[3]));
}

int64_t or_neighbor(const int n[4], int64_t site, int dir, int step)
{
    int c[4];
    coords(n, site, c);
    c[dir] = ((c[dir] + step) % n[dir] + n[dir]) % n[dir];
    return site_of(n, c);
}

int or_parity(const int n[4], int64_t site)
{
    int c[4];
    coords(n, site, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static const double *link(const double *U, int64_t site, int mu)
{
    return U + (site * 4 + mu) * 4;
}

/* ------------------------------------------------------------------------ */
/* Staple sum for link U_mu(x): the Wilson action of the plaquettes holding  */
/* this link is -(beta/2) Tr(U_mu(x) V) + const with                        */
/*   V = sum_{nu != mu} [ U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+                  */
/*                      + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu) ].         */
/* ------------------------------------------------------------------------ */
void or_staple(const int n[4], const double *U, int64_t site, int mu, double V[4])
{
    V[0] = V[1] = V[2] = V[3] = 0.0;
    int64_t xp = or_neighbor(n, site, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu)
            continue;
        double t1[4], t2[4], d[4], s[4];
        /* upper: U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
        int64_t xn = or_neighbor(n, site, nu, +1);
        or_qdag(link(U, xn, mu), d);
        or_qmul(link(U, xp, nu), d, t1);
        or_qdag(link(U, site, nu), d);
        or_qmul(t1, d, s);
        for (int k = 0; k < 4; ++k)
            V[k] += s[k];
        /* lower: U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu) */
        int64_t xm = or_neighbor(n, site, nu, -1);
        int64_t xpm = or_neighbor(n, xp, nu, -1);
        double d2[4];
        or_qdag(link(U, xpm, nu), d);
        or_qdag(link(U, xm, mu), d2);
        or_qmul(d, d2, t2);
        or_qmul(t2, link(U, xm, nu), s);
        for (int k = 0; k < 4; ++k)
            V[k] += s[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Starts (Sec. 2.1: "random SU(2) matrix initialization").                  */
/* ------------------------------------------------------------------------ */
void or_init_cold(const int n[4], double *U)
{
    int64_t nl = or_volume(n) * 4;
    for (int64_t l = 0; l < nl; ++l) {
        U[4 * l + 0] = 1.0;
        U[4 * l + 1] = 0.0;
        U[4 * l + 2] = 0.0;
        U[4 * l + 3] = 0.0;
    }
}

/* A Haar-random SU(2) element: four independent standard normals by the
 * Box-Muller transform, normalised onto the unit 3-sphere. */
static void haar_from_counter(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, double q[4])
{
    double u1, u2, u3, u4;
    draw2(seed, c0, c1, c2, 0u, &u1, &u2);
    draw2(seed, c0, c1, c2, 1u, &u3, &u4);
    double r1 = sqrt(-2.0 * log(u1));
    double r2 = sqrt(-2.0 * log(u3));
    double g[4] = {r1 * cos(2.0 * OR_PI * u2), r1 * sin(2.0 * OR_PI * u2),
                   r2 * cos(2.0 * OR_PI * u4), r2 * sin(2.0 * OR_PI * u4)};
    double norm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3]);
    for (int k = 0; k < 4; ++k)
        q[k] = g[k] / norm;
}

void or_init_hot(const int n[4], double *U, uint64_t seed, uint32_t lattice_id)
{
    int64_t vol = or_volume(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < vol; ++i)
        for (int mu = 0; mu < 4; ++mu)
            haar_from_counter(seed, (uint32_t)i, (uint32_t)(mu + 4 * 0 + 16 * lattice_id), 0u,
                              U + (i * 4 + mu) * 4);
}

/* ------------------------------------------------------------------------ */
/* Heat bath for one link.  The link's conditional law is proportional to    */
/* exp((beta/2) Tr(U V)) dU.  With k = |V| and Vhat = V/k, W = U Vhat has    */
/* density ~ exp(alpha w0) dHaar(W), alpha = beta k, i.e. w0 has density     */
/* ~ sqrt(1 - w0^2) exp(alpha w0) on [-1,1] and (w1,w2,w3) is isotropic with */
/* length sqrt(1 - w0^2).  Then U = W Vhat^dagger.                           */
/*   alpha >= 2: Kennedy-Pendleton; alpha < 2: Creutz.                       */
/* ------------------------------------------------------------------------ */
static uint32_t heatbath_link(double Ulink[4], const double V[4], double beta, uint64_t seed,
                              uint32_t site, uint32_t c1, uint32_t sweep)
{
    double k = sqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2] + V[3] * V[3]);
    if (!isfinite(k))
        return OR_FLAG_NONFINITE;
    double Vhat[4] = {1.0, 0.0, 0.0, 0.0};
    if (k > 0.0)
        for (int j = 0; j < 4; ++j)
            Vhat[j] = V[j] / k;
    double alpha = beta * k;

    double x0 = 0.0, xlen = 0.0;
    int accepted = 0;
    for (uint32_t a = 0; a < OR_MAX_ATTEMPTS && !accepted; ++a) {
        if (alpha >= 2.0) {
            /* Kennedy-Pendleton: lambda^2 from two exponentials, accept with
             * probability sqrt(1 - lambda^2), x0 = 1 - 2 lambda^2. */
            double u1, u2, u3, u4;
            draw2(seed, site, c1, sweep, 4u * a + 0u, &u1, &u2);
            draw2(seed, site, c1, sweep, 4u * a + 1u, &u3, &u4);
            double c = cos(2.0 * OR_PI * u2);
            double lam2 = -(log(u1) + c * c * log(u3)) / (2.0 * alpha);
            if (lam2 <= 1.0 && u4 * u4 <= 1.0 - lam2) {
                x0 = 1.0 - 2.0 * lam2;
                xlen = 2.0 * sqrt(lam2 * (1.0 - lam2));
                accepted = 1;
            }
        } else {
            /* Creutz: x0 from exp(alpha x0) on [-1,1] by inversion, accept
             * with probability sqrt(1 - x0^2). */
            double u1, u2;
            draw2(seed, site, c1, sweep, 4u * a + 0u, &u1, &u2);
            double t;
            if (alpha < 1e-8) {
                t = 2.0 * u1 - 1.0;
            } else {
                double e = exp(-2.0 * alpha);
                t = 1.0 + log(e + u1 * (1.0 - e)) / alpha;
            }
            if (u2 * u2 <= 1.0 - t * t) {
                x0 = t;
                double s = 1.0 - t * t;
                xlen = sqrt(s > 0.0 ? s : 0.0);
                accepted = 1;
            }
        }
    }
    if (!accepted)
        return OR_FLAG_CAP;

    /* Direction of (w1,w2,w3): uniform on the unit 2-sphere. */
    double u5, u6;
    draw2(seed, site, c1, sweep, 2u, &u5, &u6);
    double cth = 2.0 * u5 - 1.0;
    double s = 1.0 - cth * cth;
    double sth = sqrt(s > 0.0 ? s : 0.0);
    double phi = 2.0 * OR_PI * u6;
    double W[4] = {x0, xlen * sth * cos(phi), xlen * sth * sin(phi), xlen * cth};

    double Vd[4];
    or_qdag(Vhat, Vd);
    or_qmul(W, Vd, Ulink);
    return 0;
}

/* One checkerboard half-sweep: every link U_mu(x) with parity(x) = parity.
 * Links of one (mu, parity) class never appear in each other's staples. */
uint32_t or_heatbath_halfsweep(const int n[4], double *U, double beta, uint64_t seed,
                               uint32_t sweep, int mu, int parity, uint32_t lattice_id)
{
    int64_t vol = or_volume(n);
    uint32_t c1 = (uint32_t)(mu + 4 * 1 + 16 * lattice_id);
    uint32_t flags = 0;
#pragma omp parallel for schedule(static) reduction(| : flags)
    for (int64_t i = 0; i < vol; ++i) {
        if (or_parity(n, i) != parity)
            continue;
        double V[4];
        or_staple(n, U, i, mu, V);
        flags |= heatbath_link(U + (i * 4 + mu) * 4, V, beta, seed, (uint32_t)i, c1, sweep);
    }
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Heat bath for single-precision links.  The same chain step with the       */
/* precisions of the single-precision path (Sec. 2.1 runs both precisions):  */
/* links, staple and the new link in single precision; uniforms from the top */
/* 23 bits of the even Philox words; of a Kennedy-Pendleton attempt the two  */
/* logarithms and the cosine in single precision, while lambda^2, the accept */
/* test, x0 = 1 - 2 lambda^2 and |x| are formed in double (lambda^2 carries  */
/* 1 - x0, so x0 near 1 loses nothing); the Creutz branch in double; the     */
/* direction in single precision; the new link renormalised in single        */
/* precision.  Its use is to take every accept/reject decision in the same   */
/* precisions as a single-precision implementation, so that the two agree    */
/* link by link instead of up to decisions that flip between 23-bit and      */
/* 52-bit arithmetic.  Single-precision elementary functions are taken as    */
/* the double-precision value rounded to single precision.                   */
/* ------------------------------------------------------------------------ */
static void qmul_f(const float a[4], const float b[4], float out[4])
{
    float r0 = a[0] * b[0] - (a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
    float r1 = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
    float r2 = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
    float r3 = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
    out[0] = r0;
    out[1] = r1;
    out[2] = r2;
    out[3] = r3;
}

static void link_f(const double *U, int64_t site, int mu, int dagger, float q[4])
{
    const double *l = link(U, site, mu);
    q[0] = (float)l[0];
    for (int k = 1; k < 4; ++k)
        q[k] = dagger ? -(float)l[k] : (float)l[k];
}

static void staple_f32(const int n[4], const double *U, int64_t site, int mu, float V[4])
{
    V[0] = V[1] = V[2] = V[3] = 0.0f;
    int64_t xp = or_neighbor(n, site, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu)
            continue;
        float a[4], b[4], c[4], t[4], s[4];
        int64_t xn = or_neighbor(n, site, nu, +1);
        link_f(U, xp, nu, 0, a);
        link_f(U, xn, mu, 1, b);
        link_f(U, site, nu, 1, c);
        qmul_f(a, b, t);
        qmul_f(t, c, s);
        for (int k = 0; k < 4; ++k)
            V[k] += s[k];
        int64_t xm = or_neighbor(n, site, nu, -1);
        int64_t xpm = or_neighbor(n, xp, nu, -1);
        link_f(U, xpm, nu, 1, a);
        link_f(U, xm, mu, 1, b);
        link_f(U, xm, nu, 0, c);
        qmul_f(a, b, t);
        qmul_f(t, c, s);
        for (int k = 0; k < 4; ++k)
            V[k] += s[k];
    }
}

static void draw_f32(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, float *ua, float *ub)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t r[4];
    or_philox4x32_10(ctr, key, r);
    *ua = or_u01_f32(r[0]);
    *ub = or_u01_f32(r[2]);
}

static uint32_t heatbath_link_f32(double Ulink[4], const float V[4], double beta, uint64_t seed, uint32_t site,
                                  uint32_t c1, uint32_t sweep)
{
    float k = sqrtf(V[0] * V[0] + V[1] * V[1] + V[2] * V[2] + V[3] * V[3]);
    if (!isfinite(k))
        return OR_FLAG_NONFINITE;
    float Vhat[4] = {1.0f, 0.0f, 0.0f, 0.0f};
    if (k > 0.0f) {
        float inv = 1.0f / k;
        for (int j = 0; j < 4; ++j)
            Vhat[j] = V[j] * inv;
    }
    double alpha = beta * (double)k;

    double x0 = 0.0, xlen = 0.0;
    int accepted = 0;
    for (uint32_t a = 0; a < OR_MAX_ATTEMPTS && !accepted; ++a) {
        if (alpha >= 2.0) {
            float u1, u2, u3, u4;
            draw_f32(seed, site, c1, sweep, 4u * a + 0u, &u1, &u2);
            draw_f32(seed, site, c1, sweep, 4u * a + 1u, &u3, &u4);
            float c = (float)cos(2.0 * OR_PI * (double)u2);
            float l1 = (float)log((double)u1), l3 = (float)log((double)u3);
            /* Kennedy-Pendleton: lambda^2 = -(ln u1 + cos^2(2 pi u2) ln u3) / (2 alpha),
             * the single-precision logarithms and cosine taken into FP64 */
            double lam2 = -((double)l1 + (double)(c * c) * (double)l3) / (2.0 * alpha);
            if (lam2 <= 1.0 && (double)u4 * (double)u4 <= 1.0 - lam2) {
                x0 = 1.0 - 2.0 * lam2;
                xlen = 2.0 * sqrt(lam2 * (1.0 - lam2));
                accepted = 1;
            }
        } else {
            float f1, f2;
            draw_f32(seed, site, c1, sweep, 4u * a + 0u, &f1, &f2);
            double u1 = f1, u2 = f2, t;
            if (alpha < 1e-8) {
                t = 2.0 * u1 - 1.0;
            } else {
                double e = exp(-2.0 * alpha);
                t = 1.0 + log(e + u1 * (1.0 - e)) / alpha;
            }
            if (u2 * u2 <= 1.0 - t * t) {
                x0 = t;
                double sq = 1.0 - t * t;
                xlen = sqrt(sq > 0.0 ? sq : 0.0);
                accepted = 1;
            }
        }
    }
    if (!accepted)
        return OR_FLAG_CAP;

    float u5, u6;
    draw_f32(seed, site, c1, sweep, 2u, &u5, &u6);
    float cth = 2.0f * u5 - 1.0f;
    float sq = 1.0f - cth * cth;
    float sth = sqrtf(sq > 0.0f ? sq : 0.0f);
    float cph = (float)cos(2.0 * OR_PI * (double)u6), sph = (float)sin(2.0 * OR_PI * (double)u6);
    float xl = (float)xlen;
    float W[4] = {(float)x0, xl * sth * cph, xl * sth * sph, xl * cth};
    float Vd[4] = {Vhat[0], -Vhat[1], -Vhat[2], -Vhat[3]}, Un[4];
    qmul_f(W, Vd, Un);
    float nrm = 1.0f / sqrtf(Un[0] * Un[0] + Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]);
    for (int j = 0; j < 4; ++j)
        Ulink[j] = (double)(Un[j] * nrm);
    return 0;
}

uint32_t or_heatbath_halfsweep_f32(const int n[4], double *U, double beta, uint64_t seed, uint32_t sweep, int mu,
                                   int parity, uint32_t lattice_id)
{
    int64_t vol = or_volume(n);
    uint32_t c1 = (uint32_t)(mu + 4 * 1 + 16 * lattice_id);
    uint32_t flags = 0;
#pragma omp parallel for schedule(static) reduction(| : flags)
    for (int64_t i = 0; i < vol; ++i) {
        if (or_parity(n, i) != parity)
            continue;
        float V[4];
        staple_f32(n, U, i, mu, V);
        flags |= heatbath_link_f32(U + (i * 4 + mu) * 4, V, beta, seed, (uint32_t)i, c1, sweep);
    }
    return flags;
}

/* A sweep: mu = x, y, z, t in turn, even sites before odd sites. */
uint32_t or_heatbath_sweep(const int n[4], double *U, double beta, uint64_t seed,
                           uint32_t sweep, uint32_t lattice_id)
{
    uint32_t flags = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            flags |= or_heatbath_halfsweep(n, U, beta, seed, sweep, mu, p, lattice_id);
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Overrelaxation (Creutz 1987): U -> Vhat^dagger U^dagger Vhat^dagger keeps */
/* Tr(U V) and is its own inverse; links with V = 0 are left alone.          */
/* ------------------------------------------------------------------------ */
uint32_t or_overrelax_halfsweep(const int n[4], double *U, int mu, int parity)
{
    int64_t vol = or_volume(n);
    uint32_t flags = 0;
#pragma omp parallel for schedule(static) reduction(| : flags)
    for (int64_t i = 0; i < vol; ++i) {
        if (or_parity(n, i) != parity)
            continue;
        double V[4];
        or_staple(n, U, i, mu, V);
        double k = sqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2] + V[3] * V[3]);
        if (!isfinite(k)) {
            flags |= OR_FLAG_NONFINITE;
            continue;
        }
        if (k == 0.0)
            continue;
        double Vd[4], Ud[4], t[4];
        for (int j = 0; j < 4; ++j)
            Vd[j] = V[j] / k;
        Vd[1] = -Vd[1];
        Vd[2] = -Vd[2];
        Vd[3] = -Vd[3];
        double *Ul = U + (i * 4 + mu) * 4;
        or_qdag(Ul, Ud);
        or_qmul(Vd, Ud, t);
        or_qmul(t, Vd, Ul);
    }
    return flags;
}

uint32_t or_overrelax_sweep(const int n[4], double *U)
{
    uint32_t flags = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p)
            flags |= or_overrelax_halfsweep(n, U, mu, p);
    return flags;
}

/* ------------------------------------------------------------------------ */
/* Mean plaquette (Sec. 2.1): the average over all 6V plaquettes of          */
/* (1/2) Tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+].  planes[] holds the  */
/* six per-plane averages in the order (01,02,03,12,13,23).  Per-site values */
/* are stored first and summed afterwards in extended precision, so the sum */
/* does not depend on the thread count.                                      */
/* ------------------------------------------------------------------------ */
static double plaq_one(const int n[4], const double *U, int64_t i, int mu, int nu)
{
    double a[4], b[4], c[4], d[4];
    int64_t xmu = or_neighbor(n, i, mu, +1);
    int64_t xnu = or_neighbor(n, i, nu, +1);
    or_qmul(link(U, i, mu), link(U, xmu, nu), a);
    or_qdag(link(U, xnu, mu), c);
    or_qmul(a, c, b);
    or_qdag(link(U, i, nu), c);
    or_qmul(b, c, d);
    return d[0];
}

double or_plaquette(const int n[4], const double *U, double planes[6])
{
    int64_t vol = or_volume(n);
    double *per = (double *)malloc(sizeof(double) * (size_t)vol * 6);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < vol; ++i) {
        int p = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu)
                per[i * 6 + p++] = plaq_one(n, U, i, mu, nu);
    }
    long double tot[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < vol; ++i)
        for (int p = 0; p < 6; ++p)
            tot[p] += per[i * 6 + p];
    free(per);
    long double all = 0;
    for (int p = 0; p < 6; ++p) {
        if (planes)
            planes[p] = (double)(tot[p] / (long double)vol);
        all += tot[p];
    }
    return (double)(all / (6.0L * (long double)vol));
}

/* ------------------------------------------------------------------------ */
/* Polyakov loop (Sec. 2.2, eq. (1)): at each spatial site the half trace of */
/* the ordered product U_t(x,0) U_t(x,1) ... U_t(x,Nt-1).  L is indexed by   */
/* the spatial site x + Nx*(y + Ny*z).                                       */
/* ------------------------------------------------------------------------ */
void or_polyakov_field(const int n[4], const double *U, double *L)
{
    int64_t vs = (int64_t)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < vs; ++s) {
        double P[4] = {1.0, 0.0, 0.0, 0.0}, T[4];
        for (int t = 0; t < n[3]; ++t) {
            or_qmul(P, link(U, s + vs * t, 3), T);
            memcpy(P, T, sizeof P);
        }
        L[s] = P[0];
    }
}

/* out[0] = spatial average of L, out[1] = spatial average of |L|. */
void or_polyakov(const int n[4], const double *U, double out[2])
{
    int64_t vs = (int64_t)n[0] * n[1] * n[2];
    double *L = (double *)malloc(sizeof(double) * (size_t)vs);
    or_polyakov_field(n, U, L);
    long double s = 0, sa = 0;
    for (int64_t i = 0; i < vs; ++i) {
        s += L[i];
        sa += fabs(L[i]);
    }
    free(L);
    out[0] = (double)(s / (long double)vs);
    out[1] = (double)(sa / (long double)vs);
}

/* On-axis correlator (Sec. 2.2, eq. (3)): for SU(2), L is real and
 * (1/4) Tr L(y) Tr L(x)^dagger = L(y) L(x) with L normalised by 1/2, so
 *   C(r) = (1/(3 Vs)) sum_x sum_{i=x,y,z} L(x) L(x + r e_i),
 * for r = 1 .. min(Nx,Ny,Nz)/2.  C[r-1] receives C(r); returns the number
 * of r values written. */
int or_polyakov_corr(const int n[4], const double *U, double *C)
{
    int64_t vs = (int64_t)n[0] * n[1] * n[2];
    double *L = (double *)malloc(sizeof(double) * (size_t)vs);
    or_polyakov_field(n, U, L);
    int ns = n[0];
    if (n[1] < ns)
        ns = n[1];
    if (n[2] < ns)
        ns = n[2];
    int rmax = ns / 2;
    for (int r = 1; r <= rmax; ++r) {
        long double acc = 0;
        for (int64_t s = 0; s < vs; ++s) {
            int x = (int)(s % n[0]);
            int y = (int)((s / n[0]) % n[1]);
            int z = (int)(s / ((int64_t)n[0] * n[1]));
            int64_t sx = (x + r) % n[0] + (int64_t)n[0] * (y + (int64_t)n[1] * z);
            int64_t sy = x + (int64_t)n[0] * ((y + r) % n[1] + (int64_t)n[1] * z);
            int64_t sz = x + (int64_t)n[0] * (y + (int64_t)n[1] * ((z + r) % n[2]));
            acc += (long double)L[s] * L[sx] + (long double)L[s] * L[sy] +
                   (long double)L[s] * L[sz];
        }
        C[r - 1] = (double)(acc / (3.0L * (long double)vs));
    }
    free(L);
    return rmax;
}

/* ------------------------------------------------------------------------ */
/* Random gauge transformation, g(x) Haar-random (Philox kind 3).            */
/* ------------------------------------------------------------------------ */
void or_gauge_transform(const int n[4], double *U, uint64_t seed, uint32_t lattice_id)
{
    int64_t vol = or_volume(n);
    double *g = (double *)malloc(sizeof(double) * (size_t)vol * 4);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < vol; ++i)
        haar_from_counter(seed, (uint32_t)i, (uint32_t)(4 * 3 + 16 * lattice_id), 0u, g + 4 * i);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < vol; ++i) {
        for (int mu = 0; mu < 4; ++mu) {
            int64_t j = or_neighbor(n, i, mu, +1);
            double t[4], gd[4];
            double *Ul = U + (i * 4 + mu) * 4;
            or_qmul(g + 4 * i, Ul, t);
            or_qdag(g + 4 * j, gd);
            or_qmul(t, gd, Ul);
        }
    }
    free(g);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================== */
/* Learned block proposal (test reference).  A move updates the temporal    */
/* link T(e) of one spatial site e of time slice tau with the temporal      */
/* links of its six spatial neighbours o integrated out:                     */
/*   the marginal of T(e) is prod_o Z(beta |V_o(T(e))|), Z(a) = 2 I1(a)/a,   */
/* because each of the six plaquettes holding T(e) holds exactly one T(o).  */
/* T(e) is proposed from q(T) ~ exp((1/2) Tr(T M)), M = sum_o c_o S_o, and  */
/* accepted with the Metropolis-Hastings ratio of the marginal; then every  */
/* T(o) is redrawn by heat bath given the new T(e).  S_o is the staple of   */
/* T(o) without the term through e, carried to e: with that term written    */
/* X T(e)^+ Y,  S_o = X^+ V_o^rest Y^+, so that                               */
/*   |V_o(T)|^2 = |S_o|^2 + 1 + 2 (1/2)Tr(T S_o).                           */
/* c_o = beta r(a0)/sqrt(|S_o|^2+1) exp(y_o), a0 = beta sqrt(|S_o|^2+1),     */
/* r = I2/I1 (the slope of log Z), y_o supplied by the caller (the network). */
/* ======================================================================== */

/* e^{-x} I_n(x).  For x >= 1: (1/2pi) int_0^{2pi} exp(x (cos t - 1))       */
/* cos(n t) dt by the trapezoidal rule, which converges geometrically for   */
/* this periodic analytic integrand (256 points: below 1e-15 relative for   */
/* x <= 200).  For x < 1, where I_2 is small against the integrand and the  */
/* rule would lose relative accuracy: the power series                      */
/* sum_k (x/2)^(2k+n) / (k! (k+n)!).                                        */
double or_bessel_ive(int n, double x)
{
    if (x < 1.0) {
        double term = 1.0;
        for (int j = 1; j <= n; ++j)
            term *= 0.5 * x / j;
        double sum = 0.0;
        for (int k = 0; k < 30; ++k) {
            sum += term;
            term *= 0.25 * x * x / ((k + 1.0) * (k + 1.0 + n));
        }
        return sum * exp(-x);
    }
    const int K = 256;
    long double s = 0.0L;
    for (int j = 0; j < K; ++j) {
        double t = 2.0 * OR_PI * j / K;
        s += (long double)(exp(x * (cos(t) - 1.0)) * cos(n * t));
    }
    return (double)(s / K);
}

/* log Z(a) = log(2 I1(a)/a); Z(0) = 1. */
double or_log_z(double a)
{
    if (a < 1e-300)
        return 0.0;
    return log(2.0 * or_bessel_ive(1, a) / a) + a;
}

double or_bessel_ratio(double a)
{
    if (a < 1e-300)
        return 0.0;
    return or_bessel_ive(2, a) / or_bessel_ive(1, a);
}

static double qnorm(const double a[4])
{
    return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
}

/* (1/2) Tr(A B) = scalar part of the product. */
static double half_tr(const double a[4], const double b[4])
{
    double p[4];
    or_qmul(a, b, p);
    return p[0];
}

/* Neighbour o = e + s e_i (s = -1, +1) of spatial direction i, and the     */
/* pieces of the term of V_o through e: X, Y with term = X T(e)^+ Y.        */
static void block_neighbour(const int n[4], const double *U, int64_t e, int dir, int64_t *o,
                            double X[4], double Y[4])
{
    int i = dir / 2, s = (dir % 2) ? +1 : -1;
    *o = or_neighbor(n, e, i, s);
    if (s < 0) {
        /* e = o + i: upper term U_i(o+t) T(o+i)^+ U_i(o)^+ */
        int64_t ot = or_neighbor(n, *o, 3, +1);
        memcpy(X, link(U, ot, i), 4 * sizeof(double));
        or_qdag(link(U, *o, i), Y);
    } else {
        /* e = o - i: lower term U_i(o+t-i)^+ T(o-i)^+ U_i(o-i) = U_i(e+t)^+ T(e)^+ U_i(e) */
        int64_t et = or_neighbor(n, e, 3, +1);
        or_qdag(link(U, et, i), X);
        memcpy(Y, link(U, e, i), 4 * sizeof(double));
    }
}

/* S_o for direction dir (0..5 = -x,+x,-y,+y,-z,+z) of block centre e. */
void or_block_piece(const int n[4], const double *U, int64_t e, int dir, double S[4])
{
    int64_t o;
    double X[4], Y[4], V[4], t1[4], t2[4], Td[4];
    block_neighbour(n, U, e, dir, &o, X, Y);
    or_staple(n, U, o, 3, V);
    /* remove the term through e */
    or_qdag(link(U, e, 3), Td);
    or_qmul(X, Td, t1);
    or_qmul(t1, Y, t2);
    for (int k = 0; k < 4; ++k)
        V[k] -= t2[k];
    /* S = X^+ V Y^+ */
    double Xd[4], Yd[4];
    or_qdag(X, Xd);
    or_qdag(Y, Yd);
    or_qmul(Xd, V, t1);
    or_qmul(t1, Yd, S);
}

/* Marginal log density of T(e) = T (up to a constant) given the pieces. */
static double block_log_marginal(double beta, const double S[6][4], const double T[4])
{
    double lp = 0.0;
    for (int d = 0; d < 6; ++d) {
        double s2 = S[d][0] * S[d][0] + S[d][1] * S[d][1] + S[d][2] * S[d][2] + S[d][3] * S[d][3];
        double v2 = s2 + 1.0 + 2.0 * half_tr(T, S[d]);
        lp += or_log_z(beta * sqrt(v2 > 0.0 ? v2 : 0.0));
    }
    return lp;
}

double or_block_log_marginal(const int n[4], const double *U, int64_t e, double beta, const double T[4])
{
    double S[6][4];
    for (int d = 0; d < 6; ++d)
        or_block_piece(n, U, e, d, S[d]);
    return block_log_marginal(beta, S, T);
}

/* Effective staple M of the proposal at e for network outputs y[6]. */
void or_block_proposal(const int n[4], const double *U, int64_t e, double beta, const double y[6],
                       double M[4])
{
    M[0] = M[1] = M[2] = M[3] = 0.0;
    for (int d = 0; d < 6; ++d) {
        double S[4];
        or_block_piece(n, U, e, d, S);
        double s = qnorm(S);
        double a0 = beta * sqrt(s * s + 1.0);
        double c = beta * or_bessel_ratio(a0) / sqrt(s * s + 1.0) * exp(y[d]);
        for (int k = 0; k < 4; ++k)
            M[k] += c * S[k];
    }
}

/* Draw W with density ~ exp(alpha w0) dHaar (the heat-bath law) from the   */
/* counter stream (c0, c1, c2, 4 attempt + draw); returns 0 on success.     */
static uint32_t sample_w(double alpha, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, double W[4])
{
    double x0 = 0.0, xlen = 0.0;
    int ok = 0;
    for (uint32_t a = 0; a < OR_MAX_ATTEMPTS && !ok; ++a) {
        if (alpha >= 2.0) {
            double u1, u2, u3, u4;
            draw2(seed, c0, c1, c2, 4u * a + 0u, &u1, &u2);
            draw2(seed, c0, c1, c2, 4u * a + 1u, &u3, &u4);
            double c = cos(2.0 * OR_PI * u2);
            double lam2 = -(log(u1) + c * c * log(u3)) / (2.0 * alpha);
            if (lam2 <= 1.0 && u4 * u4 <= 1.0 - lam2) {
                x0 = 1.0 - 2.0 * lam2;
                xlen = 2.0 * sqrt(lam2 * (1.0 - lam2));
                ok = 1;
            }
        } else {
            double u1, u2, t;
            draw2(seed, c0, c1, c2, 4u * a + 0u, &u1, &u2);
            if (alpha < 1e-8) {
                t = 2.0 * u1 - 1.0;
            } else {
                double ex = exp(-2.0 * alpha);
                t = 1.0 + log(ex + u1 * (1.0 - ex)) / alpha;
            }
            if (u2 * u2 <= 1.0 - t * t) {
                x0 = t;
                double s = 1.0 - t * t;
                xlen = sqrt(s > 0.0 ? s : 0.0);
                ok = 1;
            }
        }
    }
    if (!ok)
        return OR_FLAG_CAP;
    double u5, u6;
    draw2(seed, c0, c1, c2, 2u, &u5, &u6);
    double cth = 2.0 * u5 - 1.0;
    double s = 1.0 - cth * cth;
    double sth = sqrt(s > 0.0 ? s : 0.0);
    double phi = 2.0 * OR_PI * u6;
    W[0] = x0;
    W[1] = xlen * sth * cos(phi);
    W[2] = xlen * sth * sin(phi);
    W[3] = xlen * cth;
    return 0;
}

/* Draw U ~ exp((1/2)Tr(U M)) dHaar: W from the law at alpha = |M|, U = W Mhat^+. */
static uint32_t sample_vmf(const double M[4], uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                           double out[4])
{
    double k = qnorm(M);
    double Mh[4] = {1.0, 0.0, 0.0, 0.0};
    if (k > 0.0)
        for (int j = 0; j < 4; ++j)
            Mh[j] = M[j] / k;
    double W[4], Md[4];
    uint32_t f = sample_w(k, seed, c0, c1, c2, W);
    if (f)
        return f;
    or_qdag(Mh, Md);
    or_qmul(W, Md, out);
    return 0;
}

/* Colour of a spatial site for the block classes: (x + 2y + 3z) mod 8.    */
/* Two sites of one parity and one colour are at L1 distance >= 4, so their */
/* blocks (centre and six neighbours) neither overlap nor read each other.  */
int or_block_colour(int x, int y, int z)
{
    return (x + 2 * y + 3 * z) % 8;
}

/* All blocks of centre parity p and colour k, every time slice: the move   */
/* described above.  y holds 6 network outputs per (slice, spatial site),   */
/* index (t * Vs + s) * 6 + d.  Counters: (site, 3 + 4*2 + 16*lattice_id,   */
/* 16*step + 8*p + k, 4*attempt + draw): proposal attempts draws 0,1, its   */
/* direction draw 2, the accept uniform draw 3 (attempt 0); each refreshed   */
/* neighbour uses its own site index with draws 0,1,2.  accepted[0] counts   */
/* accepted moves.  Returns flag bits.                                       */
uint32_t or_block_move(const int n[4], double *U, double beta, uint64_t seed, uint32_t step, int p, int k,
                       const double *y, uint32_t lattice_id, int64_t *accepted)
{
    int64_t vs = (int64_t)n[0] * n[1] * n[2];
    uint32_t c1 = (uint32_t)(3 + 4 * 2 + 16 * lattice_id);
    uint32_t c2 = 16u * step + 8u * (uint32_t)p + (uint32_t)k;
    uint32_t flags = 0;
    int64_t acc = 0;
#pragma omp parallel for schedule(static) reduction(| : flags) reduction(+ : acc)
    for (int64_t i = 0; i < or_volume(n); ++i) {
        int c[4];
        coords(n, i, c);
        if (((c[0] + c[1] + c[2]) & 1) != p || or_block_colour(c[0], c[1], c[2]) != k)
            continue;
        double S[6][4], M[4] = {0, 0, 0, 0};
        for (int d = 0; d < 6; ++d) {
            or_block_piece(n, U, i, d, S[d]);
            double s = qnorm(S[d]);
            double a0 = beta * sqrt(s * s + 1.0);
            double cf = beta * or_bessel_ratio(a0) / sqrt(s * s + 1.0) * exp(y[(c[3] * vs + i % vs) * 6 + d]);
            for (int j = 0; j < 4; ++j)
                M[j] += cf * S[d][j];
        }
        double *T = U + (i * 4 + 3) * 4;
        double Tn[4];
        uint32_t f = sample_vmf(M, seed, (uint32_t)i, c1, c2, Tn);
        if (f) {
            flags |= f;
            continue;
        }
        double logr = block_log_marginal(beta, S, Tn) - block_log_marginal(beta, S, T) +
                      half_tr(T, M) - half_tr(Tn, M);
        double ua, ub;
        draw2(seed, (uint32_t)i, c1, c2, 3u, &ua, &ub);
        if (log(ua) < logr) {
            memcpy(T, Tn, sizeof Tn);
            acc += 1;
        }
        for (int d = 0; d < 6; ++d) {
            int64_t o;
            double X[4], Y[4], V[4], Un[4];
            block_neighbour(n, U, i, d, &o, X, Y);
            or_staple(n, U, o, 3, V);
            double Vb[4] = {beta * V[0], beta * V[1], beta * V[2], beta * V[3]};
            uint32_t g = sample_vmf(Vb, seed, (uint32_t)o, c1, c2, Un);
            if (g)
                flags |= g;
            else
                memcpy(U + (o * 4 + 3) * 4, Un, sizeof Un);
        }
    }
    if (accepted)
        *accepted += acc;
    return flags;
}

/* A sweep of block moves: centre parity 0 then 1, colours 0..7. */
uint32_t or_block_sweep(const int n[4], double *U, double beta, uint64_t seed, uint32_t step, const double *y,
                        uint32_t lattice_id, int64_t *accepted)
{
    uint32_t flags = 0;
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < 8; ++k)
            flags |= or_block_move(n, U, beta, seed, step, p, k, y, lattice_id, accepted);
    return flags;
}

/* Block pieces of every site: S[(site*6 + dir)*4 + k]. */
void or_block_pieces_all(const int n[4], const double *U, double *S)
{
    int64_t vol = or_volume(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < vol; ++i)
        for (int d = 0; d < 6; ++d)
            or_block_piece(n, U, i, d, S + (i * 6 + d) * 4);
}

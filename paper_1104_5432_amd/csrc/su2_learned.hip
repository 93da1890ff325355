// su2_learned.hip -- learned block proposal on gfx950: gauge-invariant input
// features, the proposal network (3x3x3 periodic convolutions on BF16 MFMA
// with FP32 accumulation, forward and backward), its maximum-likelihood loss
// gradient, Adam, and the exact Metropolis-Hastings block move.
//
// Block move (per spatial site e of a time slice, the "centre"): the
// temporal links of e's six spatial neighbours o are integrated out, so the
// marginal of the centre's temporal link T is prod_o Z(beta |V_o(T)|),
// Z(a) = 2 I1(a)/a.  With the term of V_o through e written X T^+ Y, the
// piece S_o = X^+ (V_o - X T^+ Y) Y^+ gives |V_o(T)|^2 = |S_o|^2 + 1 +
// 2 (1/2)Tr(T S_o).  The proposal is q(T) ~ exp((1/2)Tr(T M)) with
// M = sum_o c_o S_o, c_o = beta r(a0)/sqrt(|S_o|^2+1) exp(y_o), a0 =
// beta sqrt(|S_o|^2+1), r = I2/I1, y the network output; MH accepts with the
// marginal ratio times q(T)/q(T'), then every neighbour's temporal link is
// redrawn by heat bath.  Centres of one parity and colour (x+2y+3z) mod 8 are
// >= 4 apart, so their blocks are independent and run in one launch.
#include "su2_device.hpp"
#include "su2_learned.hpp"

namespace su2 {
namespace lp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// ---------------------------------------------------------------------------
// Bessel functions I1, I2 (for the block marginal and the proposal):
// power series below x = 30 (all terms positive), the Hankel asymptotic
// expansion above.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bessel_i1_i2(double x, double &log_i1, double &ratio)
{
    if (x <= 0.0) {
        log_i1 = -INFINITY;
        ratio = 0.0;
        return;
    }
    if (x < 30.0) {
        const double q = 0.25 * x * x;
        double t1 = 0.5 * x, t2 = 0.125 * x * x;   // k = 0 terms of I1, I2
        double s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < 120; ++k) {
            s1 += t1;
            s2 += t2;
            t1 *= q / ((k + 1.0) * (k + 2.0));
            t2 *= q / ((k + 1.0) * (k + 3.0));
            if (t1 < 1e-18 * s1)
                break;
        }
        log_i1 = log(s1);
        ratio = s2 / s1;
        return;
    }
    double a1 = 1.0, a2 = 1.0, s1 = 1.0, s2 = 1.0;
    for (int k = 1; k <= 24; ++k) {
        const double odd = (2.0 * k - 1.0) * (2.0 * k - 1.0);
        a1 *= -(4.0 - odd) / (8.0 * k * x);
        a2 *= -(16.0 - odd) / (8.0 * k * x);
        s1 += a1;
        s2 += a2;
    }
    log_i1 = x - 0.5 * log(2.0 * kPi * x) + log(s1);
    ratio = s2 / s1;
}

// log Z(a) = log(2 I1(a)/a), Z(0) = 1.
__device__ __forceinline__ double log_z(double a)
{
    if (a < 1e-300)
        return 0.0;
    double li, r;
    bessel_i1_i2(a, li, r);
    return li + log(2.0 / a);
}

__device__ __forceinline__ double bessel_ratio(double a)
{
    double li, r;
    bessel_i1_i2(a, li, r);
    return r;
}

// ---------------------------------------------------------------------------
// Lattice access by linear site index.
// ---------------------------------------------------------------------------
struct Coord {
    int32_t x, y, z, t;
};

__device__ __forceinline__ Coord coord_of(const Geom &g, uint32_t site)
{
    Coord c;
    const uint32_t yzt = fdiv(site, g.div_nx);
    c.x = (int32_t)(site - yzt * (uint32_t)g.n[0]);
    const uint32_t zt = fdiv(yzt, g.div_ny);
    c.y = (int32_t)(yzt - zt * (uint32_t)g.n[1]);
    const uint32_t t = fdiv(zt, g.div_nz);
    c.z = (int32_t)(zt - t * (uint32_t)g.n[2]);
    c.t = (int32_t)t;
    return c;
}

__device__ __forceinline__ uint32_t site_at(const Geom &g, int32_t x, int32_t y, int32_t z, int32_t t)
{
    return (uint32_t)x + (uint32_t)g.n[0] * ((uint32_t)y + (uint32_t)g.n[1] * ((uint32_t)z + (uint32_t)g.n[2] * (uint32_t)t));
}

__device__ __forceinline__ uint32_t shifted(const Geom &g, const Coord &c, int d, int s)
{
    int32_t v[4] = {c.x, c.y, c.z, c.t};
    v[d] = wrap_add(v[d], s, g.n[d]);
    return site_at(g, v[0], v[1], v[2], v[3]);
}

template <class T>
__device__ __forceinline__ Quat<double> load_d(const Links<T> &U, int mu, uint32_t site, const Geom &g)
{
    const Coord c = coord_of(g, site);
    const int par = (c.x + c.y + c.z + c.t) & 1;
    const Quat<T> q = U.ld(mu, par, site >> 1);
    return {(double)q.w, (double)q.x, (double)q.y, (double)q.z};
}

template <class T>
__device__ __forceinline__ void store_d(const Links<T> &U, int mu, uint32_t site, const Geom &g, const Quat<double> &q)
{
    const Coord c = coord_of(g, site);
    const int par = (c.x + c.y + c.z + c.t) & 1;
    U.st(mu, par, site >> 1, unitize(Quat<T>{(T)q.w, (T)q.x, (T)q.y, (T)q.z}));
}

// Staple of the temporal link at `site`, in FP64.
template <class T>
__device__ __forceinline__ Quat<double> temporal_staple(const Links<T> &U, const Geom &g, uint32_t site)
{
    const Coord c = coord_of(g, site);
    Site s;
    s.c[0] = c.x;
    s.c[1] = c.y;
    s.c[2] = c.z;
    s.c[3] = c.t;
    s.site = site;
    const int par = (c.x + c.y + c.z + c.t) & 1;
    const Quat<T> V = staple<T, 3>(U, g, s, site >> 1, par);
    return {(double)V.w, (double)V.x, (double)V.y, (double)V.z};
}

// Piece S_o of centre e for direction d (0..5 = -x,+x,-y,+y,-z,+z); also
// returns the neighbour's site, the factors X, Y of its staple's term
// through e (X T(e)^+ Y) and the rest of that staple, V_o - X T(e)^+ Y.
template <class T>
__device__ __forceinline__ Quat<double> block_piece(const Links<T> &U, const Geom &g, uint32_t e,
                                                    const Quat<double> &Te, int d, uint32_t &o, Quat<double> &X,
                                                    Quat<double> &Y, Quat<double> &Vrest)
{
    const Coord ce = coord_of(g, e);
    const int i = d >> 1;
    const int sgn = (d & 1) ? 1 : -1;
    o = shifted(g, ce, i, sgn);
    if (sgn < 0) {
        // e = o + i: the upper term U_i(o+t) T(e)^+ U_i(o)^+
        const Coord co = coord_of(g, o);
        X = load_d(U, i, shifted(g, co, 3, 1), g);
        const Quat<double> a = load_d(U, i, o, g);
        Y = {a.w, -a.x, -a.y, -a.z};
    } else {
        // e = o - i: the lower term U_i(e+t)^+ T(e)^+ U_i(e)
        const Quat<double> a = load_d(U, i, shifted(g, ce, 3, 1), g);
        X = {a.w, -a.x, -a.y, -a.z};
        Y = load_d(U, i, e, g);
    }
    const Quat<double> V = temporal_staple(U, g, o);
    const Quat<double> term = qmul(qmul_nd(X, Te), Y);
    Vrest = {V.w - term.w, V.x - term.x, V.y - term.y, V.z - term.z};
    return qmul_nd(qmul_dn(X, Vrest), Y);   // X^+ Vrest Y^+
}

template <class T>
__device__ __forceinline__ Quat<double> block_piece(const Links<T> &U, const Geom &g, uint32_t e,
                                                    const Quat<double> &Te, int d, uint32_t &o)
{
    Quat<double> X, Y, Vrest;
    return block_piece(U, g, e, Te, d, o, X, Y, Vrest);
}

__device__ __forceinline__ double half_tr(const Quat<double> &a, const Quat<double> &b)
{
    return a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
}

__device__ __forceinline__ double qdot4(const Quat<double> &a, const Quat<double> &b)
{
    return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z;
}

// c_d without the network factor: beta r(a0)/sqrt(s^2+1), a0 = beta sqrt(s^2+1).
__device__ __forceinline__ double mean_field_coefficient(double beta, double s2)
{
    const double root = sqrt(s2 + 1.0);
    return beta * bessel_ratio(beta * root) / root;
}

// Draw W ~ exp(alpha w0) dHaar from the counter stream (c0,c1,c2, 4a+draw),
// then U = W Mhat^+ (FP64 for both link precisions).
__device__ __forceinline__ bool sample_vmf(const Quat<double> &M, uint32_t c0, uint32_t c1, uint32_t c2,
                                           uint32_t k0, uint32_t k1, Quat<double> &out)
{
    const double k = sqrt(qdot4(M, M));
    Quat<double> Mh = {1.0, 0.0, 0.0, 0.0};
    if (k > 0.0)
        Mh = {M.w / k, M.x / k, M.y / k, M.z / k};
    const double inv2a = 1.0 / (2.0 * fmax(k, 1.0));
    double x0 = 0.0, xlen = 0.0;
    bool ok = false;
    for (uint32_t a = 0; a < kMaxAttempts && !ok; ++a) {
        if (k >= 2.0) {
            double u1, u2, u3, u4;
            Draw<double>::two(philox(c0, c1, c2, 4u * a, k0, k1), u1, u2);
            Draw<double>::two(philox(c0, c1, c2, 4u * a + 1u, k0, k1), u3, u4);
            const double c = cos((2.0 * kPi) * u2);
            const double lam2 = -(log(u1) + c * c * log(u3)) * inv2a;
            if (lam2 <= 1.0 && u4 * u4 <= 1.0 - lam2) {
                x0 = 1.0 - 2.0 * lam2;
                xlen = 2.0 * sqrt(lam2 * (1.0 - lam2));
                ok = true;
            }
        } else {
            double u1, u2;
            Draw<double>::two(philox(c0, c1, c2, 4u * a, k0, k1), u1, u2);
            double t;
            if (k < 1e-8) {
                t = 2.0 * u1 - 1.0;
            } else {
                const double e = exp(-2.0 * k);
                t = 1.0 + log(e + u1 * (1.0 - e)) / k;
            }
            if (u2 * u2 <= 1.0 - t * t) {
                x0 = t;
                xlen = sqrt(fmax(0.0, 1.0 - t * t));
                ok = true;
            }
        }
    }
    if (!ok)
        return false;
    double u5, u6;
    Draw<double>::two(philox(c0, c1, c2, 2u, k0, k1), u5, u6);
    const double cth = 2.0 * u5 - 1.0;
    const double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
    double sph, cph;
    sincos((2.0 * kPi) * u6, &sph, &cph);
    const Quat<double> W = {x0, xlen * sth * cph, xlen * sth * sph, xlen * cth};
    out = qmul_nd(W, Mh);
    return true;
}

// ---------------------------------------------------------------------------
// Block move for centres of parity p and colour k, every slice.  A team of 8
// lanes takes one centre: lane d < 6 handles direction d (its piece,
// coefficient, marginal term and the redraw of its neighbour), M and the
// log acceptance ratio are summed over the team with xor shuffles, lane 0
// samples the proposal and takes the decision.
// ---------------------------------------------------------------------------
template <class V>
__device__ __forceinline__ V team_sum(V v)
{
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    return v;
}

__device__ __forceinline__ Quat<double> team_sum(const Quat<double> &q)
{
    return {team_sum(q.w), team_sum(q.x), team_sum(q.y), team_sum(q.z)};
}

__device__ __forceinline__ Quat<double> team_bcast(const Quat<double> &q)
{
    return {__shfl(q.w, 0, 8), __shfl(q.x, 0, 8), __shfl(q.y, 0, 8), __shfl(q.z, 0, 8)};
}

template <class T>
__global__ __launch_bounds__(64) void block_move_kernel(Links<T> U, Geom g, double beta, uint32_t k0, uint32_t k1,
                                                         uint32_t c1, uint32_t c2, int p, int colour,
                                                         const float *y, uint32_t *accepted, uint32_t *flags)
{
    const uint32_t per_slice = g.vs / 16u;
    const uint32_t count = per_slice * (uint32_t)g.n[3];
    const uint32_t j = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int d = (int)(threadIdx.x & 7u);
    const bool centre_ok = j < count;
    const bool lane_ok = centre_ok && d < 6;

    uint32_t e = 0;
    if (centre_ok) {
        const uint32_t t = j / per_slice;
        uint32_t rem = j - t * per_slice;
        const uint32_t nx8 = (uint32_t)g.n[0] / 8u, ny2 = (uint32_t)g.n[1] / 2u;
        const uint32_t xi = rem % nx8;
        rem /= nx8;
        const uint32_t yi = rem % ny2;
        const uint32_t z = rem / ny2;
        const int32_t yy = (int32_t)(2u * yi + (uint32_t)((p + colour) & 1));
        const int32_t x0 = (((colour - 2 * yy - 3 * (int32_t)z) % 8) + 8) % 8;
        e = site_at(g, x0 + 8 * (int32_t)xi, yy, (int32_t)z, (int32_t)t);
    }
    const Quat<double> Te = centre_ok ? load_d(U, 3, e, g) : Quat<double>{1.0, 0.0, 0.0, 0.0};

    Quat<double> S = {0, 0, 0, 0}, X = {1, 0, 0, 0}, Y = {1, 0, 0, 0}, Vrest = {0, 0, 0, 0};
    double s2 = 0.0, c = 0.0;
    uint32_t o = 0;
    if (lane_ok) {
        S = block_piece(U, g, e, Te, d, o, X, Y, Vrest);
        s2 = qdot4(S, S);
        c = mean_field_coefficient(beta, s2) * exp((double)y[(size_t)e * 6 + d]);
    }
    const Quat<double> M = team_sum(Quat<double>{c * S.w, c * S.x, c * S.y, c * S.z});

    Quat<double> Tn = Te;
    int ok = 1;
    if (d == 0 && centre_ok)
        ok = sample_vmf(M, e, c1, c2, k0, k1, Tn) ? 1 : 0;
    Tn = team_bcast(Tn);
    ok = __shfl(ok, 0, 8);

    double part = 0.0;
    if (lane_ok && ok) {
        const double vn = s2 + 1.0 + 2.0 * half_tr(Tn, S);
        const double vo = s2 + 1.0 + 2.0 * half_tr(Te, S);
        part = log_z(beta * sqrt(fmax(vn, 0.0))) - log_z(beta * sqrt(fmax(vo, 0.0)));
    }
    const double logmarg = team_sum(part);

    int acc = 0;
    if (d == 0 && centre_ok) {
        if (!ok) {
            atomicOr(flags, kFlagCap);
        } else {
            const double logr = logmarg + half_tr(Te, M) - half_tr(Tn, M);
            double ua, ub;
            Draw<double>::two(philox(e, c1, c2, 3u, k0, k1), ua, ub);
            if (log(ua) < logr) {
                acc = 1;
                store_d(U, 3, e, g, Tn);
                atomicAdd(accepted, 1u);
            }
        }
    }
    acc = __shfl(acc, 0, 8);
    if (!lane_ok || !ok)
        return;
    // redraw the neighbour's temporal link given the centre's current link
    const Quat<double> Tc = acc ? Tn : Te;
    const Quat<double> term = qmul(qmul_nd(X, Tc), Y);
    const Quat<double> Vb = {beta * (Vrest.w + term.w), beta * (Vrest.x + term.x), beta * (Vrest.y + term.y),
                             beta * (Vrest.z + term.z)};
    Quat<double> Un;
    if (sample_vmf(Vb, o, c1, c2, k0, k1, Un))
        store_d(U, 3, o, g, Un);
    else
        atomicOr(flags, kFlagCap);
}

// ---------------------------------------------------------------------------
// Network.  Sites are the lattice's linear site indices; a convolution reads
// its 27 neighbours within the same time slice (periodic in x, y, z).
// ---------------------------------------------------------------------------
constexpr int CIN = 8, CH = 32, NTAP = 27, NDIR = 6;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NTAP * CIN * CH, OFF_W2 = OFF_B1 + CH, OFF_B2 = OFF_W2 + NTAP * CH * CH,
              OFF_W3 = OFF_B2 + CH, OFF_B3 = OFF_W3 + NTAP * CH * CH, OFF_V = OFF_B3 + CH, OFF_BV = OFF_V + NDIR * CH,
              NPARAM = OFF_BV + NDIR;
static_assert(NPARAM == 62502, "parameter count");

__device__ __forceinline__ uint32_t tap_neighbour(const Geom &g, const Coord &c, int tap, int sign)
{
    const int dx = (tap % 3 - 1) * sign, dy = ((tap / 3) % 3 - 1) * sign, dz = (tap / 9 - 1) * sign;
    return site_at(g, wrap_add(c.x, dx, g.n[0]), wrap_add(c.y, dy, g.n[1]), wrap_add(c.z, dz, g.n[2]), c.t);
}

// Input features: spatial plaquettes of slices t and t+1 (planes xy, xz, yz), two zeros.
template <class T>
__global__ __launch_bounds__(256) void features_kernel(Links<T> U, Geom g, float *feat)
{
    const uint32_t site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= 2u * g.half)
        return;
    const Coord c = coord_of(g, site);
    float f[CIN] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int h = 0; h < 2; ++h) {
        const uint32_t s0 = h ? shifted(g, c, 3, 1) : site;
        const Coord cs = coord_of(g, s0);
        int slot = 0;
        for (int i = 0; i < 3; ++i)
            for (int jdir = i + 1; jdir < 3; ++jdir) {
                const Quat<double> ui = load_d(U, i, s0, g);
                const Quat<double> uj_i = load_d(U, jdir, shifted(g, cs, i, 1), g);
                const Quat<double> ui_j = load_d(U, i, shifted(g, cs, jdir, 1), g);
                const Quat<double> uj = load_d(U, jdir, s0, g);
                const Quat<double> a = qmul(ui, uj_i);
                const Quat<double> b = qmul(uj, ui_j);     // (ui_j^+ uj^+)^+ = uj ui_j
                f[3 * h + slot++] = (float)qdot4(a, b);    // scalar part of a b^+
            }
    }
    for (int k = 0; k < CIN; ++k)
        feat[(size_t)site * CIN + k] = f[k];
}

__device__ __forceinline__ __bf16 to_bf16(float v)
{
    return (__bf16)v;   // round to nearest even
}

// out[s][co] = tanh(b[co] + sum_{tap,ci} bf16(in[s+tap][ci]) bf16(W[tap][ci][co])), CI = 8 or 32.
// 256 threads = 4 waves, each wave 16 sites x 32 channels (two 16x16 tiles).
// MFMA 16x16x32 bf16: lane l holds A[l%16][8(l/16)+j], B[8(l/16)+j][l%16],
// and D[4(l/16)+j][l%16].  K index = tap * CI + ci.
template <int CI>
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float *in, const float *W, const float *bias, float *out,
                                                        Geom g, uint32_t nsites)
{
    __shared__ __bf16 wt[NTAP * CH * CI];   // [tap][co][ci]
    for (int i = threadIdx.x; i < NTAP * CH * CI; i += blockDim.x) {
        const int ci = i % CI, co = (i / CI) % CH, tap = i / (CI * CH);
        wt[i] = to_bf16(W[(tap * CI + ci) * CH + co]);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, row = lane & 15;
    const uint32_t base = (blockIdx.x * 4u + (uint32_t)wave) * 16u;
    if (base >= nsites)
        return;
    const Coord c = coord_of(g, base + (uint32_t)row);
    f32x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    constexpr int KSTEPS = (NTAP * CI + 31) / 32;
    for (int step = 0; step < KSTEPS; ++step) {
        const int tap = (CI == 32) ? step : 4 * step + grp;
        const int ci0 = (CI == 32) ? 8 * grp : 0;
        bf16x8 a, b0, b1;
        if (tap < NTAP) {
            const float4 *src = reinterpret_cast<const float4 *>(in + (size_t)tap_neighbour(g, c, tap, 1) * CI + ci0);
            const float4 v0 = src[0], v1 = src[1];
            a[0] = to_bf16(v0.x); a[1] = to_bf16(v0.y); a[2] = to_bf16(v0.z); a[3] = to_bf16(v0.w);
            a[4] = to_bf16(v1.x); a[5] = to_bf16(v1.y); a[6] = to_bf16(v1.z); a[7] = to_bf16(v1.w);
            const __bf16 *w0 = wt + (tap * CH + row) * CI + ci0;
            const __bf16 *w1 = wt + (tap * CH + 16 + row) * CI + ci0;
            for (int j = 0; j < 8; ++j) {
                b0[j] = w0[j];
                b1[j] = w1[j];
            }
        } else {
            for (int j = 0; j < 8; ++j) {
                a[j] = (__bf16)0.0f;
                b0[j] = (__bf16)0.0f;
                b1[j] = (__bf16)0.0f;
            }
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
    }
    for (int j = 0; j < 4; ++j) {
        const uint32_t site = base + 4u * (uint32_t)grp + (uint32_t)j;
        out[(size_t)site * CH + row] = tanhf(acc0[j] + bias[row]);
        out[(size_t)site * CH + 16 + row] = tanhf(acc1[j] + bias[16 + row]);
    }
}

// dz_in[s][ci] = (1 - a_in[s][ci]^2) sum_{tap,co} bf16(dz[s-tap][co]) bf16(W[tap][ci][co]).
__global__ __launch_bounds__(256) void conv_dgrad_kernel(const float *dz, const float *W, const float *a_in, float *dz_in,
                                                          Geom g, uint32_t nsites)
{
    __shared__ __bf16 w[NTAP * CH * CH];    // [tap][ci][co]
    for (int i = threadIdx.x; i < NTAP * CH * CH; i += blockDim.x)
        w[i] = to_bf16(W[i]);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, row = lane & 15;
    const uint32_t base = (blockIdx.x * 4u + (uint32_t)wave) * 16u;
    if (base >= nsites)
        return;
    const Coord c = coord_of(g, base + (uint32_t)row);
    f32x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    for (int tap = 0; tap < NTAP; ++tap) {
        const float4 *src = reinterpret_cast<const float4 *>(dz + (size_t)tap_neighbour(g, c, tap, -1) * CH + 8 * grp);
        const float4 v0 = src[0], v1 = src[1];
        bf16x8 a, b0, b1;
        a[0] = to_bf16(v0.x); a[1] = to_bf16(v0.y); a[2] = to_bf16(v0.z); a[3] = to_bf16(v0.w);
        a[4] = to_bf16(v1.x); a[5] = to_bf16(v1.y); a[6] = to_bf16(v1.z); a[7] = to_bf16(v1.w);
        const __bf16 *w0 = w + (tap * CH + row) * CH + 8 * grp;        // ci = row, co = 8 grp + j
        const __bf16 *w1 = w + (tap * CH + 16 + row) * CH + 8 * grp;   // ci = 16 + row
        for (int j = 0; j < 8; ++j) {
            b0[j] = w0[j];
            b1[j] = w1[j];
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
    }
    for (int j = 0; j < 4; ++j) {
        const uint32_t site = base + 4u * (uint32_t)grp + (uint32_t)j;
        const float a0 = a_in[(size_t)site * CH + row], a1 = a_in[(size_t)site * CH + 16 + row];
        dz_in[(size_t)site * CH + row] = acc0[j] * (1.0f - a0 * a0);
        dz_in[(size_t)site * CH + 16 + row] = acc1[j] * (1.0f - a1 * a1);
    }
}

// Partial weight gradients over a chunk of kChunk sites for one tap:
// part[chunk][tap][ci][co] = sum_s bf16(in[s+tap][ci]) bf16(dz[s][co]).
// One wave per (chunk, tap); A[m=ci][k=site], B[k=site][n=co] staged in LDS.
constexpr uint32_t kChunk = 512;

template <int CI>
__global__ __launch_bounds__(64) void conv_wgrad_kernel(const float *in, const float *dz, float *part, Geom g,
                                                         uint32_t nsites)
{
    __shared__ __bf16 ta[32][CI];
    __shared__ __bf16 tb[32][CH];
    const int lane = threadIdx.x, grp = lane >> 4, row = lane & 15;
    const int tap = blockIdx.y;
    const uint32_t chunk = blockIdx.x;
    constexpr int MT = (CI + 15) / 16;
    f32x4 acc[MT][2];
    for (int m = 0; m < MT; ++m)
        for (int nt = 0; nt < 2; ++nt)
            acc[m][nt] = {0, 0, 0, 0};
    for (uint32_t s0 = chunk * kChunk; s0 < (chunk + 1) * kChunk && s0 < nsites; s0 += 32) {
        __syncthreads();
        for (int i = lane; i < 32 * CI; i += 64) {
            const int sl = i / CI, ci = i % CI;
            const Coord c = coord_of(g, s0 + (uint32_t)sl);
            ta[sl][ci] = to_bf16(in[(size_t)tap_neighbour(g, c, tap, 1) * CI + ci]);
        }
        for (int i = lane; i < 32 * CH; i += 64)
            tb[i / CH][i % CH] = to_bf16(dz[(size_t)(s0 + (uint32_t)(i / CH)) * CH + i % CH]);
        __syncthreads();
        bf16x8 b0, b1;
        for (int j = 0; j < 8; ++j) {
            b0[j] = tb[8 * grp + j][row];
            b1[j] = tb[8 * grp + j][16 + row];
        }
        for (int m = 0; m < MT; ++m) {
            bf16x8 a;
            const int ci = 16 * m + row;
            for (int j = 0; j < 8; ++j)
                a[j] = (ci < CI) ? ta[8 * grp + j][ci < CI ? ci : 0] : (__bf16)0.0f;
            acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[m][0], 0, 0, 0);
            acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[m][1], 0, 0, 0);
        }
    }
    float *dst = part + ((size_t)chunk * NTAP + (size_t)tap) * CI * CH;
    for (int m = 0; m < MT; ++m)
        for (int j = 0; j < 4; ++j) {
            const int ci = 16 * m + 4 * grp + j;
            if (ci < CI) {
                dst[ci * CH + row] = acc[m][0][j];
                dst[ci * CH + 16 + row] = acc[m][1][j];
            }
        }
}

// out[i] = sum_chunk part[chunk][i] in chunk order.
__global__ __launch_bounds__(256) void sum_chunks_kernel(const float *part, uint32_t nchunk, uint32_t width, float *out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= width)
        return;
    float s = 0.0f;
    for (uint32_t c = 0; c < nchunk; ++c)
        s += part[(size_t)c * width + i];
    out[i] = s;
}

// y[s][d] = bv[d] + sum_c V[d][c] a3[s][c].
__global__ __launch_bounds__(256) void head_fwd_kernel(const float *a3, const float *V, const float *bv, float *y,
                                                        uint32_t nsites)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsites)
        return;
    for (int d = 0; d < NDIR; ++d) {
        float acc = bv[d];
        for (int c = 0; c < CH; ++c)
            acc += V[d * CH + c] * a3[(size_t)s * CH + c];
        y[(size_t)s * NDIR + d] = acc;
    }
}

// Per site: loss term -log q(T|M) and dL/dy (L = mean over sites).
template <class T>
__global__ __launch_bounds__(256) void loss_grad_kernel(Links<T> U, Geom g, double beta, const float *y, float *dy,
                                                         double *loss_part, uint32_t nsites)
{
    __shared__ double red[256];
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (e < nsites) {
        const Quat<double> Te = load_d(U, 3, e, g);
        Quat<double> S[6];
        double c[6];
        Quat<double> M = {0, 0, 0, 0};
        for (int d = 0; d < 6; ++d) {
            uint32_t o;
            S[d] = block_piece(U, g, e, Te, d, o);
            c[d] = mean_field_coefficient(beta, qdot4(S[d], S[d])) * exp((double)y[(size_t)e * 6 + d]);
            M = {M.w + c[d] * S[d].w, M.x + c[d] * S[d].x, M.y + c[d] * S[d].y, M.z + c[d] * S[d].z};
        }
        const double k = sqrt(qdot4(M, M));
        l = -(half_tr(Te, M) - log_z(k));
        const double r = k > 0.0 ? bessel_ratio(k) : 0.0;
        const double inv = 1.0 / (double)nsites;
        for (int d = 0; d < 6; ++d) {
            const double dot = k > 0.0 ? qdot4(M, S[d]) / k : 0.0;
            dy[(size_t)e * 6 + d] = (float)(-(half_tr(Te, S[d]) - r * dot) * c[d] * inv);
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss_part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void loss_total_kernel(const double *part, uint32_t n, uint32_t nsites, double *loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += 256)
        s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *loss = red[0] / (double)nsites;
}

// Head backward per site: dz3 = (dy V) (1 - a3^2); per-block partials of
// dV[d][c] = sum_s dy[s][d] a3[s][c] and dbv[d] = sum_s dy[s][d].
__global__ __launch_bounds__(256) void head_bwd_kernel(const float *dy, const float *a3, const float *V, float *dz3,
                                                        float *part, uint32_t nsites)
{
    __shared__ float red[256];
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    float dys[NDIR] = {0, 0, 0, 0, 0, 0};
    float av[CH];
    for (int c = 0; c < CH; ++c)
        av[c] = 0.0f;
    if (s < nsites) {
        for (int d = 0; d < NDIR; ++d)
            dys[d] = dy[(size_t)s * NDIR + d];
        for (int c = 0; c < CH; ++c) {
            av[c] = a3[(size_t)s * CH + c];
            float acc = 0.0f;
            for (int d = 0; d < NDIR; ++d)
                acc += dys[d] * V[d * CH + c];
            dz3[(size_t)s * CH + c] = acc * (1.0f - av[c] * av[c]);
        }
    }
    float *dst = part + (size_t)blockIdx.x * (NDIR * CH + NDIR);
    for (int d = 0; d < NDIR; ++d) {
        for (int c = 0; c <= CH; ++c) {
            red[threadIdx.x] = dys[d] * (c < CH ? av[c] : 1.0f);
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w)
                    red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0)
                dst[c < CH ? d * CH + c : NDIR * CH + d] = red[0];
            __syncthreads();
        }
    }
}

// Per-block partial column sums of dz[s][co] (bias gradients).
__global__ __launch_bounds__(256) void bias_part_kernel(const float *dz, float *part, uint32_t nsites)
{
    __shared__ float red[256];
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = 0; c < CH; ++c) {
        red[threadIdx.x] = s < nsites ? dz[(size_t)s * CH + c] : 0.0f;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            part[(size_t)blockIdx.x * CH + c] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void adam_kernel(float *p, const float *grad, float *m, float *v, uint32_t n, float lr,
                                                    float b1, float b2, float eps, float c1, float c2)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static Geom geom_of(const LaunchArgs &a)
{
    return make_geom(a.n, -1); // plain walk; the learned kernels index sites directly
}

template <class T>
static Links<T> links_of(const LaunchArgs &a)
{
    Links<T> L;
    L.p = reinterpret_cast<decltype(L.p)>(a.links);
    L.stride = plane_stride((uint32_t)(a.volume / 2), sizeof(T) == 8);
    return L;
}

int param_count()
{
    return NPARAM;
}

WorkLayout work_layout(const int32_t n[4])
{
    const uint64_t N = (uint64_t)n[0] * n[1] * n[2] * n[3];
    WorkLayout w = {};
    auto r256 = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    uint64_t off = 0;
    w.feat = off;
    off += r256(N * CIN * 4);
    w.a1 = off;
    off += r256(N * CH * 4);
    w.a2 = off;
    off += r256(N * CH * 4);
    w.a3 = off;
    off += r256(N * CH * 4);
    w.y = off;
    off += r256(N * NDIR * 4);
    w.dy = off;
    off += r256(N * NDIR * 4);
    w.dz_a = off;
    off += r256(N * CH * 4);
    w.dz_b = off;
    off += r256(N * CH * 4);
    const uint64_t nchunk = (N + kChunk - 1) / kChunk;
    const uint64_t nblk = (N + 255) / 256;
    uint64_t part = nchunk * NTAP * CH * CH;
    if (nblk * (NDIR * CH + NDIR) > part)
        part = nblk * (NDIR * CH + NDIR);
    w.part = off;
    off += r256(part * 4);
    w.loss_part = off;
    off += r256(nblk * 8);
    w.total = off;
    return w;
}

template <class T>
static void forward_t(const LaunchArgs &a, const float *params, char *work, const WorkLayout &w, float *y,
                      hipStream_t st)
{
    const Geom g = geom_of(a);
    const uint32_t N = (uint32_t)a.volume;
    float *feat = reinterpret_cast<float *>(work + w.feat);
    float *a1 = reinterpret_cast<float *>(work + w.a1);
    float *a2 = reinterpret_cast<float *>(work + w.a2);
    float *a3 = reinterpret_cast<float *>(work + w.a3);
    features_kernel<T><<<(N + 255) / 256, 256, 0, st>>>(links_of<T>(a), g, feat);
    const uint32_t cblocks = (N + 63) / 64;
    conv_fwd_kernel<CIN><<<cblocks, 256, 0, st>>>(feat, params + OFF_W1, params + OFF_B1, a1, g, N);
    conv_fwd_kernel<CH><<<cblocks, 256, 0, st>>>(a1, params + OFF_W2, params + OFF_B2, a2, g, N);
    conv_fwd_kernel<CH><<<cblocks, 256, 0, st>>>(a2, params + OFF_W3, params + OFF_B3, a3, g, N);
    head_fwd_kernel<<<(N + 255) / 256, 256, 0, st>>>(a3, params + OFF_V, params + OFF_BV, y, N);
}

void launch_forward(const LaunchArgs &a, const float *params, char *work, float *y, hipStream_t st)
{
    const WorkLayout w = work_layout(a.n);
    if (a.prec == kF32)
        forward_t<float>(a, params, work, w, y, st);
    else
        forward_t<double>(a, params, work, w, y, st);
}

template <class T>
static void loss_grad_t(const LaunchArgs &a, double beta, const float *params, char *work, float *grad, double *loss,
                        hipStream_t st)
{
    const WorkLayout w = work_layout(a.n);
    const Geom g = geom_of(a);
    const uint32_t N = (uint32_t)a.volume;
    float *y = reinterpret_cast<float *>(work + w.y);
    forward_t<T>(a, params, work, w, y, st);
    float *feat = reinterpret_cast<float *>(work + w.feat);
    float *a1 = reinterpret_cast<float *>(work + w.a1);
    float *a2 = reinterpret_cast<float *>(work + w.a2);
    float *a3 = reinterpret_cast<float *>(work + w.a3);
    float *dy = reinterpret_cast<float *>(work + w.dy);
    float *dza = reinterpret_cast<float *>(work + w.dz_a);
    float *dzb = reinterpret_cast<float *>(work + w.dz_b);
    float *part = reinterpret_cast<float *>(work + w.part);
    double *lp = reinterpret_cast<double *>(work + w.loss_part);
    const uint32_t nblk = (N + 255) / 256;
    const uint32_t nchunk = (N + kChunk - 1) / kChunk;
    const uint32_t cblocks = (N + 63) / 64;
    loss_grad_kernel<T><<<nblk, 256, 0, st>>>(links_of<T>(a), g, beta, y, dy, lp, N);
    loss_total_kernel<<<1, 256, 0, st>>>(lp, nblk, N, loss);
    // head
    head_bwd_kernel<<<nblk, 256, 0, st>>>(dy, a3, params + OFF_V, dza, part, N);
    sum_chunks_kernel<<<1, 256, 0, st>>>(part, nblk, NDIR * CH + NDIR, grad + OFF_V);   // V then bv (contiguous)
    // layer 3: dz3 in dza
    conv_wgrad_kernel<CH><<<dim3(nchunk, NTAP), 64, 0, st>>>(a2, dza, part, g, N);
    sum_chunks_kernel<<<(NTAP * CH * CH + 255) / 256, 256, 0, st>>>(part, nchunk, NTAP * CH * CH, grad + OFF_W3);
    bias_part_kernel<<<nblk, 256, 0, st>>>(dza, part, N);
    sum_chunks_kernel<<<1, 256, 0, st>>>(part, nblk, CH, grad + OFF_B3);
    conv_dgrad_kernel<<<cblocks, 256, 0, st>>>(dza, params + OFF_W3, a2, dzb, g, N);
    // layer 2: dz2 in dzb
    conv_wgrad_kernel<CH><<<dim3(nchunk, NTAP), 64, 0, st>>>(a1, dzb, part, g, N);
    sum_chunks_kernel<<<(NTAP * CH * CH + 255) / 256, 256, 0, st>>>(part, nchunk, NTAP * CH * CH, grad + OFF_W2);
    bias_part_kernel<<<nblk, 256, 0, st>>>(dzb, part, N);
    sum_chunks_kernel<<<1, 256, 0, st>>>(part, nblk, CH, grad + OFF_B2);
    conv_dgrad_kernel<<<cblocks, 256, 0, st>>>(dzb, params + OFF_W2, a1, dza, g, N);
    // layer 1: dz1 in dza
    conv_wgrad_kernel<CIN><<<dim3(nchunk, NTAP), 64, 0, st>>>(feat, dza, part, g, N);
    sum_chunks_kernel<<<(NTAP * CIN * CH + 255) / 256, 256, 0, st>>>(part, nchunk, NTAP * CIN * CH, grad + OFF_W1);
    bias_part_kernel<<<nblk, 256, 0, st>>>(dza, part, N);
    sum_chunks_kernel<<<1, 256, 0, st>>>(part, nblk, CH, grad + OFF_B1);
}

void launch_loss_grad(const LaunchArgs &a, double beta, const float *params, char *work, float *grad, double *loss,
                      hipStream_t st)
{
    if (a.prec == kF32)
        loss_grad_t<float>(a, beta, params, work, grad, loss, st);
    else
        loss_grad_t<double>(a, beta, params, work, grad, loss, st);
}

void launch_adam(float *p, const float *grad, float *m, float *v, uint32_t n, int step, float lr, float b1, float b2,
                 float eps, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    adam_kernel<<<(n + 255) / 256, 256, 0, st>>>(p, grad, m, v, n, lr, b1, b2, eps, c1, c2);
}

void launch_block_move(const LaunchArgs &a, double beta, uint64_t seed, uint32_t step, int parity, int colour,
                       const float *y, uint32_t *accepted, hipStream_t st)
{
    const Geom g = geom_of(a);
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const uint32_t c1 = 3u + 4u * 2u + 16u * (uint32_t)a.lattice_id;
    const uint32_t c2 = 16u * step + 8u * (uint32_t)parity + (uint32_t)colour;
    const uint32_t count = g.vs / 16u * (uint32_t)a.n[3];
    const uint32_t blocks = (count * 8u + 63) / 64;   // 8 lanes per centre
    if (a.prec == kF32)
        block_move_kernel<float><<<blocks, 64, 0, st>>>(links_of<float>(a), g, beta, k0, k1, c1, c2, parity, colour, y,
                                                        accepted, a.flags);
    else
        block_move_kernel<double><<<blocks, 64, 0, st>>>(links_of<double>(a), g, beta, k0, k1, c1, c2, parity, colour,
                                                         y, accepted, a.flags);
}

} // namespace lp
} // namespace su2

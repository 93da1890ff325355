// su2_heatbath.hpp -- the heat bath's sampling of one link from its staple
// (shared by the global-memory and the LDS-staged update kernels, so both
// form every new link with the same arithmetic).
#pragma once

#include "su2_device.hpp"

namespace su2 {

// ---------------------------------------------------------------------------
// Heat bath for one class.  With k = |V|, Vhat = V/k and alpha = beta k, the
// new link is W Vhat^dagger where W has density ~ exp(alpha w0) w.r.t. Haar
// measure: w0 by Kennedy-Pendleton (alpha >= 2) or Creutz (alpha < 2), the
// vector part isotropic with length sqrt(1 - w0^2).  Random numbers: counter
// (site, c1, sweep, 4*attempt + draw); draws 0,1 feed sampler attempt
// `attempt`, draw 2 (of attempt 0) the direction.
//
// One attempt of the sampler.  FP64 links: everything in FP64.  FP32 links:
// uniforms from 23 bits, the logarithms and cosines in FP32, and lambda^2,
// the accept test, x0 = 1 - 2 lambda^2 and |x| = 2 sqrt(lambda^2 (1 -
// lambda^2)) assembled in FP64; lambda^2 carries 1 - x0 directly, so x0 near
// 1 suffers no cancellation.  The Creutz branch (alpha < 2) is FP64 for both.
// ---------------------------------------------------------------------------
template <class T>
struct KP;

// One attempt from its two Philox outputs: ra = counter 4a, rb = 4a + 1.
template <>
struct KP<double> {
    __device__ static __forceinline__ bool attempt(double inv2a, const U32x4 &ra, const U32x4 &rb, double &x0,
                                                   double &xlen)
    {
        double u1, u2, u3, u4;
        Draw<double>::two(ra, u1, u2);
        Draw<double>::two(rb, u3, u4);
        const double c = cos((2.0 * kPi) * u2);
        const double lam2 = -(log(u1) + c * c * log(u3)) * inv2a;
        if (lam2 <= 1.0 && u4 * u4 <= 1.0 - lam2) {
            x0 = 1.0 - 2.0 * lam2;
            xlen = 2.0 * sqrt(lam2 * (1.0 - lam2));
            return true;
        }
        return false;
    }
};

template <>
struct KP<float> {
    __device__ static __forceinline__ bool attempt(double inv2a, const U32x4 &ra, const U32x4 &rb, double &x0,
                                                   double &xlen)
    {
        const float u1 = u01_f32(ra.r0), u2 = u01_f32(ra.r2);
        const float u3 = u01_f32(rb.r0), u4 = u01_f32(rb.r2);
        const float c = cospif(2.0f * u2);
        const double lam2 = -((double)logf(u1) + (double)(c * c) * (double)logf(u3)) * inv2a;
        const double u4d = (double)u4;
        if (lam2 <= 1.0 && u4d * u4d <= 1.0 - lam2) {
            x0 = 1.0 - 2.0 * lam2;
            xlen = 2.0 * sqrt(lam2 * (1.0 - lam2));
            return true;
        }
        return false;
    }
};

// One Creutz attempt from its Philox output ra (counter 4a).
template <class T>
__device__ __forceinline__ bool creutz_attempt(double alpha, const U32x4 &ra, double &x0, double &xlen)
{
    double u1, u2;
    Draw<T>::two(ra, u1, u2);
    double t;
    if (alpha < 1e-8) {
        t = 2.0 * u1 - 1.0;
    } else {
        const double e = exp(-2.0 * alpha);
        t = 1.0 + log(e + u1 * (1.0 - e)) / alpha;
    }
    if (u2 * u2 <= 1.0 - t * t) {
        x0 = t;
        xlen = sqrt(fmax(0.0, 1.0 - t * t));
        return true;
    }
    return false;
}

// An attempt from its random words (ra, rb as above; Creutz uses ra only).
template <class T>
__device__ __forceinline__ bool sampler_attempt_drawn(double alpha, double inv2a, const U32x4 &ra, const U32x4 &rb,
                                                      double &x0, double &xlen)
{
    if (alpha >= 2.0)
        return KP<T>::attempt(inv2a, ra, rb, x0, xlen);
    return creutz_attempt<T>(alpha, ra, x0, xlen);
}

// Attempt a of the link at `site`, drawing its words.
template <class T>
__device__ __forceinline__ bool sampler_attempt(double alpha, double inv2a, uint32_t site, uint32_t c1,
                                                uint32_t sweep, uint32_t a, uint32_t k0, uint32_t k1, double &x0,
                                                double &xlen)
{
    const U32x4 ra = philox(site, c1, sweep, 4u * a, k0, k1);
    if (alpha >= 2.0)
        return KP<T>::attempt(inv2a, ra, philox(site, c1, sweep, 4u * a + 1u, k0, k1), x0, xlen);
    return creutz_attempt<T>(alpha, ra, x0, xlen);
}

// Direction of the vector part: cos(theta) = 2 u5 - 1, phi = 2 pi u6.
template <class T>
struct Direction;

template <>
struct Direction<double> {
    __device__ static __forceinline__ Quat<double> make(double x0, double xlen, const U32x4 &r)
    {
        double u5, u6;
        Draw<double>::two(r, u5, u6);
        const double cth = 2.0 * u5 - 1.0;
        const double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
        double sph, cph;
        sincos((2.0 * kPi) * u6, &sph, &cph);
        return {x0, xlen * sth * cph, xlen * sth * sph, xlen * cth};
    }
};

template <>
struct Direction<float> {
    __device__ static __forceinline__ Quat<float> make(double x0, double xlen, const U32x4 &r)
    {
        const float u5 = u01_f32(r.r0), u6 = u01_f32(r.r2);
        const float cth = 2.0f * u5 - 1.0f;
        const float sth = sqrtf(fmaxf(0.0f, 1.0f - cth * cth));
        float sph, cph;
        sincospif(2.0f * u6, &sph, &cph);
        const float xl = (float)xlen;
        return {(float)x0, xl * sth * cph, xl * sth * sph, xl * cth};
    }
};

// Block-shared state of the compaction of rejected lanes, for blocks of NT
// threads (one per kernel, so that a kernel running several classes holds
// it once).
template <int NT>
struct HbSharedT {
    uint32_t queue[NT];
    uint32_t site[NT];
    double alpha[NT];
    double x0[NT];
    double xlen[NT];
    uint32_t wcount[NT / 64];
};
using HbShared = HbSharedT<kBlock>;

// What the heat bath takes from the staple V: Vhat = V/|V| (1 if V = 0) and
// alpha = beta |V|; false (and the non-finite flag) if |V| is not finite,
// in which case the link is kept.
template <class T>
__device__ __forceinline__ bool hb_staple_law(const Quat<T> &V, double beta, uint32_t *flags, Quat<T> &Vh,
                                              double &alpha)
{
    const T k = sqrt(V.w * V.w + V.x * V.x + V.y * V.y + V.z * V.z);
    if (!isfinite(k)) {
        atomicOr(flags, kFlagNonFinite);
        return false;
    }
    if (k > T(0)) {
        const T inv = T(1) / k;
        Vh = {V.w * inv, V.x * inv, V.y * inv, V.z * inv};
    }
    alpha = beta * (double)k;
    return true;
}

// w0 (as x0 and |x| = xlen) for every lane of a block of NT threads that
// needs one: attempt 0 from the words r0, r1 drawn by the caller, then the
// lanes that rejected are compacted block-wide through LDS (wave ballots,
// no atomics) and retried by as few lanes as there are rejections, so a
// wave no longer idles until its slowest lane accepts.  A link's attempt
// sequence, and so its result, does not depend on which lane runs it.
// Every thread of the block must call it (it holds two block barriers).
// Returns whether the lane has a sample; a lane that exhausts the attempt
// cap sets the cap flag and keeps its link.
template <class T, int NT>
__device__ __forceinline__ bool hb_sample(bool need, double alpha, uint32_t site, const U32x4 &r0, const U32x4 &r1,
                                          uint32_t c1, uint32_t sweep, uint32_t k0, uint32_t k1, uint32_t *flags,
                                          HbSharedT<NT> &sh, double &x0, double &xlen)
{
    const uint32_t tid = threadIdx.x;
    const double inv2a = 1.0 / (2.0 * fmax(alpha, 1.0));

    // attempt 0 on every lane
    x0 = 0.0;
    xlen = 0.0;
    bool ok = false;
    if (need)
        ok = sampler_attempt_drawn<T>(alpha, inv2a, r0, r1, x0, xlen);
    const bool retry = need && !ok;

    // compact the rejected lanes of the block
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint64_t mask = __ballot(retry);
    if (retry) {
        const uint32_t rank = __popcll(mask & ((1ull << lane) - 1ull));
        sh.queue[wave * 64u + rank] = tid;
        sh.site[tid] = site;
        sh.alpha[tid] = alpha;
    }
    if (lane == 0)
        sh.wcount[wave] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w)
        total += sh.wcount[w];
    for (uint32_t qi = tid; qi < total; qi += NT) {
        uint32_t w = 0, r = qi;
        while (r >= sh.wcount[w]) {
            r -= sh.wcount[w];
            ++w;
        }
        const uint32_t src = sh.queue[w * 64u + r];
        const double a_src = sh.alpha[src];
        const double inv2a_src = 1.0 / (2.0 * fmax(a_src, 1.0));
        double qx0 = 0.0, qxl = -1.0;
        for (uint32_t a = 1; a < kMaxAttempts; ++a)
            if (sampler_attempt<T>(a_src, inv2a_src, sh.site[src], c1, sweep, a, k0, k1, qx0, qxl))
                break;
        sh.x0[src] = qx0;
        sh.xlen[src] = qxl;
    }
    __syncthreads();
    if (retry) {
        x0 = sh.x0[tid];
        xlen = sh.xlen[tid];
        ok = xlen >= 0.0;
        if (!ok)
            atomicOr(flags, kFlagCap);
    }
    return ok;
}

} // namespace su2

// Device helpers shared by the Vecchia kernels: covariance closed forms,
// parameter unpacking, deterministic wave/block reductions and compensated
// (double-double) accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exp_table.h"

namespace vecchia {

constexpr int kWave = 64;                     // CDNA wavefront width
constexpr double kLog2Pi = 1.8378770664093454835606594728112;
constexpr int64_t kNoFailure = INT64_MAX;     // "no failing point" sentinel in partial status words
constexpr int kChunk = 16;                    // conditionals summed per partial (fixed: fixes the summation order)

// Covariance parameters as the kernels use them; alpha is the exponent of
// the power exponential (unused by the Matern codes).
struct Params {
    double sigma2, beta, tau2, inv_beta, alpha;
    bool valid;
};

__device__ inline Params load_params(const double *__restrict__ theta, double alpha = 1.0) {
    Params p;
    p.sigma2 = theta[0];
    p.beta = theta[1];
    p.tau2 = theta[2];
    p.valid = (p.sigma2 > 0.0) && (p.beta > 0.0) && (p.tau2 >= 0.0) && isfinite(p.sigma2) && isfinite(p.beta) &&
              isfinite(p.tau2);
    p.inv_beta = 1.0 / p.beta;
    p.alpha = alpha;
    return p;
}

// Covariance codes of the kernels: KC = family + 4 * metric, family 0, 1, 2
// for Matern nu = 1/2, 3/2, 5/2 (Eq. (2)) and 3 for the power exponential
// sigma2 exp(-d^alpha / beta) (Sec. V-C); metric 0 Euclidean on (x, y), 1
// great-circle on (longitude, latitude) in degrees, in kilometres.
__host__ __device__ constexpr int kc_family(int KC) { return KC & 3; }
__host__ __device__ constexpr bool kc_gcd(int KC) { return (KC >> 2) != 0; }
constexpr double kEarthRadiusKm = 6371.0;
constexpr double kDeg2Rad = 0.017453292519943295769236907684886;

// e^{-r} for r >= 0.  Range reduction x = -r = k ln2 + f with |f| <= ln2/2
// (ln2 split into a head with trailing zero bits and a tail, so k*ln2_head is
// exact), e^f by its Taylor polynomial of degree 13 (truncation below 6e-18
// relative), then scaling by 2^k.  Results below the double range flush to
// 0; NaN propagates.  About 19 instructions, no table.
__device__ __forceinline__ double exp_neg(double r) {
    double x = -r;
    x = (x < -745.5) ? -745.5 : x;  // keeps NaN (the comparison is false)
    const double k = __builtin_rint(x * 1.4426950408889634074);
    double f = fma(k, -6.93147180369123816490e-01, x);
    f = fma(k, -1.90821492927058770002e-10, f);
    double p = 1.0 / 6227020800.0;          // 1/13!
    p = fma(p, f, 1.0 / 479001600.0);       // 1/12!
    p = fma(p, f, 1.0 / 39916800.0);        // 1/11!
    p = fma(p, f, 1.0 / 3628800.0);         // 1/10!
    p = fma(p, f, 1.0 / 362880.0);          // 1/9!
    p = fma(p, f, 1.0 / 40320.0);           // 1/8!
    p = fma(p, f, 1.0 / 5040.0);            // 1/7!
    p = fma(p, f, 1.0 / 720.0);             // 1/6!
    p = fma(p, f, 1.0 / 120.0);             // 1/5!
    p = fma(p, f, 1.0 / 24.0);              // 1/4!
    p = fma(p, f, 1.0 / 6.0);               // 1/3!
    p = fma(p, f, 0.5);
    p = fma(p, f, 1.0);
    p = fma(p, f, 1.0);
    return __builtin_ldexp(p, (int)k);
}

// sqrt(s) for a squared distance s >= 0: hardware reciprocal square root and
// two coupled Newton (Goldschmidt) refinements of sqrt and 1/(2 sqrt), as in
// a correctly rounded software sqrt, without the denormal rescaling: s below
// 1e-290 (coincident points up to 1e-145) gives 0.  NaN propagates.
__device__ __forceinline__ double sqrt_dist(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y;
    double h = 0.5 * y;
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, s);
    g = fma(d, h, g);
    return (s > 1e-290) ? g : ((s >= 0.0) ? 0.0 : s);
}

// e^{-r} for r >= 0 by Tang's table-driven method: -r = (64 k + j) ln2/64 + f
// with |f| <= ln2/128, so e^{-r} = 2^k 2^{j/64} e^f.  `tab` holds 2^{j/64}
// as hi + lo pairs (kExp2Frac64, staged in LDS by the caller); q = e^f - 1 by
// its Taylor polynomial of degree 6 (truncation below 3e-20), and the result
// hi + (lo + hi q) rounds once at the end, so the error stays just above half
// an ulp.  ln2/64 is split into a 36-bit head (n ln2/64 exact for |n| < 2^17)
// and a tail.  Arguments beyond 746 give 0; a NaN argument gives 0 as well,
// so callers validate their inputs instead.
__device__ __forceinline__ double exp_neg_tab(double r, const double *tab) {
    const double x = fmax(-r, -746.0);
    const double nf = __builtin_rint(x * 0x1.71547652b82fep+6);  // 64 / ln2
    const int n = (int)nf;
    double f = fma(nf, -0x1.62e42fefa0000p-7, x);  // head of ln2/64
    f = fma(nf, -0x1.cf79abc9e3b3ap-46, f);        // tail of ln2/64
    double q = fma(f, 1.0 / 720.0, 1.0 / 120.0);
    q = fma(q, f, 1.0 / 24.0);
    q = fma(q, f, 1.0 / 6.0);
    q = fma(q, f, 0.5);
    q = fma(q, f, 1.0);
    q *= f;  // e^f - 1
    const double2 t = *reinterpret_cast<const double2 *>(tab + 2 * (n & 63));
    return __builtin_ldexp(t.x + fma(t.x, q, t.y), n >> 6);
}

// sqrt(s) for a squared distance s >= 0 without a branch: s is raised by
// 2^-1000 (below half an ulp of any s >= 2^-946, so other distances are
// unchanged) so that the reciprocal square root never sees 0; coincident
// points get distance 2^-500, whose covariance is the zero-distance value to
// the last bit.  Then the coupled Newton refinement of sqrt_dist.
__device__ __forceinline__ double sqrt_pos(double s) {
    s += 0x1p-1000;
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y;
    double h = 0.5 * y;
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, s);
    return fma(d, h, g);
}

// sin x.  Neighbouring points give half-angle differences far below 0.25
// rad, where the Taylor polynomial to x^13 is used (truncation below 1e-21
// relative, Horner in x^2, one rounding at the end); larger arguments take
// the library sine.
__device__ __forceinline__ double sin_short(double x) {
    if (fabs(x) <= 0.25) {
        const double x2 = x * x;
        double q = 1.0 / 6227020800.0;   // 1/13!
        q = fma(q, x2, -1.0 / 39916800.0);  // -1/11!
        q = fma(q, x2, 1.0 / 362880.0);     // 1/9!
        q = fma(q, x2, -1.0 / 5040.0);      // -1/7!
        q = fma(q, x2, 1.0 / 120.0);        // 1/5!
        q = fma(q, x2, -1.0 / 6.0);         // -1/3!
        return fma(x * x2, q, x);
    }
    return sin(x);
}

// asin(sqrt(h)) for 0 <= h <= 1.  For h <= 0.01 (great-circle distances up
// to about 1270 km) the series asin s = s (1 + sum_n c_n s^2n), c_n =
// (2n)! / (4^n (n!)^2 (2n + 1)), to n = 8 (truncation below 2e-18
// relative); otherwise the library asin.
__device__ __forceinline__ double asin_sqrt(double h) {
    const double s = sqrt(h);
    if (h <= 0.01) {
        double p = 6435.0 / 557056.0;
        p = fma(p, h, 143.0 / 10240.0);
        p = fma(p, h, 231.0 / 13312.0);
        p = fma(p, h, 63.0 / 2816.0);
        p = fma(p, h, 35.0 / 1152.0);
        p = fma(p, h, 5.0 / 112.0);
        p = fma(p, h, 3.0 / 40.0);
        p = fma(p, h, 1.0 / 6.0);
        return fma(s * h, p, s);
    }
    return asin(s);
}

// Great-circle distance in km between (lon, lat) points a and b in degrees,
// given cos(lat) of each: hav(d / R) = hav(dlat) + cos lat_a cos lat_b hav(dlon)
// with hav(t) = sin^2(t / 2), differences taken in degrees first.  Coincident
// points give exactly 0.
__device__ __forceinline__ double gcd_km(double lona, double lata, double ca, double lonb, double latb, double cb) {
    const double s1 = sin_short(0.5 * ((lata - latb) * kDeg2Rad));
    const double s2 = sin_short(0.5 * ((lona - lonb) * kDeg2Rad));
    const double h = fmin(fma(s1, s1, (ca * cb) * (s2 * s2)), 1.0);
    return (2.0 * kEarthRadiusKm) * asin_sqrt(h);
}

// The parameter-free part of the scaled distance: d (Matern) or d^alpha
// (power exponential; alpha = 1 and 2 without the exponential, otherwise
// e^(alpha ln d) with the table exponential, and 0 for d = 0).  alpha is
// fixed per call, so this is shared by every (sigma2, beta, tau2).
template <int KC>
__device__ __forceinline__ double dist_pow(double d, const Params &P, const double *tab) {
    if constexpr (kc_family(KC) == 3) {
        double da;
        if (P.alpha == 1.0) {
            da = d;
        } else if (P.alpha == 2.0) {
            da = d * d;
        } else {
            da = (d > 0.0) ? exp_neg_tab(-(P.alpha * log(d)), tab) : 0.0;
        }
        return da;
    } else {
        return d;
    }
}

// Scaled distance r fed to the closed forms: d / beta (Matern) or
// d^alpha / beta (power exponential).
template <int KC>
__device__ __forceinline__ double cov_scaled(double d, const Params &P, const double *tab) {
    return dist_pow<KC>(d, P, tab) * P.inv_beta;
}

// dist_pow of the distance between points a and b (cos of the latitudes in
// ca, cb for the great-circle codes).  The coordinates must be finite.
template <int KC>
__device__ __forceinline__ double pair_dist_pow(double xa, double ya, double ca, double xb, double yb, double cb,
                                                const Params &P, const double *tab) {
    if constexpr (kc_gcd(KC)) {
        return dist_pow<KC>(gcd_km(xa, ya, ca, xb, yb, cb), P, tab);
    } else {
        const double dx = xa - xb, dy = ya - yb;
        return dist_pow<KC>(sqrt_pos(fma(dx, dx, dy * dy)), P, tab);
    }
}

// Covariance C and, with WITH_D, its beta-derivative from da = dist_pow of
// the pair's distance, using exp_neg_tab.  With r = da / beta the scaled
// distance, the Matern forms are sigma2 m(r) and sigma2 h(r) / beta (h as in
// matern_dbeta_r); the power exponential is sigma2 e^-r with derivative
// sigma2 r e^-r / beta, the nu = 1/2 form.
template <int KC, bool WITH_D>
__device__ __forceinline__ void cov_from_dist(double da, const Params &P, double s2b, const double *tab, double &c,
                                              double &db) {
    double r = da * P.inv_beta;
    constexpr int F = kc_family(KC);
    // for nu = 3/2 and 5/2, r is opaque to the optimiser: 1 + r below could
    // be fused with the product that forms r in one kernel and not in another
    // (it was, for nu = 3/2 on great-circle distances), and kernels that share
    // distances between parameter vectors must give the bits of those that do
    // not
    if constexpr (F == 1 || F == 2) asm volatile("" : "+v"(r));
    const double e = exp_neg_tab(r, tab);
    if constexpr (F == 0 || F == 3) {
        c = P.sigma2 * e;
        if constexpr (WITH_D) db = s2b * (r * e);
    } else if constexpr (F == 1) {
        c = P.sigma2 * ((1.0 + r) * e);
        if constexpr (WITH_D) db = s2b * ((r * r) * e);
    } else {
        c = P.sigma2 * ((1.0 + r * (1.0 + r * (1.0 / 3.0))) * e);
        if constexpr (WITH_D) db = s2b * ((r * r) * (1.0 + r) * (1.0 / 3.0) * e);
    }
}

// Covariance C(d) and, with WITH_D, its beta-derivative for points a and b
// (cos of the latitudes in ca, cb for the great-circle codes).  The
// coordinates must be finite.
template <int KC, bool WITH_D>
__device__ __forceinline__ void cov_pair(double xa, double ya, double ca, double xb, double yb, double cb,
                                         const Params &P, double s2b, const double *tab, double &c, double &db) {
    cov_from_dist<KC, WITH_D>(pair_dist_pow<KC>(xa, ya, ca, xb, yb, cb, P, tab), P, s2b, tab, c, db);
}

// Closed forms in the scaled distance r: Matern, Eq. (2), for half-integer
// smoothness (NU: 0 -> nu = 0.5, 1 -> nu = 1.5, 2 -> nu = 2.5, r = d / beta)
// and the power exponential (NU = 3, r = d^alpha / beta), whose form is the
// nu = 1/2 one.
template <int NU>
__device__ __forceinline__ double matern_r(double r, double sigma2) {
    double e = exp_neg(r);
    if constexpr (NU == 0 || NU == 3) {
        return sigma2 * e;
    } else if constexpr (NU == 1) {
        return sigma2 * ((1.0 + r) * e);
    } else {
        return sigma2 * ((1.0 + r * (1.0 + r * (1.0 / 3.0))) * e);
    }
}

// beta-derivative of the covariance: dC/dbeta = sigma2 h(r) / beta with
//   h = r e^-r (nu = 0.5), r^2 e^-r (nu = 1.5), r^2 (1 + r) e^-r / 3 (nu = 2.5).
template <int NU>
__device__ __forceinline__ double matern_dbeta_r(double r, double sigma2_over_beta) {
    double e = exp_neg(r);
    if constexpr (NU == 0 || NU == 3) {
        return sigma2_over_beta * (r * e);
    } else if constexpr (NU == 1) {
        return sigma2_over_beta * ((r * r) * e);
    } else {
        return sigma2_over_beta * ((r * r) * (1.0 + r) * (1.0 / 3.0) * e);
    }
}

// Both at once (one exponential).
template <int NU>
__device__ __forceinline__ void matern_and_dbeta_r(double r, double sigma2, double sigma2_over_beta, double &c,
                                                   double &db) {
    double e = exp_neg(r);
    if constexpr (NU == 0 || NU == 3) {
        c = sigma2 * e;
        db = sigma2_over_beta * (r * e);
    } else if constexpr (NU == 1) {
        c = sigma2 * ((1.0 + r) * e);
        db = sigma2_over_beta * ((r * r) * e);
    } else {
        c = sigma2 * ((1.0 + r * (1.0 + r * (1.0 / 3.0))) * e);
        db = sigma2_over_beta * ((r * r) * (1.0 + r) * (1.0 / 3.0) * e);
    }
}

__device__ __forceinline__ double dist2d(double ax, double ay, double bx, double by) {
    double dx = ax - bx;
    double dy = ay - by;
    return sqrt_dist(fma(dx, dx, dy * dy));
}

// 2^(j/64) as (hi, lo) pairs in global memory, for code that does not stage
// the table in LDS.
__device__ __forceinline__ const double *exp_table_global() { return reinterpret_cast<const double *>(kExp2Frac64); }

// Scaled distance of a pair under covariance code KC (the unblocked kernel's form).
template <int KC>
__device__ __forceinline__ double cov_r(double xa, double ya, double ca, double xb, double yb, double cb,
                                        const Params &P) {
    if constexpr (kc_gcd(KC)) {
        return cov_scaled<KC>(gcd_km(xa, ya, ca, xb, yb, cb), P, exp_table_global());
    } else {
        return cov_scaled<KC>(dist2d(xa, ya, xb, yb), P, exp_table_global());
    }
}

// Sum over the 64 lanes of a wavefront; fixed butterfly order, every lane gets the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide sum in a fixed order.  `scratch` holds at least NWAVES doubles.
// Must be reached by every thread of the block.  Every thread gets the total.
template <int NWAVES>
__device__ __forceinline__ double block_sum(double v, double *scratch) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) t += scratch[w];
    return t;
}

// Double-double accumulation (Knuth two-sum), used for the final reductions.
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_add(DD a, double b) {
    double s = a.hi + b;
    double bb = s - a.hi;
    double err = (a.hi - (s - bb)) + (b - bb);
    DD r;
    r.hi = s;
    r.lo = a.lo + err;
    double t = r.hi + r.lo;
    r.lo = r.lo - (t - r.hi);
    r.hi = t;
    return r;
}

__device__ __forceinline__ DD dd_add(DD a, DD b) {
    DD r = dd_add(a, b.hi);
    return dd_add(r, b.lo);
}

}  // namespace vecchia

// Device helpers shared by the Vecchia kernels: covariance closed forms,
// parameter unpacking, deterministic wave/block reductions and compensated
// (double-double) accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vecchia {

constexpr int kWave = 64;                     // CDNA wavefront width
constexpr double kLog2Pi = 1.8378770664093454835606594728112;
constexpr int64_t kNoFailure = INT64_MAX;     // "no failing point" sentinel in partial status words
constexpr int kChunk = 16;                    // conditionals summed per partial (fixed: fixes the summation order)

// Covariance parameters as the kernels use them.
struct Params {
    double sigma2, beta, tau2, inv_beta;
    bool valid;
};

__device__ inline Params load_params(const double *__restrict__ theta) {
    Params p;
    p.sigma2 = theta[0];
    p.beta = theta[1];
    p.tau2 = theta[2];
    p.valid = (p.sigma2 > 0.0) && (p.beta > 0.0) && (p.tau2 >= 0.0) && isfinite(p.sigma2) && isfinite(p.beta) &&
              isfinite(p.tau2);
    p.inv_beta = 1.0 / p.beta;
    return p;
}

// Matern covariance, Eq. (2), for half-integer smoothness in closed form.
// NU: 0 -> nu = 0.5, 1 -> nu = 1.5, 2 -> nu = 2.5.  r = distance / beta.
template <int NU>
__device__ __forceinline__ double matern_r(double r, double sigma2) {
    double e = exp(-r);
    if constexpr (NU == 0) {
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
    double e = exp(-r);
    if constexpr (NU == 0) {
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
    double e = exp(-r);
    if constexpr (NU == 0) {
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
    return sqrt(dx * dx + dy * dy);
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

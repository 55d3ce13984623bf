// C ABI and launch logic of the Vecchia log-likelihood library (gfx950).
//
// Pipeline of one evaluation (Algorithm 1, fused):
//   conditional kernel  one workgroup per point i: gathers the neighbours,
//                       builds the covariance block, factors it, solves, forms
//                       l_i (and its gradient) and writes the four values and
//                       a failure flag for i;
//   reduce kernel       every thread adds a fixed chunk of kChunk consecutive
//                       points in ascending order; each workgroup combines its
//                       threads' sums in a fixed tree (double-double);
//   finalize kernel     sums the workgroup partials in a fixed order and writes
//                       l, the gradient and the status.
// All summation orders are fixed, so results are bitwise reproducible
// whatever order the hardware runs the workgroups in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "vecchia.h"
#include "launch.h"

using namespace vecchia;

namespace {

constexpr int kFinalizeThreads = 256;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int kReduceThreads = 256;
constexpr int64_t kPointsPerReduceBlock = (int64_t)kChunk * kReduceThreads;

int64_t num_reduce_blocks(int64_t n) { return (n + kPointsPerReduceBlock - 1) / kPointsPerReduceBlock; }

// Workspace layout: per-point values [n][4] double, per-point flags [n] int32,
// then per-reduce-block partials [nb][4] double-double and first failures [nb] int64.
struct WsLayout {
    double *vals;
    int32_t *flags;
    double *partial;
    int64_t *pfail;
    size_t bytes;
};

WsLayout ws_layout(void *ws, int64_t n) {
    const int64_t nb = num_reduce_blocks(n);
    WsLayout L;
    const size_t vbytes = align256((size_t)n * 4 * sizeof(double));
    const size_t fbytes = align256((size_t)n * sizeof(int32_t));
    const size_t pbytes = align256((size_t)nb * 8 * sizeof(double));  // double-double pairs
    const size_t qbytes = align256((size_t)nb * sizeof(int64_t));
    L.bytes = vbytes + fbytes + pbytes + qbytes + 256;
    char *base = (char *)ws;
    L.vals = (double *)base;
    L.flags = (int32_t *)(base + vbytes);
    L.partial = (double *)(base + vbytes + fbytes);
    L.pfail = (int64_t *)(base + vbytes + fbytes + pbytes);
    return L;
}

// Level 1 of the fixed-order sum: thread c of the grid adds points
// [c kChunk, (c+1) kChunk) in ascending order; each workgroup combines its
// threads in a fixed tree (double-double) into partial[block].
__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const double *__restrict__ vals,
                                                                const int32_t *__restrict__ flags, int64_t n,
                                                                double *__restrict__ partial,
                                                                int64_t *__restrict__ pfail) {
    __shared__ DD sh[4][kReduceThreads];
    __shared__ int64_t shf[kReduceThreads];
    const int t = threadIdx.x;
    const int64_t i0 = ((int64_t)blockIdx.x * kReduceThreads + t) * kChunk;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t f = kNoFailure;
    for (int64_t i = i0; i < i0 + kChunk && i < n; ++i) {
        a0 += vals[4 * i + 0];
        a1 += vals[4 * i + 1];
        a2 += vals[4 * i + 2];
        a3 += vals[4 * i + 3];
        if (flags[i] && f == kNoFailure) f = i + 1;
    }
    sh[0][t] = DD{a0, 0.0};
    sh[1][t] = DD{a1, 0.0};
    sh[2][t] = DD{a2, 0.0};
    sh[3][t] = DD{a3, 0.0};
    shf[t] = f;
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sh[q][t] = dd_add(sh[q][t], sh[q][t + s]);
            shf[t] = min(shf[t], shf[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            partial[8 * blockIdx.x + 2 * q] = sh[q][0].hi;
            partial[8 * blockIdx.x + 2 * q + 1] = sh[q][0].lo;
        }
        pfail[blockIdx.x] = shf[0];
    }
}

__global__ void status_init_kernel(unsigned long long *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = (unsigned long long)kNoFailure;
}

__global__ void status_fix_kernel(unsigned long long *status, const double *__restrict__ theta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const Params P = load_params(theta);
        long long s = (long long)*status;
        if (!P.valid) s = VECCHIA_STATUS_THETA;
        else if (s == (long long)kNoFailure) s = 0;
        *status = (unsigned long long)s;
    }
}

// Level 2 of the fixed-order sum: the reduce-block partials (double-double)
// in a fixed order; writes l, the gradient and the status.
__global__ void __launch_bounds__(kFinalizeThreads) finalize_kernel(const double *__restrict__ partial,
                                                                    const int64_t *__restrict__ pfail,
                                                                    int64_t nblocks,
                                                                    const double *__restrict__ theta,
                                                                    double *__restrict__ out,
                                                                    double *__restrict__ grad,
                                                                    int64_t *__restrict__ status) {
    __shared__ DD sh[4][kFinalizeThreads];
    __shared__ int64_t shf[kFinalizeThreads];
    const int t = threadIdx.x;
    const Params P = load_params(theta);
    DD a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    int64_t f = kNoFailure;
    if (P.valid) {
        for (int64_t c = t; c < nblocks; c += kFinalizeThreads) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = dd_add(a[q], DD{partial[8 * c + 2 * q], partial[8 * c + 2 * q + 1]});
            f = min(f, pfail[c]);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q][t] = a[q];
    shf[t] = f;
    __syncthreads();
    for (int s = kFinalizeThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sh[q][t] = dd_add(sh[q][t], sh[q][t + s]);
            shf[t] = min(shf[t], shf[t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double nan = __builtin_nan("");
        int64_t st;
        if (!P.valid) st = VECCHIA_STATUS_THETA;
        else st = (shf[0] == kNoFailure) ? 0 : shf[0];
        const bool ok = (st == 0);
        out[0] = ok ? sh[0][0].hi + sh[0][0].lo : nan;
        if (grad) {
            grad[0] = ok ? sh[1][0].hi + sh[1][0].lo : nan;
            grad[1] = ok ? sh[2][0].hi + sh[2][0].lo : nan;
            grad[2] = ok ? sh[3][0].hi + sh[3][0].lo : nan;
        }
        status[0] = st;
    }
}

// ---------------------------------------------------------------- dispatch
// host-side variant table, indexed by [with_grad][m]; 0 = default
int g_variant[2][VECCHIA_MAX_M + 1] = {};

int resolve_variant(int m, bool grad, int requested) {
    int v = requested != V_AUTO ? requested : g_variant[grad ? 1 : 0][m];
    if (v == V_AUTO || !variant_feasible(v, m)) v = default_variant(m);
    return v;
}

int nu_code(double nu) {
    if (nu == 0.5) return 0;
    if (nu == 1.5) return 1;
    if (nu == 2.5) return 2;
    return -1;
}

int launch_any(int nuc, bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    switch (nuc) {
        case 0: return launch_nu05(grad, variant, a, s);
        case 1: return launch_nu15(grad, variant, a, s);
        default: return launch_nu25(grad, variant, a, s);
    }
}

int check_common(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                 const double *theta) {
    if (n < 0 || m < 0) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (nu_code(nu) < 0) return VECCHIA_EINVAL;
    if (!theta) return VECCHIA_EINVAL;
    if (n > 0 && (!locs || !z)) return VECCHIA_EINVAL;
    if (n > 1 && m > 0 && !nbr) return VECCHIA_EINVAL;
    if (n > (int64_t)INT32_MAX * kChunk) return VECCHIA_EUNSUPPORTED;
    return VECCHIA_OK;
}

int run_sum(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
            const double *theta, double *out, double *grad, int64_t *status, void *ws, size_t ws_bytes,
            void *stream, bool with_grad, int variant) {
    int rc = check_common(locs, z, nbr, n, m, nu, theta);
    if (rc != VECCHIA_OK) return rc;
    if (!out || !status || (with_grad && !grad)) return VECCHIA_EINVAL;
    WsLayout L = ws_layout(ws, n);
    if (!ws || ws_bytes < L.bytes) return VECCHIA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    EvalArgs a{locs, z, nbr, n, m, theta, nullptr, n, L.vals, 4, with_grad ? L.vals + 1 : nullptr, 4, L.flags,
               nullptr};
    if (!with_grad) {
        // the gradient slots of vals stay unwritten; the reduction still reads them
        if (n > 0 && hipMemsetAsync(L.vals, 0, (size_t)n * 4 * sizeof(double), s) != hipSuccess) return VECCHIA_EHIP;
    }
    rc = launch_any(nu_code(nu), with_grad, resolve_variant(m, with_grad, variant), a, s);
    if (rc != VECCHIA_OK) return rc;
    const int64_t nb = num_reduce_blocks(n);
    if (nb > 0)
        hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)nb), dim3(kReduceThreads), 0, s, L.vals, L.flags, n,
                           L.partial, L.pfail);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, L.partial, L.pfail, nb, theta, out,
                       with_grad ? grad : nullptr, status);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

int run_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
              const double *theta, const int64_t *idx, int64_t nidx, double *terms, double *gterms,
              int64_t *status, void *stream, int variant) {
    int rc = check_common(locs, z, nbr, n, m, nu, theta);
    if (rc != VECCHIA_OK) return rc;
    if (nidx < 0 || !status || (nidx > 0 && !terms) || (!idx && nidx != n)) return VECCHIA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *st = (unsigned long long *)status;
    const bool g = gterms != nullptr;
    EvalArgs a{locs, z, nbr, n, m, theta, idx, nidx, terms, 1, gterms, 3, nullptr, st};
    hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, s, st);
    rc = launch_any(nu_code(nu), g, resolve_variant(m, g, variant), a, s);
    if (rc != VECCHIA_OK) return rc;
    hipLaunchKernelGGL(status_fix_kernel, dim3(1), dim3(64), 0, s, st, theta);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

const char *vecchia_strerror(int code) {
    switch (code) {
        case VECCHIA_OK: return "success";
        case VECCHIA_EINVAL: return "invalid argument";
        case VECCHIA_EUNSUPPORTED: return "unsupported size or option";
        case VECCHIA_EHIP: return "HIP runtime error";
        case VECCHIA_EWORKSPACE: return "workspace missing or too small";
        default: return "unknown error";
    }
}

const char *vecchia_version(void) { return "vecchia-mi355x 0.1 (gfx950, FP64)"; }

size_t vecchia_workspace_size(int64_t n, int32_t m) {
    (void)m;
    if (n < 0) return 0;
    return ws_layout(nullptr, n).bytes;
}

int vecchia_loglik(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                   const double *theta, double *out, int64_t *status, void *ws, size_t ws_bytes, void *stream) {
    return run_sum(locs, z, nbr, n, m, nu, theta, out, nullptr, status, ws, ws_bytes, stream, false, V_AUTO);
}

int vecchia_loglik_grad(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                        const double *theta, double *out, double *grad, int64_t *status, void *ws,
                        size_t ws_bytes, void *stream) {
    return run_sum(locs, z, nbr, n, m, nu, theta, out, grad, status, ws, ws_bytes, stream, true, V_AUTO);
}

int vecchia_loglik_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                         double nu, const double *theta, const int64_t *idx, int64_t nidx, double *terms,
                         double *gterms, int64_t *status, void *stream) {
    return run_terms(locs, z, nbr, n, m, nu, theta, idx, nidx, terms, gterms, status, stream, V_AUTO);
}

int vecchia_set_variant(int32_t m, int32_t with_grad, int32_t variant) {
    if (m < 0 || m > VECCHIA_MAX_M || variant < V_AUTO || variant > V_TILE_W8) return VECCHIA_EINVAL;
    if (variant != V_AUTO && !variant_feasible(variant, m)) return VECCHIA_EUNSUPPORTED;
    g_variant[with_grad ? 1 : 0][m] = variant;
    return VECCHIA_OK;
}

int vecchia_get_variant(int32_t m, int32_t with_grad) {
    if (m < 0 || m > VECCHIA_MAX_M) return -VECCHIA_EINVAL;
    return resolve_variant(m, with_grad != 0, V_AUTO);
}

int vecchia_variant_feasible(int32_t m, int32_t variant) {
    if (m < 0 || m > VECCHIA_MAX_M || variant <= V_AUTO || variant > V_TILE_W8) return 0;
    return variant_feasible(variant, m) ? 1 : 0;
}

int vecchia_loglik_variant(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                           double nu, const double *theta, int32_t variant, double *out, double *grad,
                           int64_t *status, void *ws, size_t ws_bytes, void *stream) {
    if (variant < V_AUTO || variant > V_TILE_W8) return VECCHIA_EINVAL;
    if (variant != V_AUTO && m >= 0 && m <= VECCHIA_MAX_M && !variant_feasible(variant, m))
        return VECCHIA_EUNSUPPORTED;
    return run_sum(locs, z, nbr, n, m, nu, theta, out, grad, status, ws, ws_bytes, stream, grad != nullptr,
                   variant);
}

int vecchia_loglik_terms_variant(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                                 double nu, const double *theta, int32_t variant, const int64_t *idx, int64_t nidx,
                                 double *terms, double *gterms, int64_t *status, void *stream) {
    if (variant < V_AUTO || variant > V_TILE_W8) return VECCHIA_EINVAL;
    if (variant != V_AUTO && m >= 0 && m <= VECCHIA_MAX_M && !variant_feasible(variant, m))
        return VECCHIA_EUNSUPPORTED;
    return run_terms(locs, z, nbr, n, m, nu, theta, idx, nidx, terms, gterms, status, stream, variant);
}

}  // extern "C"

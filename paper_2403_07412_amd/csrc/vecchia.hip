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
#include "reduce.h"

using namespace vecchia;

namespace vecchia {

// ---------------------------------------------------------------- dispatch
// host-side variant table, indexed by [with_grad][m]; 0 = default
int g_variant[2][VECCHIA_MAX_M + 1] = {};

int resolve_variant(int m, bool grad, int requested, int kc) {
    int v = requested != V_AUTO ? requested : g_variant[grad ? 1 : 0][m];
    if (v == V_AUTO || !variant_feasible(v, m)) v = default_variant(m, grad, kc);
    return v;
}

int nu_code(double nu) {
    if (nu == 0.5) return 0;
    if (nu == 1.5) return 1;
    if (nu == 2.5) return 2;
    return -1;
}

int launch_any(int kc, bool grad, int variant, const EvalArgs &a, hipStream_t s) {
    switch (kc) {
        case 0: return launch_nu05(grad, variant, a, s);
        case 1: return launch_nu15(grad, variant, a, s);
        case 2: return launch_nu25(grad, variant, a, s);
        case 3: return launch_kc3(grad, variant, a, s);
        case 4: return launch_kc4(grad, variant, a, s);
        case 5: return launch_kc5(grad, variant, a, s);
        case 6: return launch_kc6(grad, variant, a, s);
        case 7: return launch_kc7(grad, variant, a, s);
        default: return VECCHIA_EINVAL;
    }
}

// Covariance code of a model (family + 4 metric, as kc_family / kc_gcd
// read it) and its power-exponential exponent; -1 for an invalid model.
int cov_code(const vecchia_cov *cov, double *alpha) {
    if (!cov || (cov->metric != VECCHIA_EUCLIDEAN && cov->metric != VECCHIA_GREAT_CIRCLE)) return -1;
    int fam;
    if (cov->family == VECCHIA_MATERN) {
        fam = nu_code(cov->smoothness);
        if (fam < 0) return -1;
        *alpha = 1.0;
    } else if (cov->family == VECCHIA_POWEXP) {
        if (!(cov->smoothness > 0.0 && cov->smoothness <= 2.0)) return -1;
        fam = 3;
        *alpha = cov->smoothness;
    } else {
        return -1;
    }
    return fam + 4 * (cov->metric == VECCHIA_GREAT_CIRCLE ? 1 : 0);
}

}  // namespace vecchia

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

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

__global__ void __launch_bounds__(kReduceThreads) reduce_kernel(const double *__restrict__ vals,
                                                                const int32_t *__restrict__ flags, int64_t n,
                                                                double *__restrict__ partial,
                                                                int64_t *__restrict__ pfail) {
    reduce_segment_block(vals, flags, n, blockIdx.x, partial + 8 * (int64_t)blockIdx.x, pfail + blockIdx.x);
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

__global__ void __launch_bounds__(kFinalizeThreads) finalize_kernel(const double *__restrict__ partial,
                                                                    const int64_t *__restrict__ pfail,
                                                                    int64_t nblocks,
                                                                    const double *__restrict__ theta,
                                                                    double *__restrict__ out,
                                                                    double *__restrict__ grad,
                                                                    int64_t *__restrict__ status) {
    finalize_segment(partial, pfail, nblocks, theta, out, grad, status);
}

int check_common(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, int kc,
                 const double *theta) {
    if (n < 0 || m < 0) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (kc < 0) return VECCHIA_EINVAL;
    if (!theta) return VECCHIA_EINVAL;
    if (n > 0 && (!locs || !z)) return VECCHIA_EINVAL;
    if (n > 1 && m > 0 && !nbr) return VECCHIA_EINVAL;
    if (n > (int64_t)INT32_MAX * kChunk) return VECCHIA_EUNSUPPORTED;
    return VECCHIA_OK;
}

int run_sum(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, int kc, double alpha,
            const double *theta, double *out, double *grad, int64_t *status, void *ws, size_t ws_bytes,
            void *stream, bool with_grad, int variant) {
    int rc = check_common(locs, z, nbr, n, m, kc, theta);
    if (rc != VECCHIA_OK) return rc;
    if (!out || !status || (with_grad && !grad)) return VECCHIA_EINVAL;
    WsLayout L = ws_layout(ws, n);
    if (!ws || ws_bytes < L.bytes) return VECCHIA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    // the gradient columns are always written (zeros for a value-only evaluation)
    EvalArgs a{};
    a.k.locs = locs;
    a.k.z = z;
    a.k.nbr = nbr;
    a.k.n = n;
    a.k.m = m;
    a.k.theta = theta;
    a.k.ell = L.vals;
    a.k.ell_stride = 4;
    a.k.g = L.vals + 1;
    a.k.g_stride = 4;
    a.k.flags = L.flags;
    a.k.alpha = alpha;
    a.t_begin = 0;
    a.t_end = n;
    a.m_max = m;
    rc = launch_any(kc, with_grad, resolve_variant(m, with_grad, variant, kc), a, s);
    if (rc != VECCHIA_OK) return rc;
    const int64_t nb = num_reduce_blocks(n);
    if (nb > 0)
        hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)nb), dim3(kReduceThreads), 0, s, L.vals, L.flags, n,
                           L.partial, L.pfail);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, L.partial, L.pfail, nb, theta, out,
                       with_grad ? grad : nullptr, status);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

int run_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, int kc, double alpha,
              const double *theta, const int64_t *idx, int64_t nidx, double *terms, double *gterms,
              int64_t *status, void *stream, int variant) {
    int rc = check_common(locs, z, nbr, n, m, kc, theta);
    if (rc != VECCHIA_OK) return rc;
    if (nidx < 0 || !status || (nidx > 0 && !terms) || (!idx && nidx != n)) return VECCHIA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *st = (unsigned long long *)status;
    const bool g = gterms != nullptr;
    EvalArgs a{};
    a.k.locs = locs;
    a.k.z = z;
    a.k.nbr = nbr;
    a.k.n = n;
    a.k.m = m;
    a.k.theta = theta;
    a.k.idx = idx;
    a.k.ell = terms;
    a.k.ell_stride = 1;
    a.k.g = gterms;
    a.k.g_stride = 3;
    a.k.status = st;
    a.k.alpha = alpha;
    a.t_begin = 0;
    a.t_end = nidx;
    a.m_max = m;
    hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, s, st);
    rc = launch_any(kc, g, resolve_variant(m, g, variant, kc), a, s);
    if (rc != VECCHIA_OK) return rc;
    hipLaunchKernelGGL(status_fix_kernel, dim3(1), dim3(64), 0, s, st, theta);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

int run_predict(const double *locs, const double *z, int64_t n, const double *qlocs, int64_t nq,
                const int32_t *nbr, int32_t m, int kc, double alpha, const double *theta, double *mean, double *var,
                int64_t *status, void *stream) {
    if (n < 0 || nq < 0 || m < 0 || kc < 0 || !theta || !status) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (nq > (int64_t)INT32_MAX * kChunk) return VECCHIA_EUNSUPPORTED;
    if (nq > 0 && (!qlocs || !mean || !var)) return VECCHIA_EINVAL;
    const int32_t k = (int32_t)std::min<int64_t>(n, m);
    if (k > 0 && (!locs || !z || !nbr)) return VECCHIA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *st = (unsigned long long *)status;
    EvalArgs a{};
    a.k.locs = locs;
    a.k.z = z;
    a.k.nbr = nbr;
    a.k.n = n;
    a.k.m = m;
    a.k.theta = theta;
    a.k.status = st;
    a.k.alpha = alpha;
    a.k.qlocs = qlocs;
    a.k.nq = nq;
    a.k.pmean = mean;
    a.k.pvar = var;
    a.t_begin = 0;
    a.t_end = nq;
    a.m_max = m;
    hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, s, st);
    const int rc = launch_any(kc, false, resolve_variant(m, false, V_AUTO), a, s);
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
    return run_sum(locs, z, nbr, n, m, nu_code(nu), 1.0, theta, out, nullptr, status, ws, ws_bytes, stream, false,
                   V_AUTO);
}

int vecchia_loglik_grad(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                        const double *theta, double *out, double *grad, int64_t *status, void *ws,
                        size_t ws_bytes, void *stream) {
    return run_sum(locs, z, nbr, n, m, nu_code(nu), 1.0, theta, out, grad, status, ws, ws_bytes, stream, true,
                   V_AUTO);
}

int vecchia_loglik_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                         double nu, const double *theta, const int64_t *idx, int64_t nidx, double *terms,
                         double *gterms, int64_t *status, void *stream) {
    return run_terms(locs, z, nbr, n, m, nu_code(nu), 1.0, theta, idx, nidx, terms, gterms, status, stream, V_AUTO);
}

int vecchia_loglik_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                       const vecchia_cov *cov, const double *theta, double *out, double *grad, int64_t *status,
                       void *ws, size_t ws_bytes, void *stream) {
    double alpha = 1.0;
    const int kc = cov_code(cov, &alpha);
    return run_sum(locs, z, nbr, n, m, kc, alpha, theta, out, grad, status, ws, ws_bytes, stream, grad != nullptr,
                   V_AUTO);
}

int vecchia_loglik_terms_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                             const vecchia_cov *cov, const double *theta, const int64_t *idx, int64_t nidx,
                             double *terms, double *gterms, int64_t *status, void *stream) {
    double alpha = 1.0;
    const int kc = cov_code(cov, &alpha);
    return run_terms(locs, z, nbr, n, m, kc, alpha, theta, idx, nidx, terms, gterms, status, stream, V_AUTO);
}

int vecchia_predict(const double *locs, const double *z, int64_t n, const double *qlocs, int64_t nq,
                    const int32_t *nbr, int32_t m, const vecchia_cov *cov, const double *theta, double *mean,
                    double *var, int64_t *status, void *stream) {
    double alpha = 1.0;
    const int kc = cov_code(cov, &alpha);
    return run_predict(locs, z, n, qlocs, nq, nbr, m, kc, alpha, theta, mean, var, status, stream);
}

int vecchia_set_variant(int32_t m, int32_t with_grad, int32_t variant) {
    if (m < 0 || m > VECCHIA_MAX_M || variant < V_AUTO || variant > V_TILE_W8) return VECCHIA_EINVAL;
    if (variant != V_AUTO && !variant_feasible(variant, m)) return VECCHIA_EUNSUPPORTED;
    g_variant[with_grad ? 1 : 0][m] = variant;
    return VECCHIA_OK;
}

int vecchia_get_variant(int32_t m, int32_t with_grad) {
    if (m < 0 || m > VECCHIA_MAX_M) return -VECCHIA_EINVAL;
    return resolve_variant(m, with_grad != 0, V_AUTO, 0);
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
    return run_sum(locs, z, nbr, n, m, nu_code(nu), 1.0, theta, out, grad, status, ws, ws_bytes, stream,
                   grad != nullptr, variant);
}

int vecchia_loglik_terms_variant(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                                 double nu, const double *theta, int32_t variant, const int64_t *idx, int64_t nidx,
                                 double *terms, double *gterms, int64_t *status, void *stream) {
    if (variant < V_AUTO || variant > V_TILE_W8) return VECCHIA_EINVAL;
    if (variant != V_AUTO && m >= 0 && m <= VECCHIA_MAX_M && !variant_feasible(variant, m))
        return VECCHIA_EUNSUPPORTED;
    return run_terms(locs, z, nbr, n, m, nu_code(nu), 1.0, theta, idx, nidx, terms, gterms, status, stream,
                     variant);
}

}  // extern "C"

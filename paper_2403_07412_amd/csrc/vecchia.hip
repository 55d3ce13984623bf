// C ABI and launch logic of the Vecchia log-likelihood library (gfx950).
//
// Pipeline of one evaluation (Algorithm 1, fused):
//   conditional kernel  every workgroup takes a fixed chunk of kChunk points
//                       and, point by point, gathers the neighbours, builds the
//                       covariance block, factors it, solves, forms l_i (and
//                       its gradient), and adds the results in ascending i into
//                       one partial per chunk;
//   finalize kernel     sums the partials in a fixed order with double-double
//                       accumulation and writes l, the gradient and the status.
// Chunk boundaries and both summation orders are fixed, so results are
// bitwise reproducible whatever order the hardware runs the workgroups in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "../../include/vecchia.h"
#include "device_common.h"
#include "kernel_lds.h"

using namespace vecchia;

namespace {

constexpr int kThreads = 256;
constexpr int kFinalizeThreads = 256;

int64_t num_chunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Workspace layout: partials [nchunks][4] double, then first failures [nchunks] int64.
struct WsLayout {
    double *partial;
    int64_t *pfail;
    size_t bytes;
};

WsLayout ws_layout(void *ws, int64_t n) {
    const int64_t nc = num_chunks(n);
    WsLayout L;
    const size_t pbytes = align256((size_t)nc * 4 * sizeof(double));
    const size_t fbytes = align256((size_t)nc * sizeof(int64_t));
    L.bytes = pbytes + fbytes + 256;
    char *base = (char *)ws;
    L.partial = (double *)base;
    L.pfail = (int64_t *)(base + pbytes);
    return L;
}

// ---------------------------------------------------------------- kernels
template <int NU, bool GRAD>
__global__ void __launch_bounds__(kThreads) chunk_kernel_lds(const double *__restrict__ locs,
                                                             const double *__restrict__ z,
                                                             const int32_t *__restrict__ nbr, int64_t n, int32_t m,
                                                             const double *__restrict__ theta,
                                                             double *__restrict__ partial,
                                                             int64_t *__restrict__ pfail) {
    extern __shared__ double smem[];
    const Params P = load_params(theta);
    if (!P.valid) return;  // uniform: the finalize kernel reports the bad parameters
    const int64_t c = blockIdx.x;
    const int64_t i0 = c * kChunk;
    const int64_t i1 = (i0 + kChunk < n) ? i0 + kChunk : n;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int64_t fail = kNoFailure;
    for (int64_t i = i0; i < i1; ++i) {
        const CondOut o = lds_conditional<NU, GRAD>(locs, z, nbr, i, m, P, smem);
        acc0 += o.ell;
        acc1 += o.g0;
        acc2 += o.g1;
        acc3 += o.g2;
        if (o.bad && fail == kNoFailure) fail = i + 1;
    }
    if (threadIdx.x == 0) {
        partial[4 * c + 0] = acc0;
        partial[4 * c + 1] = acc1;
        partial[4 * c + 2] = acc2;
        partial[4 * c + 3] = acc3;
        pfail[c] = fail;
    }
}

template <int NU, bool GRAD>
__global__ void __launch_bounds__(kThreads) terms_kernel_lds(const double *__restrict__ locs,
                                                             const double *__restrict__ z,
                                                             const int32_t *__restrict__ nbr, int64_t n, int32_t m,
                                                             const double *__restrict__ theta,
                                                             const int64_t *__restrict__ idx, int64_t nidx,
                                                             double *__restrict__ terms,
                                                             double *__restrict__ gterms,
                                                             unsigned long long *__restrict__ status) {
    extern __shared__ double smem[];
    const Params P = load_params(theta);
    for (int64_t t = blockIdx.x; t < nidx; t += gridDim.x) {
        const int64_t i = idx ? idx[t] : t;
        CondOut o;
        bool bad = false;
        if (!P.valid || i < 0 || i >= n) {
            const double nan = __builtin_nan("");
            o.ell = o.g0 = o.g1 = o.g2 = nan;
            bad = P.valid;  // bad parameters are reported once by the status fix-up
        } else {
            o = lds_conditional<NU, GRAD>(locs, z, nbr, i, m, P, smem);
            bad = o.bad;
            if (bad) o.ell = o.g0 = o.g1 = o.g2 = __builtin_nan("");
        }
        if (threadIdx.x == 0) {
            terms[t] = o.ell;
            if (gterms) {
                gterms[3 * t + 0] = o.g0;
                gterms[3 * t + 1] = o.g1;
                gterms[3 * t + 2] = o.g2;
            }
            if (bad) atomicMin(status, (unsigned long long)(t + 1));
        }
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

// Sums the chunk partials in a fixed order (strided per thread, then a fixed
// tree) with double-double accumulation; writes l, the gradient and the status.
__global__ void __launch_bounds__(kFinalizeThreads) finalize_kernel(const double *__restrict__ partial,
                                                                    const int64_t *__restrict__ pfail,
                                                                    int64_t nchunks,
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
        for (int64_t c = t; c < nchunks; c += kFinalizeThreads) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = dd_add(a[q], partial[4 * c + q]);
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
int nu_code(double nu) {
    if (nu == 0.5) return 0;
    if (nu == 1.5) return 1;
    if (nu == 2.5) return 2;
    return -1;
}

template <typename K>
hipError_t allow_smem(K kernel, size_t bytes) {
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int NU, bool GRAD>
int launch_chunks_lds(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                      const double *theta, const WsLayout &L, hipStream_t s) {
    const int64_t nc = num_chunks(n);
    if (nc == 0) return VECCHIA_OK;
    const size_t smem = lds_kernel_smem_bytes(m);
    auto kern = chunk_kernel_lds<NU, GRAD>;
    if (allow_smem(kern, smem) != hipSuccess) return VECCHIA_EHIP;
    hipLaunchKernelGGL(kern, dim3((unsigned)nc), dim3(kThreads), smem, s, locs, z, nbr, n, m, theta, L.partial,
                       L.pfail);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

template <bool GRAD>
int launch_chunks(int nc_, const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                  const double *theta, const WsLayout &L, hipStream_t s) {
    switch (nc_) {
        case 0: return launch_chunks_lds<0, GRAD>(locs, z, nbr, n, m, theta, L, s);
        case 1: return launch_chunks_lds<1, GRAD>(locs, z, nbr, n, m, theta, L, s);
        default: return launch_chunks_lds<2, GRAD>(locs, z, nbr, n, m, theta, L, s);
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
            void *stream, bool with_grad) {
    int rc = check_common(locs, z, nbr, n, m, nu, theta);
    if (rc != VECCHIA_OK) return rc;
    if (!out || !status || (with_grad && !grad)) return VECCHIA_EINVAL;
    WsLayout L = ws_layout(ws, n);
    if (!ws || ws_bytes < L.bytes) return VECCHIA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int nc_ = nu_code(nu);
    rc = with_grad ? launch_chunks<true>(nc_, locs, z, nbr, n, m, theta, L, s)
                   : launch_chunks<false>(nc_, locs, z, nbr, n, m, theta, L, s);
    if (rc != VECCHIA_OK) return rc;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, L.partial, L.pfail, num_chunks(n),
                       theta, out, with_grad ? grad : nullptr, status);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

template <int NU, bool GRAD>
int launch_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                 const double *theta, const int64_t *idx, int64_t nidx, double *terms, double *gterms,
                 int64_t *status, hipStream_t s) {
    const size_t smem = lds_kernel_smem_bytes(m);
    auto kern = terms_kernel_lds<NU, GRAD>;
    if (allow_smem(kern, smem) != hipSuccess) return VECCHIA_EHIP;
    unsigned long long *st = (unsigned long long *)status;
    hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, s, st);
    if (nidx > 0) {
        const int64_t grid = std::min<int64_t>(nidx, 1 << 20);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), smem, s, locs, z, nbr, n, m, theta, idx,
                           nidx, terms, gterms, st);
    }
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
    return run_sum(locs, z, nbr, n, m, nu, theta, out, nullptr, status, ws, ws_bytes, stream, false);
}

int vecchia_loglik_grad(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                        const double *theta, double *out, double *grad, int64_t *status, void *ws,
                        size_t ws_bytes, void *stream) {
    return run_sum(locs, z, nbr, n, m, nu, theta, out, grad, status, ws, ws_bytes, stream, true);
}

int vecchia_loglik_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                         double nu, const double *theta, const int64_t *idx, int64_t nidx, double *terms,
                         double *gterms, int64_t *status, void *stream) {
    int rc = check_common(locs, z, nbr, n, m, nu, theta);
    if (rc != VECCHIA_OK) return rc;
    if (nidx < 0 || !status || (nidx > 0 && !terms) || (!idx && nidx != n)) return VECCHIA_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const bool g = gterms != nullptr;
    switch (nu_code(nu)) {
        case 0: return g ? launch_terms<0, true>(locs, z, nbr, n, m, theta, idx, nidx, terms, gterms, status, s)
                         : launch_terms<0, false>(locs, z, nbr, n, m, theta, idx, nidx, terms, gterms, status, s);
        case 1: return g ? launch_terms<1, true>(locs, z, nbr, n, m, theta, idx, nidx, terms, gterms, status, s)
                         : launch_terms<1, false>(locs, z, nbr, n, m, theta, idx, nidx, terms, gterms, status, s);
        default: return g ? launch_terms<2, true>(locs, z, nbr, n, m, theta, idx, nidx, terms, gterms, status, s)
                          : launch_terms<2, false>(locs, z, nbr, n, m, theta, idx, nidx, terms, gterms, status, s);
    }
}

}  // extern "C"

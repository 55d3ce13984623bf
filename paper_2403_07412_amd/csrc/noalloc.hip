// vecchia_loglik_grad without a caller workspace, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The per-point rows and the reduction partials that vecchia_loglik_grad keeps
// in the caller's workspace live here in one static device array, `scratch`,
// of kScratchBytes.  Points are evaluated in slices of kSlicePoints rows, each
// slice's rows reduced into the per-block partials before the next slice
// reuses them; slices start on reduce-block boundaries, so every partial sums
// the same points in the same order as in vecchia_loglik_grad and the results
// are bitwise equal to it (same kernel variant).
//
// Each GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device, taken once per device
// on the first call there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "launch.h"
#include "reduce.h"
#include "vecchia.h"

using namespace vecchia;

namespace {

constexpr int64_t kSlicePoints = (int64_t)1 << 18;                       // rows per slice
constexpr int64_t kMaxReduceBlocks = (int64_t)VECCHIA_NOALLOC_MAX_N / kPointsPerReduceBlock;
static_assert(kSlicePoints % kPointsPerReduceBlock == 0, "slices must start on reduce-block boundaries");
static_assert((int64_t)VECCHIA_NOALLOC_MAX_N % kPointsPerReduceBlock == 0, "whole reduce blocks");

constexpr size_t kValsOff = 0;                                                     // [kSlicePoints][4] double
constexpr size_t kFlagsOff = kValsOff + (size_t)kSlicePoints * 4 * sizeof(double);  // [kSlicePoints] int32
constexpr size_t kPartialOff = kFlagsOff + (size_t)kSlicePoints * sizeof(int32_t);  // [blocks][8] double
constexpr size_t kPfailOff = kPartialOff + (size_t)kMaxReduceBlocks * 8 * sizeof(double);  // [blocks] int64
constexpr size_t kScratchBytes = kPfailOff + (size_t)kMaxReduceBlocks * sizeof(int64_t);
static_assert(kScratchBytes <= ((size_t)12 << 20), "scratch stays modest");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device ordinal

// The device address of `scratch` on the current device (the symbol's host
// name is not a device address).
int scratch_address(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VECCHIA_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VECCHIA_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = (char *)g_scratch_dev[dev];
    return VECCHIA_OK;
}

// Level 1 of the fixed-order sum for the reduce blocks [b0, b0 + gridDim.x)
// of a slice whose rows start at point row0.
__global__ void __launch_bounds__(kReduceThreads) slice_reduce_kernel(const double *__restrict__ vals,
                                                                      const int32_t *__restrict__ flags,
                                                                      int64_t n_end, int64_t b0, int64_t row0,
                                                                      double *__restrict__ partial,
                                                                      int64_t *__restrict__ pfail) {
    const int64_t bx = b0 + blockIdx.x;
    reduce_segment_block(vals, flags, n_end, bx, partial + 8 * bx, pfail + bx, row0);
}

__global__ void __launch_bounds__(kFinalizeThreads) noalloc_finalize_kernel(const double *__restrict__ partial,
                                                                            const int64_t *__restrict__ pfail,
                                                                            int64_t nblocks,
                                                                            const double *__restrict__ theta,
                                                                            double *__restrict__ out,
                                                                            double *__restrict__ grad,
                                                                            int64_t *__restrict__ status) {
    finalize_segment(partial, pfail, nblocks, theta, out, grad, status);
}

}  // namespace

extern "C" int vecchia_loglik_grad_noalloc(const double *locs, const double *z, const int32_t *nbr, int64_t n,
                                           int32_t m, double nu, const double *theta, double *out, double *grad,
                                           int64_t *status, void *stream) {
    const int kc = nu_code(nu);
    if (n < 0 || m < 0 || kc < 0 || !theta || !out || !grad || !status) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (n > 0 && (!locs || !z)) return VECCHIA_EINVAL;
    if (n > 1 && m > 0 && !nbr) return VECCHIA_EINVAL;
    if (n > (int64_t)VECCHIA_NOALLOC_MAX_N) return VECCHIA_EUNSUPPORTED;
    char *base = nullptr;
    const int rc0 = scratch_address(&base);
    if (rc0 != VECCHIA_OK) return rc0;
    double *vals = (double *)(base + kValsOff);
    int32_t *flags = (int32_t *)(base + kFlagsOff);
    double *partial = (double *)(base + kPartialOff);
    int64_t *pfail = (int64_t *)(base + kPfailOff);
    hipStream_t s = (hipStream_t)stream;
    const int variant = resolve_variant(m, true, V_AUTO);
    for (int64_t s0 = 0; s0 < n; s0 += kSlicePoints) {
        const int64_t s1 = std::min(n, s0 + kSlicePoints);
        EvalArgs a{};
        a.k.locs = locs;
        a.k.z = z;
        a.k.nbr = nbr;
        a.k.n = n;
        a.k.m = m;
        a.k.theta = theta;
        a.k.ell = vals;
        a.k.ell_stride = 4;
        a.k.g = vals + 1;
        a.k.g_stride = 4;
        a.k.flags = flags;
        a.k.row0 = s0;
        a.t_begin = s0;
        a.t_end = s1;
        a.m_max = m;
        const int rc = launch_any(kc, true, variant, a, s);
        if (rc != VECCHIA_OK) return rc;
        const int64_t b0 = s0 / kPointsPerReduceBlock;
        const int64_t b1 = num_reduce_blocks(s1);
        hipLaunchKernelGGL(slice_reduce_kernel, dim3((unsigned)(b1 - b0)), dim3(kReduceThreads), 0, s, vals, flags,
                           s1, b0, s0, partial, pfail);
    }
    hipLaunchKernelGGL(noalloc_finalize_kernel, dim3(1), dim3(kFinalizeThreads), 0, s, partial, pfail,
                       num_reduce_blocks(n), theta, out, grad, status);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

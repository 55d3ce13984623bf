// Fixed-order, two-level summation of per-point results (Alg. 1's final sum,
// plus the three gradient components and the first failure).  One segment is
// one evaluation: n per-point rows (l_i, three gradient terms) and flags.
//   level 1  thread c of reduce block b adds points [b 4096 + 16 c, +16) in
//            ascending order; the block combines its 256 sums in a fixed tree
//            (double-double) into one partial;
//   level 2  one block adds the partials of the segment in a fixed strided
//            order and tree (double-double) and writes the outputs.
// The order depends only on n, so a segment gives bitwise the same result in
// the single and the batched entry points.
#pragma once

#include "device_common.h"
#include "vecchia.h"

namespace vecchia {

constexpr int kReduceThreads = 256;
constexpr int kFinalizeThreads = 256;
constexpr int64_t kPointsPerReduceBlock = (int64_t)kChunk * kReduceThreads;

__host__ __device__ inline int64_t num_reduce_blocks(int64_t n) {
    return (n + kPointsPerReduceBlock - 1) / kPointsPerReduceBlock;
}

// Level 1 for reduce block bx of a segment: point i's row is i - row0 of
// vals [.][4] and flags [.] (row0 > 0 when the rows hold a slice of the
// segment that starts at point row0); writes partial[0..8) (four
// double-double pairs) and *pfail (first failing point + 1 in the block, or
// kNoFailure).  Called by every thread of a kReduceThreads-thread block.
__device__ __forceinline__ void reduce_segment_block(const double *__restrict__ vals,
                                                     const int32_t *__restrict__ flags, int64_t n, int64_t bx,
                                                     double *__restrict__ partial, int64_t *__restrict__ pfail,
                                                     int64_t row0 = 0) {
    __shared__ DD sh[4][kReduceThreads];
    __shared__ int64_t shf[kReduceThreads];
    const int t = threadIdx.x;
    const int64_t i0 = (bx * kReduceThreads + t) * kChunk;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t f = kNoFailure;
    for (int64_t i = i0; i < i0 + kChunk && i < n; ++i) {
        const int64_t r = i - row0;
        a0 += vals[4 * r + 0];
        a1 += vals[4 * r + 1];
        a2 += vals[4 * r + 2];
        a3 += vals[4 * r + 3];
        if (flags[r] && f == kNoFailure) f = i + 1;
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
            partial[2 * q] = sh[q][0].hi;
            partial[2 * q + 1] = sh[q][0].lo;
        }
        *pfail = shf[0];
    }
}

// Level 2 for one segment: partial [nblocks][8], pfail [nblocks]; writes
// out[0], grad[0..3) (if grad) and status[0].  Called by every thread of a
// kFinalizeThreads-thread block.
__device__ __forceinline__ void finalize_segment(const double *__restrict__ partial,
                                                 const int64_t *__restrict__ pfail, int64_t nblocks,
                                                 const double *__restrict__ theta, double *__restrict__ out,
                                                 double *__restrict__ grad, int64_t *__restrict__ status) {
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

}  // namespace vecchia

// Device-wide primitives of the preprocessing: a stable least-significant-
// digit radix sort of (key, int32 value) pairs and an exclusive prefix sum of
// int32 counts.  Only kernel launches on the caller's stream (no memset, no
// copy, no synchronisation), with all temporary storage in the caller's
// workspace, so the preprocessing that uses them can be captured in a graph.
//
// Radix sort, per 8-bit digit from the least significant:
//   histogram  one wavefront per tile of 1024 keys counts its digits in LDS
//              and writes them digit-major: counts[d][tile];
//   scan       an exclusive prefix sum over that array gives every (digit,
//              tile) its first output position;
//   scatter    the tile's keys are ranked 64 at a time in input order: the
//              lanes holding the same digit are found with eight ballots, the
//              rank is the number of such lanes below, and a running count
//              per digit in LDS carries the order across the 16 rounds.
// Equal digits keep their input order in every pass, so the sort is stable.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace vecchia {

constexpr int kSortWave = 64;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortWave * kSortRounds;  // keys per tile
constexpr int kSortDigits = 256;
constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanChunk = kScanThreads * kScanPerThread;  // elements per scan block

__host__ __device__ inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

template <class K>
__device__ __forceinline__ int sort_digit(K key, int shift, int dmask) {
    return (int)((key >> shift) & (K)dmask);
}

template <class K>
__global__ void __launch_bounds__(kSortWave) sort_histogram_kernel(const K *__restrict__ keys, int64_t n, int shift,
                                                                   int dmask, int32_t *__restrict__ counts,
                                                                   int64_t ntiles) {
    __shared__ int32_t hist[kSortDigits];
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    for (int d = lane; d < kSortDigits; d += kSortWave) hist[d] = 0;
    __syncthreads();
    const int64_t base = tile * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t idx = base + r * kSortWave + lane;
        if (idx < n) atomicAdd(&hist[sort_digit(keys[idx], shift, dmask)], 1);
    }
    __syncthreads();
    for (int d = lane; d < kSortDigits; d += kSortWave) counts[(int64_t)d * ntiles + tile] = hist[d];
}

template <class K>
__global__ void __launch_bounds__(kSortWave) sort_scatter_kernel(const K *__restrict__ kin,
                                                                 const int32_t *__restrict__ vin,
                                                                 K *__restrict__ kout, int32_t *__restrict__ vout,
                                                                 int64_t n, int shift, int dmask,
                                                                 const int32_t *__restrict__ offsets,
                                                                 int64_t ntiles) {
    __shared__ int32_t running[kSortDigits];
    const int lane = threadIdx.x;
    const int64_t tile = blockIdx.x;
    for (int d = lane; d < kSortDigits; d += kSortWave) running[d] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes under this one
    const int64_t base = tile * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t idx = base + r * kSortWave + lane;
        const bool valid = idx < n;
        K key = 0;
        int32_t val = 0;
        int d = 0;
        if (valid) {
            key = kin[idx];
            val = vin[idx];
            d = sort_digit(key, shift, dmask);
        }
        // lanes holding this lane's digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t ones = __ballot(bit);
            same &= bit ? ones : ~ones;
        }
        const int rank = __popcll(same & below);
        const int before = valid ? running[d] : 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid && rank == 0) running[d] = before + __popcll(same);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid) {
            const int64_t pos = (int64_t)offsets[(int64_t)d * ntiles + tile] + before + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
    }
}

// Exclusive prefix sum, level 1: the sum of every chunk of kScanChunk elements.
__global__ void __launch_bounds__(kScanThreads) scan_chunk_sums_kernel(const int32_t *__restrict__ in, int64_t n,
                                                                       int32_t *__restrict__ sums) {
    __shared__ int32_t red[kScanThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int32_t s = 0;
    for (int q = 0; q < kScanPerThread; ++q) {
        const int64_t idx = base + (int64_t)q * kScanThreads + t;
        if (idx < n) s += in[idx];
    }
    red[t] = s;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) sums[blockIdx.x] = red[0];
}

// Block-wide exclusive scan of one value per thread (Hillis-Steele in LDS);
// returns the exclusive prefix and sets `total`.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *sh, int32_t &total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int32_t add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    const int32_t excl = sh[t] - v;
    __syncthreads();
    return excl;
}

// Level 2: exclusive scan of the chunk sums in place (one block, any count).
__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(int32_t *__restrict__ sums, int64_t count) {
    __shared__ int32_t sh[kScanThreads];
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < count; b0 += kScanThreads) {
        const int64_t idx = b0 + threadIdx.x;
        const int32_t v = idx < count ? sums[idx] : 0;
        int32_t total;
        const int32_t excl = block_exclusive_scan(v, sh, total);
        if (idx < count) sums[idx] = carry + excl;
        carry += total;
    }
}

// Level 3: every chunk scanned in order from its offset.  Thread t owns the
// kScanPerThread consecutive elements starting at t * kScanPerThread.
__global__ void __launch_bounds__(kScanThreads) scan_chunks_kernel(const int32_t *__restrict__ in, int64_t n,
                                                                   const int32_t *__restrict__ sums,
                                                                   int32_t *__restrict__ out) {
    __shared__ int32_t sh[kScanThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)t * kScanPerThread;
    int32_t local[kScanPerThread];
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
        const int64_t idx = base + q;
        local[q] = idx < n ? in[idx] : 0;
        s += local[q];
    }
    int32_t total;
    int32_t run = sums[blockIdx.x] + block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
        const int64_t idx = base + q;
        if (idx < n) out[idx] = run;
        run += local[q];
    }
}

inline size_t sort_align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Temporary bytes of exclusive_scan_i32 for n elements.
inline size_t scan_temp_bytes(int64_t n) {
    const int64_t chunks = std::max<int64_t>(1, (n + kScanChunk - 1) / kScanChunk);
    return sort_align256(sizeof(int32_t) * (size_t)chunks);
}

// out[i] = in[0] + ... + in[i-1] over distinct arrays (int32: the total must fit).
inline hipError_t exclusive_scan_i32(void *temp, size_t temp_bytes, const int32_t *in, int32_t *out, int64_t n,
                                     hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (temp_bytes < scan_temp_bytes(n)) return hipErrorInvalidValue;
    const int64_t chunks = (n + kScanChunk - 1) / kScanChunk;
    int32_t *sums = (int32_t *)temp;
    hipLaunchKernelGGL(scan_chunk_sums_kernel, dim3((unsigned)chunks), dim3(kScanThreads), 0, s, in, n, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, chunks);
    hipLaunchKernelGGL(scan_chunks_kernel, dim3((unsigned)chunks), dim3(kScanThreads), 0, s, in, n,
                       (const int32_t *)sums, out);
    return hipGetLastError();
}

// Temporary bytes of radix_sort_pairs for n pairs of key type K: the
// alternate key and value buffers, the digit counts and the scan's own.
template <class K>
size_t radix_sort_temp_bytes(int64_t n) {
    const int64_t nn = std::max<int64_t>(n, 1);
    const int64_t cnt = (int64_t)kSortDigits * sort_tiles(nn);
    return sort_align256(sizeof(K) * (size_t)nn) + sort_align256(sizeof(int32_t) * (size_t)nn) +
           2 * sort_align256(sizeof(int32_t) * (size_t)cnt) + scan_temp_bytes(cnt);
}

// Stable sort of n (key, value) pairs by bits [begin_bit, end_bit) of the
// key: kin/vin are read, kout/vout receive the result (distinct arrays).
template <class K>
hipError_t radix_sort_pairs(void *temp, size_t temp_bytes, const K *kin, K *kout, const int32_t *vin, int32_t *vout,
                            int64_t n, int begin_bit, int end_bit, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (temp_bytes < radix_sort_temp_bytes<K>(n) || end_bit <= begin_bit || end_bit > (int)(8 * sizeof(K)))
        return hipErrorInvalidValue;
    const int64_t ntiles = sort_tiles(n);
    const int64_t cnt = (int64_t)kSortDigits * ntiles;
    char *p = (char *)temp;
    K *kalt = (K *)p;
    p += sort_align256(sizeof(K) * (size_t)n);
    int32_t *valt = (int32_t *)p;
    p += sort_align256(sizeof(int32_t) * (size_t)n);
    int32_t *counts = (int32_t *)p;
    p += sort_align256(sizeof(int32_t) * (size_t)cnt);
    int32_t *offsets = (int32_t *)p;
    p += sort_align256(sizeof(int32_t) * (size_t)cnt);
    void *scan_temp = p;
    const int passes = (end_bit - begin_bit + 7) / 8;
    const K *ki = kin;
    const int32_t *vi = vin;
    for (int pass = 0; pass < passes; ++pass) {
        // the last pass lands in the output arrays
        const bool to_out = ((passes - 1 - pass) % 2) == 0;
        K *ko = to_out ? kout : kalt;
        int32_t *vo = to_out ? vout : valt;
        const int shift = begin_bit + 8 * pass;
        const int dmask = (1 << std::min(8, end_bit - shift)) - 1;  // bits past end_bit take no part
        hipLaunchKernelGGL(sort_histogram_kernel<K>, dim3((unsigned)ntiles), dim3(kSortWave), 0, s, ki, n, shift,
                           dmask, counts, ntiles);
        const hipError_t e = exclusive_scan_i32(scan_temp, scan_temp_bytes(cnt), counts, offsets, cnt, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sort_scatter_kernel<K>, dim3((unsigned)ntiles), dim3(kSortWave), 0, s, ki, vi, ko, vo, n,
                           shift, dmask, (const int32_t *)offsets, ntiles);
        ki = ko;
        vi = vo;
    }
    return hipGetLastError();
}

}  // namespace vecchia

// Preprocessing on the GPU: the m nearest previously ordered neighbours of
// every point (the conditioning sets J_i of Eq. (7), Sec. IV-B), the m
// nearest observed points of prediction points (kriging, Sec. V-C) and the
// Morton ordering (Sec. IV-A).
//
// Neighbour search: points are binned into a uniform grid over their bounding
// box (about two points per cell) by a stable radix sort of (cell, index), so
// every cell lists its points in ascending index and the points before i form
// a prefix of each list.  One wavefront serves one query point: it scans rings
// of cells around the query until no unscanned cell can hold a point closer
// than the current m-th best, keeping candidates in an LDS buffer that is
// sorted (bitonic, by squared distance then index) and cut back to m whenever
// it fills.  Early points (i below kBruteMax) scan all j < i instead.  The
// result is exactly the brute-force answer: the order (squared distance,
// index) is total and every candidate that could beat the m-th best is seen.
// Prediction points search all observed points the same way.  Great-circle
// sets (points as (longitude, latitude) in degrees) rank candidates by the
// haversine value on the same grid, with a haversine lower bound for the
// unscanned rings.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "sort.h"
#include "vecchia.h"

using vecchia::exclusive_scan_i32;
using vecchia::radix_sort_pairs;
using vecchia::radix_sort_temp_bytes;
using vecchia::scan_temp_bytes;

namespace {

constexpr int kWaveK = 64;
constexpr int kKnnWaves = 4;         // query wavefronts per block
constexpr int kKnnCap = 256;         // candidate buffer per wavefront (>= VECCHIA_MAX_M + 64)
constexpr int64_t kBruteMax = 8192;  // queries up to this index scan all earlier points
constexpr int kBoxBlocks = 256;
constexpr int kMaxGrid = 8192;
static_assert(kKnnCap >= VECCHIA_MAX_M + kWaveK, "candidate buffer too small");

// squared distance with each product rounded (no contraction), as the
// conditioning sets are defined
#pragma clang fp contract(off)
__device__ __forceinline__ double sqdist(double ax, double ay, double bx, double by) {
    const double dx = ax - bx;
    const double dy = ay - by;
    return dx * dx + dy * dy;
}
#pragma clang fp contract(on)

constexpr double kDeg2Rad = 0.017453292519943295769236907684886;

// haversine value sin^2(dlat/2) + cos lat_q cos lat_p sin^2(dlon/2), clamped
// to 1, differences in degrees first: monotone in the great-circle distance
#pragma clang fp contract(off)
__device__ __forceinline__ double hav_key(double lonq, double latq, double cq, double lonp, double latp, double cp) {
    const double s1 = sin(0.5 * ((latq - latp) * kDeg2Rad));
    const double s2 = sin(0.5 * ((lonq - lonp) * kDeg2Rad));
    const double h = s1 * s1 + (cq * cp) * (s2 * s2);
    return h > 1.0 ? 1.0 : h;
}
#pragma clang fp contract(on)

__device__ __forceinline__ bool pair_less(double d1, int32_t j1, double d2, int32_t j2) {
    return d1 < d2 || (d1 == d2 && j1 < j2);
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Grid of g x g cells of side h with origin (x0, y0), computed on the device
// from the bounding box.
struct GridParams {
    double x0, y0, h, inv_h;
    double xmax, ymax;
};

__host__ __device__ inline int grid_side(int64_t n) {
    double g = std::ceil(std::sqrt((double)n / 2.0));
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return (int)g;
}

// ---- bounding box -----------------------------------------------------------

__global__ void __launch_bounds__(256) box_partial_kernel(const double *__restrict__ locs, int64_t n,
                                                          double *__restrict__ part) {
    __shared__ double red[4][256];
    double xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = locs[2 * i], y = locs[2 * i + 1];
        xmin = fmin(xmin, x);
        xmax = fmax(xmax, x);
        ymin = fmin(ymin, y);
        ymax = fmax(ymax, y);
    }
    red[0][threadIdx.x] = xmin;
    red[1][threadIdx.x] = ymin;
    red[2][threadIdx.x] = xmax;
    red[3][threadIdx.x] = ymax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = fmin(red[1][threadIdx.x], red[1][threadIdx.x + s]);
            red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + s]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Reduces the partial boxes; with g > 0 also derives the grid (cell side h a
// hair larger than the box over g, so every point falls inside).
__global__ void __launch_bounds__(kBoxBlocks) box_final_kernel(const double *__restrict__ part, int g,
                                                               GridParams *__restrict__ gp) {
    __shared__ double red[4][kBoxBlocks];
    const int t = threadIdx.x;
    red[0][t] = part[4 * t + 0];
    red[1][t] = part[4 * t + 1];
    red[2][t] = part[4 * t + 2];
    red[3][t] = part[4 * t + 3];
    __syncthreads();
    for (int s = kBoxBlocks / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] = fmin(red[0][t], red[0][t + s]);
            red[1][t] = fmin(red[1][t], red[1][t + s]);
            red[2][t] = fmax(red[2][t], red[2][t + s]);
            red[3][t] = fmax(red[3][t], red[3][t + s]);
        }
        __syncthreads();
    }
    if (t == 0) {
        GridParams p;
        p.x0 = red[0][0];
        p.y0 = red[1][0];
        p.xmax = red[2][0];
        p.ymax = red[3][0];
        double w = fmax(p.xmax - p.x0, p.ymax - p.y0);
        if (!(w > 0.0) || !isfinite(w)) w = 1.0;
        p.h = g > 0 ? w / g * (1.0 + 1e-12) : w;
        p.inv_h = 1.0 / p.h;
        *gp = p;
    }
}

// ---- binning ----------------------------------------------------------------

__device__ __forceinline__ int cell_coord(double v, double v0, double inv_h, int g) {
    const double f = (v - v0) * inv_h;
    // NaN compares false and lands in cell 0: every index stays in range
    return (f >= 0.0) ? (f < (double)g ? (int)f : g - 1) : 0;
}

__global__ void fill_int_kernel(int32_t *__restrict__ a, int64_t count, int32_t v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        a[t] = v;
}

__global__ void cell_kernel(const double *__restrict__ locs, int64_t n, const GridParams *__restrict__ gp, int g,
                            int32_t *__restrict__ key, int32_t *__restrict__ val, int32_t *__restrict__ count) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const GridParams p = *gp;
    const int cx = cell_coord(locs[2 * i], p.x0, p.inv_h, g);
    const int cy = cell_coord(locs[2 * i + 1], p.y0, p.inv_h, g);
    const int c = cy * g + cx;
    key[i] = c;
    val[i] = (int32_t)i;
    atomicAdd(count + c, 1);
}

// Points in cell order; with clat (great-circle sets) also their cos(latitude).
__global__ void gather_sorted_kernel(const double *__restrict__ locs, int64_t n, const int32_t *__restrict__ idx,
                                     const double *__restrict__ clat, double2 *__restrict__ sxy,
                                     double *__restrict__ sclat) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t j = idx[p];
    sxy[p] = double2{locs[2 * j], locs[2 * j + 1]};
    if (clat) sclat[p] = clat[j];
}

// ---- queries ----------------------------------------------------------------

// One wavefront's candidate buffer: sorts [0, c) (padded to kKnnCap) by
// (distance, index), keeps min(c, k) entries and returns the new count.
__device__ __forceinline__ int trim_buffer(double *bd, int32_t *bj, int c, int k, int lane) {
    for (int t = c + lane; t < kKnnCap; t += kWaveK) {
        bd[t] = INFINITY;
        bj[t] = INT32_MAX;
    }
    wave_sync_lds();
    for (int size = 2; size <= kKnnCap; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < kKnnCap / 2; t += kWaveK) {
                const int a = 2 * stride * (t / stride) + (t % stride);
                const int b = a + stride;
                const bool up = (a & size) == 0;
                const double da = bd[a], db = bd[b];
                const int32_t ja = bj[a], jb = bj[b];
                const bool swap = up ? pair_less(db, jb, da, ja) : pair_less(da, ja, db, jb);
                if (swap) {
                    bd[a] = db;
                    bd[b] = da;
                    bj[a] = jb;
                    bj[b] = ja;
                }
            }
            wave_sync_lds();
        }
    }
    return c < k ? c : k;
}

struct TopK {
    double *bd;
    int32_t *bj;
    int c, k, lane;
    double thr_d;
    int32_t thr_j;

    __device__ __forceinline__ void trim() {
        c = trim_buffer(bd, bj, c, k, lane);
        if (c == k) {
            thr_d = bd[k - 1];
            thr_j = bj[k - 1];
        }
        wave_sync_lds();
    }

    // one candidate per lane (valid lanes only); wave-uniform call
    __device__ __forceinline__ void consider(bool valid, double d, int32_t j) {
        const bool accept = valid && pair_less(d, j, thr_d, thr_j);
        const uint64_t mask = __ballot(accept);
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
        if (accept) {
            bd[c + below] = d;
            bj[c + below] = j;
        }
        c += __popcll(mask);
        wave_sync_lds();
        if (c > kKnnCap - kWaveK) trim();
    }
};

// cell (dx, dy) of ring r (r >= 1) for position e in [0, 8r): the four sides
// of the square perimeter, each 2r cells long, without overlap
__device__ __forceinline__ void ring_cell(int r, int e, int &dx, int &dy) {
    const int side = e / (2 * r), off = e % (2 * r);
    if (side == 0) {
        dx = -r + off;
        dy = -r;
    } else if (side == 1) {
        dx = r;
        dy = -r + off;
    } else if (side == 2) {
        dx = r - off;
        dy = r;
    } else {
        dx = -r;
        dy = r - off;
    }
}

// Query i (0 <= i < nq): its candidates are the points j < lim of locs, with
// lim = i for conditioning sets (qlocs == NULL, query point locs[i]) and
// lim = n for prediction points (query point qlocs[i]).
//
// GCD: points are (longitude, latitude) degrees on the same grid, keys are
// hav_key values (clat / sclat hold cos(latitude) in input / cell order).
// An unscanned point lies at least a = r h degrees away in longitude or in
// latitude; with both spans within 180 degrees its haversine value is at
// least sin^2(a / 2) min(1, cos lat_q cos lat_min), cos lat_min the least
// cosine over the points' latitudes (all in [-90, 90]).  A query whose
// longitude span exceeds 180 degrees scans every cell.
template <bool GCD>
__global__ void __launch_bounds__(kKnnWaves *kWaveK) knn_query_kernel(
    const double *__restrict__ locs, int64_t n, const double *__restrict__ qlocs, int64_t nq, int32_t m,
    const double2 *__restrict__ sxy, const int32_t *__restrict__ sidx, const int32_t *__restrict__ cstart,
    const GridParams *__restrict__ gp, int g, const double *__restrict__ clat, const double *__restrict__ sclat,
    int32_t *__restrict__ nbr) {
    __shared__ double sbd[kKnnWaves][kKnnCap];
    __shared__ int32_t sbj[kKnnWaves][kKnnCap];
    const int w = threadIdx.x / kWaveK, lane = threadIdx.x % kWaveK;
    const int64_t i = blockIdx.x * (int64_t)kKnnWaves + w;
    if (i >= nq) return;  // whole wavefront; the kernel has no workgroup barrier
    const int64_t lim = qlocs ? n : i;
    const int k = (int)(lim < m ? lim : m);
    int32_t *out = nbr + i * (int64_t)m;
    if (k == 0) {
        for (int t = lane; t < m; t += kWaveK) out[t] = -1;
        return;
    }
    const double *qp = qlocs ? qlocs + 2 * i : locs + 2 * i;
    const double qx = qp[0], qy = qp[1];
    double cq = 0.0;
    if constexpr (GCD) cq = qlocs ? cos(qy * kDeg2Rad) : clat[i];
    TopK top{sbd[w], sbj[w], 0, k, lane, INFINITY, INT32_MAX};

    if (lim <= kBruteMax) {
        for (int64_t base = 0; base < lim; base += kWaveK) {
            const int64_t j = base + lane;
            const bool valid = j < lim;
            double d = 0.0;
            if (valid) {
                if constexpr (GCD) d = hav_key(qx, qy, cq, locs[2 * j], locs[2 * j + 1], clat[j]);
                else d = sqdist(qx, qy, locs[2 * j], locs[2 * j + 1]);
            }
            top.consider(valid, d, (int32_t)j);
        }
    } else {
        const GridParams p = *gp;
        const int cx = cell_coord(qx, p.x0, p.inv_h, g);
        const int cy = cell_coord(qy, p.y0, p.inv_h, g);
        double hfac = 0.0;  // GCD: min(1, cos lat_q cos lat_min), 0 when no bound applies
        if constexpr (GCD) {
            const double span = fmax(p.xmax, qx) - fmin(p.x0, qx);
            const double cmin = fmin(cos(p.y0 * kDeg2Rad), cos(p.ymax * kDeg2Rad));
            hfac = (span <= 180.0) ? fmin(1.0, cq * cmin) : 0.0;
        }
        for (int r = 0;; ++r) {
            const int ncell = (r == 0) ? 1 : 8 * r;
            for (int e0 = 0; e0 < ncell; e0 += kWaveK) {
                const int e = e0 + lane;
                int dx = 0, dy = 0;
                if (r > 0 && e < ncell) ring_cell(r, e, dx, dy);
                const int X = cx + dx, Y = cy + dy;
                const bool inside = e < ncell && X >= 0 && X < g && Y >= 0 && Y < g;
                int32_t pp = inside ? cstart[Y * g + X] : 0;
                const int32_t pe = inside ? cstart[Y * g + X + 1] : 0;
                // walk each lane's cell while its points precede lim
                for (;;) {
                    const bool active = pp < pe && sidx[pp] < lim;
                    if (__ballot(active) == 0) break;
                    double d = 0.0;
                    int32_t j = 0;
                    if (active) {
                        const double2 s = sxy[pp];
                        if constexpr (GCD) d = hav_key(qx, qy, cq, s.x, s.y, sclat[pp]);
                        else d = sqdist(qx, qy, s.x, s.y);
                        j = sidx[pp];
                        ++pp;
                    }
                    top.consider(active, d, j);
                }
            }
            const bool covered = cx - r <= 0 && cx + r >= g - 1 && cy - r <= 0 && cy + r >= g - 1;
            if (covered) break;
            if (top.c >= k) {
                if (top.c > k) top.trim();
                // every unscanned point lies at least r cells off in x or y:
                // its offset exceeds r h up to the rounding of the binning,
                // which the margins cover
                const double dmin = (double)r * p.h * (1.0 - 1e-9) - 1e-12 * (double)g * p.h;
                if constexpr (GCD) {
                    if (dmin > 0.0 && hfac > 0.0) {
                        const double sa = sin(0.5 * (fmin(dmin, 180.0) * kDeg2Rad));
                        if ((sa * sa) * hfac * (1.0 - 1e-9) > top.thr_d) break;
                    }
                } else {
                    if (dmin > 0.0 && dmin * dmin > top.thr_d) break;
                }
            }
        }
    }
    top.trim();
    for (int t = lane; t < m; t += kWaveK) out[t] = (t < top.c) ? top.bj[t] : -1;
}

__global__ void cos_lat_kernel(const double *__restrict__ locs, int64_t n, double *__restrict__ clat) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) clat[i] = cos(locs[2 * i + 1] * kDeg2Rad);
}

// ---- Morton ordering --------------------------------------------------------

#pragma clang fp contract(off)
__device__ __forceinline__ uint32_t morton_cell(double v, double lo, double hi) {
    const double w = hi - lo;
    if (!(w > 0.0)) return 0;
    double q = floor((v - lo) / w * 65536.0);
    q = q < 0.0 ? 0.0 : q;
    q = q > 65535.0 ? 65535.0 : q;
    return (uint32_t)q;
}
#pragma clang fp contract(on)

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__global__ void morton_code_kernel(const double *__restrict__ locs, int64_t n, const GridParams *__restrict__ gp,
                                   uint32_t *__restrict__ code, int32_t *__restrict__ val) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const GridParams p = *gp;
    const uint32_t qx = morton_cell(locs[2 * i], p.x0, p.xmax);
    const uint32_t qy = morton_cell(locs[2 * i + 1], p.y0, p.ymax);
    code[i] = spread16(qx) | (spread16(qy) << 1);
    val[i] = (int32_t)i;
}

// ---- approximate maxmin ordering ---------------------------------------------
//
// Rounds of elections over grids of G x G square cells (G = 2^min(r, Lmax))
// on the square box of side w = the larger side of the bounding box: each
// cell elects its unselected point nearest the cell centre (ties by index);
// a round's points follow the earlier rounds in ascending mix64(seed ^ i).
// The decisions use the same rounded operations as their definition (no
// contraction), so the permutation is exact.

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

#pragma clang fp contract(off)
__device__ __forceinline__ int64_t maxmin_cell(double v, double v0, double w, int64_t G) {
    double f = floor((v - v0) / w * (double)G);
    f = (f >= 0.0) ? f : 0.0;  // negative or NaN: cell 0, so every index stays in range
    f = f > (double)(G - 1) ? (double)(G - 1) : f;
    return (int64_t)f;
}

// cell index and squared distance to the cell centre of point i
__device__ __forceinline__ void maxmin_pos(const double *__restrict__ locs, int64_t i, const GridParams &p, double w,
                                           int64_t G, int64_t &c, double &d) {
    const double x = locs[2 * i], y = locs[2 * i + 1];
    const int64_t cx = maxmin_cell(x, p.x0, w, G), cy = maxmin_cell(y, p.y0, w, G);
    const double dx = x - (p.x0 + ((double)cx + 0.5) * w / (double)G);
    const double dy = y - (p.y0 + ((double)cy + 0.5) * w / (double)G);
    d = dx * dx + dy * dy;
    c = cy * G + cx;
}
#pragma clang fp contract(on)

__device__ __forceinline__ double maxmin_side(const GridParams &p) {
    const double w = fmax(p.xmax - p.x0, p.ymax - p.y0);
    return (w > 0.0) ? w : 1.0;
}

__global__ void fill_u64_kernel(uint64_t *__restrict__ a, int64_t count, uint64_t v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
        a[t] = v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, kWaveK);
        v = o < v ? o : v;
    }
    return v;
}

// phase 1: the least squared distance of each cell (non-negative doubles
// order as their bit patterns).  On the coarse grids (at most 16 cells) every
// wavefront first takes the minimum per cell, so a cell sees one atomic per
// wavefront instead of one per point.
__global__ void maxmin_dist_kernel(const double *__restrict__ locs, int64_t n, const GridParams *__restrict__ gp,
                                   int64_t G, const int32_t *__restrict__ sel, unsigned long long *__restrict__ cd) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool active = i < n && !sel[i];
    int64_t c = 0;
    double d = 0.0;
    if (active) {
        const GridParams p = *gp;
        maxmin_pos(locs, i, p, maxmin_side(p), G, c, d);
    }
    const unsigned long long key = (unsigned long long)__double_as_longlong(d);
    if (G * G <= 16) {  // uniform over the launch
        const int lane = threadIdx.x % kWaveK;
        for (int64_t cc = 0; cc < G * G; ++cc) {
            const unsigned long long v = wave_min_u64((active && c == cc) ? key : ~0ull);
            if (lane == 0 && v != ~0ull) atomicMin(cd + cc, v);
        }
    } else if (active) {
        atomicMin(cd + c, key);
    }
}

// phase 2: the least index at that distance
__global__ void maxmin_index_kernel(const double *__restrict__ locs, int64_t n, const GridParams *__restrict__ gp,
                                    int64_t G, const int32_t *__restrict__ sel,
                                    const unsigned long long *__restrict__ cd, int32_t *__restrict__ ci) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || sel[i]) return;
    const GridParams p = *gp;
    int64_t c;
    double d;
    maxmin_pos(locs, i, p, maxmin_side(p), G, c, d);
    if ((unsigned long long)__double_as_longlong(d) == cd[c]) atomicMin(ci + c, (int32_t)i);
}

// phase 3: elected points (all unselected ones when G == 0) join the round's list
__global__ void maxmin_elect_kernel(const double *__restrict__ locs, int64_t n, const GridParams *__restrict__ gp,
                                    int64_t G, int32_t *__restrict__ sel, const int32_t *__restrict__ ci,
                                    uint64_t seed, uint64_t *__restrict__ key, int32_t *__restrict__ val,
                                    int32_t *__restrict__ count) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || sel[i]) return;
    bool elected = true;
    if (G > 0) {
        const GridParams p = *gp;
        int64_t c;
        double d;
        maxmin_pos(locs, i, p, maxmin_side(p), G, c, d);
        elected = ci[c] == (int32_t)i;
    }
    if (!elected) return;
    sel[i] = 1;
    const int32_t slot = atomicAdd(count, 1);
    key[slot] = mix64(seed ^ (uint64_t)i);
    val[slot] = (int32_t)i;
}

__global__ void append_kernel(const int32_t *__restrict__ v, int64_t cnt, int64_t *__restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < cnt) out[t] = v[t];
}

__global__ void widen_kernel(const int32_t *__restrict__ v, int64_t n, int64_t *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = v[i];
}

// ---- workspace layouts ------------------------------------------------------

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct KnnLayout {
    size_t part, params, key, val, skey, sval, count, cstart, sxy, clat, sclat, temp, total, temp_bytes;
    int g;
    int64_t cells;
};

size_t knn_temp_bytes(int64_t n, int64_t cells) {
    return std::max(radix_sort_temp_bytes<uint32_t>(n), scan_temp_bytes(cells + 1));
}

KnnLayout knn_layout(int64_t n) {
    KnnLayout L{};
    L.g = grid_side(n);
    L.cells = (int64_t)L.g * L.g;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t o = 0;
    L.part = o;   o += align256(sizeof(double) * 4 * kBoxBlocks);
    L.params = o; o += align256(sizeof(GridParams));
    L.key = o;    o += align256(sizeof(int32_t) * nn);
    L.val = o;    o += align256(sizeof(int32_t) * nn);
    L.skey = o;   o += align256(sizeof(int32_t) * nn);
    L.sval = o;   o += align256(sizeof(int32_t) * nn);
    L.count = o;  o += align256(sizeof(int32_t) * (size_t)(L.cells + 1));
    L.cstart = o; o += align256(sizeof(int32_t) * (size_t)(L.cells + 1));
    L.sxy = o;    o += align256(sizeof(double2) * nn);
    L.clat = o;   o += align256(sizeof(double) * nn);
    L.sclat = o;  o += align256(sizeof(double) * nn);
    L.temp_bytes = knn_temp_bytes((int64_t)nn, L.cells);
    L.temp = o;   o += align256(L.temp_bytes);
    L.total = o;
    return L;
}

struct MortonLayout {
    size_t part, params, key, val, skey, sval, temp, total, temp_bytes;
};

MortonLayout morton_layout(int64_t n) {
    MortonLayout L{};
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t o = 0;
    L.part = o;   o += align256(sizeof(double) * 4 * kBoxBlocks);
    L.params = o; o += align256(sizeof(GridParams));
    L.key = o;    o += align256(sizeof(uint32_t) * nn);
    L.val = o;    o += align256(sizeof(int32_t) * nn);
    L.skey = o;   o += align256(sizeof(uint32_t) * nn);
    L.sval = o;   o += align256(sizeof(int32_t) * nn);
    L.temp_bytes = radix_sort_temp_bytes<uint32_t>((int64_t)nn);
    L.temp = o;   o += align256(L.temp_bytes);
    L.total = o;
    return L;
}

// Lmax: the least L >= 0 with 4^L >= n, plus 1, at most 15
int maxmin_levels(int64_t n) {
    int l = 0;
    while (l < 14 && ((int64_t)1 << (2 * l)) < n) ++l;
    return l + 1;
}

struct MaxminLayout {
    size_t part, params, sel, cd, ci, key, val, skey, sval, count, temp, total, temp_bytes;
    int64_t cells;
};

MaxminLayout maxmin_layout(int64_t n) {
    MaxminLayout L{};
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const int64_t G = (int64_t)1 << maxmin_levels(n);
    L.cells = G * G;
    size_t o = 0;
    L.part = o;   o += align256(sizeof(double) * 4 * kBoxBlocks);
    L.params = o; o += align256(sizeof(GridParams));
    L.sel = o;    o += align256(sizeof(int32_t) * nn);
    L.cd = o;     o += align256(sizeof(uint64_t) * (size_t)L.cells);
    L.ci = o;     o += align256(sizeof(int32_t) * (size_t)L.cells);
    L.key = o;    o += align256(sizeof(uint64_t) * nn);
    L.val = o;    o += align256(sizeof(int32_t) * nn);
    L.skey = o;   o += align256(sizeof(uint64_t) * nn);
    L.sval = o;   o += align256(sizeof(int32_t) * nn);
    L.count = o;  o += 256;
    L.temp_bytes = radix_sort_temp_bytes<uint64_t>((int64_t)nn);
    L.temp = o;   o += align256(L.temp_bytes);
    L.total = o;
    return L;
}

int bits_for(int64_t v) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) <= v) ++b;
    return b;
}

int blocks_for(int64_t count, int threads) { return (int)((count + threads - 1) / threads); }

}  // namespace

extern "C" size_t vecchia_knn_workspace_size(int64_t n) { return knn_layout(n < 0 ? 0 : n).total; }

namespace {

// Sets of nq queries against the n points of locs (self sets when qlocs is
// NULL, then nq = n).  The grid over locs serves the Euclidean metric.
int knn_run(const double *locs, int64_t n, const double *qlocs, int64_t nq, int32_t m, int32_t metric, int32_t *nbr,
            void *ws, size_t ws_bytes, hipStream_t s) {
    const KnnLayout L = knn_layout(n);
    if (!ws || ws_bytes < L.total) return VECCHIA_EWORKSPACE;
    const bool gcd = metric == VECCHIA_GREAT_CIRCLE;
    char *base = (char *)ws;
    double *part = (double *)(base + L.part);
    GridParams *gp = (GridParams *)(base + L.params);
    int32_t *key = (int32_t *)(base + L.key), *val = (int32_t *)(base + L.val);
    int32_t *skey = (int32_t *)(base + L.skey), *sval = (int32_t *)(base + L.sval);
    int32_t *count = (int32_t *)(base + L.count), *cstart = (int32_t *)(base + L.cstart);
    double2 *sxy = (double2 *)(base + L.sxy);
    double *clat = gcd ? (double *)(base + L.clat) : nullptr;
    double *sclat = gcd ? (double *)(base + L.sclat) : nullptr;
    void *temp = base + L.temp;
    if (n > 0) {
        if (gcd) hipLaunchKernelGGL(cos_lat_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, locs, n, clat);
        hipLaunchKernelGGL(box_partial_kernel, dim3(kBoxBlocks), dim3(256), 0, s, locs, n, part);
        hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(kBoxBlocks), 0, s, part, L.g, gp);
        hipLaunchKernelGGL(fill_int_kernel, dim3(std::min(blocks_for(L.cells + 1, 256), 4096)), dim3(256), 0, s,
                           count, L.cells + 1, 0);
        hipLaunchKernelGGL(cell_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, locs, n, gp, L.g, key, val,
                           count);
        if (hipGetLastError() != hipSuccess) return VECCHIA_EHIP;
        if (radix_sort_pairs<uint32_t>(temp, L.temp_bytes, (const uint32_t *)key, (uint32_t *)skey, val, sval, n, 0,
                                       bits_for(L.cells), s) != hipSuccess)
            return VECCHIA_EHIP;
        if (exclusive_scan_i32(temp, L.temp_bytes, count, cstart, L.cells + 1, s) != hipSuccess)
            return VECCHIA_EHIP;
        hipLaunchKernelGGL(gather_sorted_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, locs, n, sval,
                           (const double *)clat, sxy, sclat);
    }
    if (gcd)
        hipLaunchKernelGGL(knn_query_kernel<true>, dim3(blocks_for(nq, kKnnWaves)), dim3(kKnnWaves * kWaveK), 0, s,
                           locs, n, qlocs, nq, m, (const double2 *)sxy, (const int32_t *)sval,
                           (const int32_t *)cstart, (const GridParams *)gp, L.g, (const double *)clat,
                           (const double *)sclat, nbr);
    else
        hipLaunchKernelGGL(knn_query_kernel<false>, dim3(blocks_for(nq, kKnnWaves)), dim3(kKnnWaves * kWaveK), 0, s,
                           locs, n, qlocs, nq, m, (const double2 *)sxy, (const int32_t *)sval,
                           (const int32_t *)cstart, (const GridParams *)gp, L.g, (const double *)nullptr,
                           (const double *)nullptr, nbr);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

}  // namespace

extern "C" int vecchia_knn_metric(const double *locs, int64_t n, int32_t m, int32_t metric, int32_t *nbr, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (n < 0 || m < 0 || n > INT32_MAX) return VECCHIA_EINVAL;
    if (metric != VECCHIA_EUCLIDEAN && metric != VECCHIA_GREAT_CIRCLE) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (n == 0 || m == 0) return VECCHIA_OK;
    if (!locs || !nbr) return VECCHIA_EINVAL;
    return knn_run(locs, n, nullptr, n, m, metric, nbr, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int vecchia_knn(const double *locs, int64_t n, int32_t m, int32_t *nbr, void *ws, size_t ws_bytes,
                           void *stream) {
    return vecchia_knn_metric(locs, n, m, VECCHIA_EUCLIDEAN, nbr, ws, ws_bytes, stream);
}

extern "C" int vecchia_knn_query(const double *locs, int64_t n, const double *qlocs, int64_t nq, int32_t m,
                                 int32_t metric, int32_t *nbr, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0 || nq < 0 || m < 0 || n > INT32_MAX || nq > INT32_MAX) return VECCHIA_EINVAL;
    if (metric != VECCHIA_EUCLIDEAN && metric != VECCHIA_GREAT_CIRCLE) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (nq == 0 || m == 0) return VECCHIA_OK;
    if (!qlocs || !nbr || (n > 0 && !locs)) return VECCHIA_EINVAL;
    return knn_run(locs, n, qlocs, nq, m, metric, nbr, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" size_t vecchia_morton_workspace_size(int64_t n) { return morton_layout(n < 0 ? 0 : n).total; }

extern "C" int vecchia_morton_order(const double *locs, int64_t n, int64_t *perm, void *ws, size_t ws_bytes,
                                    void *stream) {
    if (n < 0 || n > INT32_MAX) return VECCHIA_EINVAL;
    if (n == 0) return VECCHIA_OK;
    if (!locs || !perm) return VECCHIA_EINVAL;
    const MortonLayout L = morton_layout(n);
    if (!ws || ws_bytes < L.total) return VECCHIA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    double *part = (double *)(base + L.part);
    GridParams *gp = (GridParams *)(base + L.params);
    uint32_t *key = (uint32_t *)(base + L.key), *skey = (uint32_t *)(base + L.skey);
    int32_t *val = (int32_t *)(base + L.val), *sval = (int32_t *)(base + L.sval);
    hipLaunchKernelGGL(box_partial_kernel, dim3(kBoxBlocks), dim3(256), 0, s, locs, n, part);
    hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(kBoxBlocks), 0, s, part, 0, gp);
    hipLaunchKernelGGL(morton_code_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, locs, n, gp, key, val);
    if (hipGetLastError() != hipSuccess) return VECCHIA_EHIP;
    if (radix_sort_pairs<uint32_t>(base + L.temp, L.temp_bytes, key, skey, val, sval, n, 0, 32, s) != hipSuccess)
        return VECCHIA_EHIP;
    hipLaunchKernelGGL(widen_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, sval, n, perm);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

// ---- random ordering ----------------------------------------------------------

namespace {

__global__ void random_key_kernel(int64_t n, uint64_t seed, uint64_t *__restrict__ key, int32_t *__restrict__ val) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        key[i] = mix64(seed ^ (uint64_t)i);
        val[i] = (int32_t)i;
    }
}

struct RandomLayout {
    size_t key, val, skey, sval, temp, total, temp_bytes;
};

RandomLayout random_layout(int64_t n) {
    RandomLayout L{};
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t o = 0;
    L.key = o;    o += align256(sizeof(uint64_t) * nn);
    L.val = o;    o += align256(sizeof(int32_t) * nn);
    L.skey = o;   o += align256(sizeof(uint64_t) * nn);
    L.sval = o;   o += align256(sizeof(int32_t) * nn);
    L.temp_bytes = radix_sort_temp_bytes<uint64_t>((int64_t)nn);
    L.temp = o;   o += align256(L.temp_bytes);
    L.total = o;
    return L;
}

}  // namespace

extern "C" size_t vecchia_random_order_workspace_size(int64_t n) { return random_layout(n < 0 ? 0 : n).total; }

extern "C" int vecchia_random_order(int64_t n, uint64_t seed, int64_t *perm, void *ws, size_t ws_bytes,
                                    void *stream) {
    if (n < 0 || n > INT32_MAX) return VECCHIA_EINVAL;
    if (n == 0) return VECCHIA_OK;
    if (!perm) return VECCHIA_EINVAL;
    const RandomLayout L = random_layout(n);
    if (!ws || ws_bytes < L.total) return VECCHIA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    uint64_t *key = (uint64_t *)(base + L.key), *skey = (uint64_t *)(base + L.skey);
    int32_t *val = (int32_t *)(base + L.val), *sval = (int32_t *)(base + L.sval);
    hipLaunchKernelGGL(random_key_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, seed, key, val);
    if (radix_sort_pairs<uint64_t>(base + L.temp, L.temp_bytes, key, skey, val, sval, n, 0, 64, s) != hipSuccess)
        return VECCHIA_EHIP;
    hipLaunchKernelGGL(widen_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, sval, n, perm);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

extern "C" size_t vecchia_maxmin_workspace_size(int64_t n) { return maxmin_layout(n < 0 ? 0 : n).total; }

extern "C" int vecchia_maxmin_order(const double *locs, int64_t n, uint64_t seed, int64_t *perm, void *ws,
                                    size_t ws_bytes, void *stream) {
    if (n < 0 || n > INT32_MAX) return VECCHIA_EINVAL;
    if (n == 0) return VECCHIA_OK;
    if (!locs || !perm) return VECCHIA_EINVAL;
    const MaxminLayout L = maxmin_layout(n);
    if (!ws || ws_bytes < L.total) return VECCHIA_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    double *part = (double *)(base + L.part);
    GridParams *gp = (GridParams *)(base + L.params);
    int32_t *sel = (int32_t *)(base + L.sel);
    unsigned long long *cd = (unsigned long long *)(base + L.cd);
    int32_t *ci = (int32_t *)(base + L.ci);
    uint64_t *key = (uint64_t *)(base + L.key), *skey = (uint64_t *)(base + L.skey);
    int32_t *val = (int32_t *)(base + L.val), *sval = (int32_t *)(base + L.sval);
    int32_t *count = (int32_t *)(base + L.count);
    const int lmax = maxmin_levels(n);
    const int nb = blocks_for(n, 256);
    hipLaunchKernelGGL(box_partial_kernel, dim3(kBoxBlocks), dim3(256), 0, s, locs, n, part);
    hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(kBoxBlocks), 0, s, part, 0, gp);
    hipLaunchKernelGGL(fill_int_kernel, dim3(std::min(nb, 4096)), dim3(256), 0, s, sel, n, 0);
    int64_t done = 0;
    for (int r = 0; done < n; ++r) {
        const bool last = r >= lmax + 33;
        const int64_t G = last ? 0 : (int64_t)1 << std::min(r, lmax);
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, count, 1, 0);
        if (!last) {
            const int64_t cells = G * G;
            const int cb = std::min(blocks_for(cells, 256), 4096);
            hipLaunchKernelGGL(fill_u64_kernel, dim3(cb), dim3(256), 0, s, (uint64_t *)cd, cells, ~(uint64_t)0);
            hipLaunchKernelGGL(fill_int_kernel, dim3(cb), dim3(256), 0, s, ci, cells, INT32_MAX);
            hipLaunchKernelGGL(maxmin_dist_kernel, dim3(nb), dim3(256), 0, s, locs, n, (const GridParams *)gp, G,
                               (const int32_t *)sel, cd);
            hipLaunchKernelGGL(maxmin_index_kernel, dim3(nb), dim3(256), 0, s, locs, n, (const GridParams *)gp, G,
                               (const int32_t *)sel, (const unsigned long long *)cd, ci);
        }
        hipLaunchKernelGGL(maxmin_elect_kernel, dim3(nb), dim3(256), 0, s, locs, n, (const GridParams *)gp, G, sel,
                           (const int32_t *)ci, seed, key, val, count);
        if (hipGetLastError() != hipSuccess) return VECCHIA_EHIP;
        int32_t cnt = 0;
        if (hipMemcpyAsync(&cnt, count, sizeof(cnt), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return VECCHIA_EHIP;
        if (cnt <= 0 || done + cnt > n) return VECCHIA_EHIP;  // every round elects at least one point
        if (radix_sort_pairs<uint64_t>(base + L.temp, L.temp_bytes, key, skey, val, sval, cnt, 0, 64, s) !=
            hipSuccess)
            return VECCHIA_EHIP;
        hipLaunchKernelGGL(append_kernel, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, (const int32_t *)sval,
                           (int64_t)cnt, perm + done);
        done += cnt;
    }
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

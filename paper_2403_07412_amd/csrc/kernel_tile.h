// Tiled kernel: one workgroup of W wavefronts per conditional, the augmented
// block held in registers as 16x16 tiles, the Cholesky blocked by tile
// columns with its trailing updates on FP64 matrix cores.
//
// Block layout (same augmented block as the unblocked kernel): rows 0..k-1
// neighbours, row k the point itself, row k+1 the observations, rows k+2..
// 16T-1 identity padding.  Factoring rows 0..k gives L_kk^2 = c_i and, in row
// k+1, the two forward solves of Algorithm 1 (POTRF + 2 TRSV, fused).
//
// Register tiles.  v_mfma_f64_16x16x4f64 leaves D[4r + l/16][l%16] in
// accumulator register r of lane l.  Every tile M of the block is kept in
// the transposed form of that layout ("T-layout"): lane (g, j) = (l/16, l%16),
// register r holds M[j][4r + g].  With the inner index of a product taken as
// kk = 4s + g in instruction s, a T-layout tile is directly the B operand of
// M' M^T-style products and the panel operands need no transposes:
//   TRSM  X^T = Linv A^T     A operand Linv[m][4s+g] (Linv in T-layout),
//                            B operand register s of the tile itself;
//   SYRK  A^T -= X_C X_R^T   both operands register s of the panel tiles.
// The result of each product lands again in T-layout.
//
// Per tile column t:
//   1. the owner of the diagonal tile factors it (16 columns, one row per lane,
//      64-bit DPP row broadcasts) and forms its inverse Linv_t (columns split
//      over the four lane groups, which yields Linv_t in T-layout directly);
//   2. owners of the tiles below apply X = A Linv_t^T (4 MFMAs per tile) and
//      publish X to the LDS panel;
//   3. owners of the trailing tiles subtract X_R X_C^T (4 MFMAs per tile).
// Gradient: the same back substitution as the unblocked kernel, by tiles:
//   x_t = Linv_t^T q_t, then q_C -= L_tC^T x_t for the tiles left of t.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "kernel_lds.h"

namespace vecchia {

typedef double dvec4 __attribute__((ext_vector_type(4)));

#ifndef VECCHIA_KEEP_DBETA
#define VECCHIA_KEEP_DBETA 1
#endif

__host__ __device__ constexpr int tile_count(int T) { return T * (T + 1) / 2; }
__host__ __device__ constexpr int tiles_per_wave(int T, int W) { return (tile_count(T) + W - 1) / W; }

// Occupancy target (wavefronts per SIMD) the register allocation aims at.
// Workgroups per CU are limited by LDS and by registers: each lane holds 8
// VGPRs per tile (16 when the beta-derivative tiles are kept) plus about 96
// for the diagonal factorisation, the covariance code and addressing.  Two
// shapes were measured to need about 64 more and get that allowance.
__host__ __device__ constexpr int tile_extra_vgprs(int T, int W) {
    return ((T == 5 && W == 4) || (T == 7 && W == 8)) ? 64 : 0;
}

// One more workgroup per CU is worth a few spilled registers: the kernel is
// bound by the latency of each conditional's dependency chain, and one more
// resident workgroup hides more of it than the spill code costs, as long as
// each wave keeps at least 102 VGPRs (5 wavefronts per SIMD).  Measured at
// m = 120 (T = 8, W = 4, value + gradient): 40 VGPRs spilled for a fourth
// workgroup, 8 % faster; W = 2 with 72 spilled for a fifth was 40 % slower,
// and W = 8 at 6 wavefronts per SIMD (85 VGPRs) lost up to a third.
constexpr int kTileSpillAllowance = 40;
constexpr int kTileMaxRaisedWaves = 5;

__host__ __device__ constexpr int tile_waves_per_simd(int T, int W, bool keep_d, bool gcd = false) {
    const int lds = ((T + (T > 1 ? 2 : 1)) * 256 + 272 + (gcd ? 9 : 8) * 16 * T + 80 + 2 * kExpTableSize) * 8;  // TileLds::BYTES
    const int blocks_lds = 163840 / lds;
    const int need = 8 * tiles_per_wave(T, W) * (keep_d ? 2 : 1) + 96 + tile_extra_vgprs(T, W);
    const int wps_regs = 512 / need;                 // wavefronts per SIMD the registers allow
    const int blocks_regs = (wps_regs * 4) / W;      // workgroups per CU the registers allow
    int blocks = blocks_lds < blocks_regs ? blocks_lds : blocks_regs;
    if (blocks < 1) blocks = 1;
    if (blocks + 1 <= blocks_lds) {                  // one more, if LDS allows and the spill stays small
        const int wps1 = ((blocks + 1) * W + 3) / 4;
        if (wps1 <= kTileMaxRaisedWaves && need - 512 / wps1 <= kTileSpillAllowance) blocks += 1;
    }
    int wps = (blocks * W + 3) / 4;
    if (wps < 1) wps = 1;
    if (wps > 8) wps = 8;
    return wps;
}

// Whether the gradient keeps the beta-derivative tiles in registers (one
// exponential per entry) or recomputes them after the solves: kept only when
// the extra registers cost no occupancy.
__host__ __device__ constexpr bool keep_dbeta(int T, int W, bool gcd = false) {
    return VECCHIA_KEEP_DBETA && tile_waves_per_simd(T, W, true, gcd) >= tile_waves_per_simd(T, W, false, gcd);
}

// LDS layout of the tiled kernel, in doubles.  The great-circle codes add
// cos(latitude) of every row at the end; the other offsets do not depend on it.
//
// One array of T tile slots serves both the panel and the stored inverses:
// while column t is processed, slot R > t holds the panel tile X_R, and
// slot t' <= t holds Linv_t' in N-layout (gradient only), written once the
// last TRSM of column t' is done.  A slot never holds both at once.  The
// factorisation publishes Linv_t for the TRSM in T-layout to CUR[t % 2]:
// the buffer it overwrites served column t - 2, whose readers all passed a
// workgroup barrier since.  A single tile column needs one such buffer.
template <int T, bool GCD = false>
struct TileLds {
    static constexpr int KP = 16 * T;
    static constexpr int NCUR = T > 1 ? 2 : 1;
    static constexpr int CUR = 0;                   // [NCUR][64 lanes][4] Linv_t of the current column, T-layout
    static constexpr int SLOT = CUR + NCUR * 256;   // [T][64 lanes][4]   panel X_R (slot R > t), Linv_t N-layout (slot t)
    static constexpr int DIAG = SLOT + T * 256;     // [16][17]           diagonal tile, row-major
    static constexpr int XY = DIAG + 272;           // [KP][2]            coordinates
    static constexpr int ZV = XY + 2 * KP;          // [KP]               observations
    static constexpr int YP = ZV + KP;              // [KP]               factor row k+1
    static constexpr int Q = YP + KP;               // [KP][2]            back-substitution right-hand sides
    static constexpr int UB = Q + 2 * KP;           // [KP][2]            solutions (u, b)
    static constexpr int SCAL = UB + 2 * KP;        // [16]               scalars: [0] L_kk
    static constexpr int RED = SCAL + 16;           // [2][32]            reductions (two values, up to 8 waves x 4 rows)
    static constexpr int EXPT = RED + 64;           // [64][2]            2^(j/64) as hi, lo for exp_neg_tab
    static constexpr int CL = EXPT + 2 * kExpTableSize;  // [KP]         cos(latitude) (great-circle codes only)
    static constexpr int TOTAL = CL + (GCD ? KP : 0);
    static constexpr size_t BYTES = (size_t)TOTAL * sizeof(double);
    static_assert(TOTAL == (T + NCUR) * 256 + 272 + (GCD ? 9 : 8) * KP + 80 + 2 * kExpTableSize,
                  "occupancy estimate out of date");
};

// Tile enumeration: column C descending, row R ascending inside a column, so
// the tiles still active after step t form a prefix and a round-robin owner
// assignment balances every step.
__device__ inline void tile_rc(int T, int idx, int &R, int &C) {
    int start = 0;
    R = -1;
    C = -1;
    for (int c = T - 1; c >= 0; --c) {
        const int cnt = T - c;
        if (idx < start + cnt) {
            C = c;
            R = c + (idx - start);
            return;
        }
        start += cnt;
    }
}

__device__ inline int tile_index(int T, int R, int C) {
    // tiles of columns T-1 .. C+1 come first
    const int before = (T - 1 - C) * (T - C) / 2;
    return before + (R - C);
}

template <int SRC>
__device__ __forceinline__ double bcast_row(double v) {
    // every lane of each 16-lane row receives lane SRC of that row (64-bit DPP row_newbcast)
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + SRC, 0xF, 0xF, false);
}

// acc -= v(lane SRC of this lane's row) * w, one fused 64-bit DPP FMA with a
// negated operand.  With NOP, two wait states precede it: a DPP source
// written by the instruction just before needs them, and the compiler does
// not look inside inline assembly for that hazard.
template <int SRC, bool NOP>
__device__ __forceinline__ void fms_bcast_row(double &acc, double v, double w) {
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(v), "v"(w), "i"(SRC));
    else
        asm volatile("v_fmac_f64_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(v), "v"(w), "i"(SRC));
}

// acc += acc(lane SRC of this lane's row) * w: the accumulator is also the
// broadcast source (one register, no copy).
template <int SRC, bool NOP>
__device__ __forceinline__ void fma_bcast_row_self(double &acc, double w) {
    if constexpr (NOP)
        asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(w), "i"(SRC));
    else
        asm volatile("v_fmac_f64_dpp %0, %0, %1 row_newbcast:%2 row_mask:0xf bank_mask:0xf"
                     : "+v"(acc)
                     : "v"(w), "i"(SRC));
}

// compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// 1/sqrt(x) for x > 0: the hardware estimate y (relative error near 2^-24)
// and one third-order correction y (1 + e/2 + 3e^2/8), e = 1 - x y^2.  The
// residual e is formed without rounding loss (x y split into h + hl), so
// the result is within about half an ulp; five dependent steps where two
// Newton steps take six.
__device__ __forceinline__ double rsqrt_refined(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double hl = fma(x, y, -h);  // x y = h + hl exactly
    const double e = fma(-hl, y, fma(-h, y, 1.0));
    const double p = fma(e, 0.375, 0.5);
    return fma(y * e, p, y);
}


// 64-bit DPP move of both halves of a double (any DPP control).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of each row by DPP (pairs, quads, half rows, rows);
// every lane of the row ends with the same bits.
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}

// Workgroup sums of two values in a fixed order (rows, then rows of waves in
// ascending order); every thread gets both totals.  `red` holds 2 * 4W doubles.
template <int W>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red) {
    const int l = threadIdx.x % kWave, w = threadIdx.x / kWave;
    a = row_sum16(a);
    b = row_sum16(b);
    __syncthreads();
    if (l % 16 == 0) {
        red[4 * w + l / 16] = a;
        red[4 * W + 4 * w + l / 16] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < 4 * W; ++i) {
        sa += red[i];
        sb += red[4 * W + i];
    }
    a = sa;
    b = sb;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry (a, b) of the augmented block for rows or columns past k, given the
// covariance entry v (nugget included): the observation row k+1 holds z of
// the other index, the padding beyond it is the identity.  The diagonal of
// row k+1 is never used as a result; 2^600 keeps its pivot positive (it
// exceeds the squared norm of the row by far for any finite data), so the
// factorisation needs no special case for it.
__device__ __forceinline__ double augment_value(int a, int b, int k, double v, const double *__restrict__ Z) {
    const int hi = a > b ? a : b, lo = a > b ? b : a;
    if (hi == k + 1) v = (lo == k + 1) ? 0x1p600 : Z[lo];
    if (hi > k + 1) v = (a == b) ? 1.0 : 0.0;
    return v;
}

// Stores a diagonal tile (T-layout registers) row-major into the DIAG area.
template <int T>
__device__ __forceinline__ void store_diag(const dvec4 &v, double *smem) {
    const int l = threadIdx.x % kWave, g = l / 16, j = l % 16;
#pragma unroll
    for (int r = 0; r < 4; ++r) smem[TileLds<T>::DIAG + j * 17 + 4 * r + g] = v[r];
}

// Copies Linv_t from CUR[t % 2] in T-layout (lane (g, j), register r:
// Linv[j][4r + g]) to slot t in N-layout (lane (g, n), register r:
// Linv[4r + g][n]), by the wave that owns it.
template <int T>
__device__ __forceinline__ void linv_to_nlayout(int t, double *smem) {
    const int l = threadIdx.x % kWave, g = l / 16, j = l % 16;
    const dvec4 v = *reinterpret_cast<const dvec4 *>(smem + TileLds<T>::CUR + (t & 1) * 256 + l * 4);
    double *Lt = smem + TileLds<T>::SLOT + t * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) Lt[(16 * (j % 4) + 4 * r + g) * 4 + j / 4] = v[r];
}

// Factors diagonal tile t, which the calling wave has stored row-major in the
// DIAG area of LDS; publishes Linv_t (T-layout, lane-major) to CUR[t % 2] and records L_kk
// and the part of factor row k+1 that falls in this tile.  Every row is
// factored: the padding rows have pivot 1 and the observation row's diagonal
// is 2^600 (augment_value), so their pivots are positive and nothing past row
// k reaches rows up to k.  A pivot that is not positive and finite turns
// L_kk, and with it the conditional's value, into NaN, which the caller
// reports.
template <int T>
__device__ __forceinline__ void factor_diag(int t, int k, double *smem) {
    using Ls = TileLds<T>;
    int l = threadIdx.x % kWave;
    asm volatile("" : "+v"(l));  // keep the lane masks below inside the tile loop (no hoisting)
    const int g = l / 16, j = l % 16;
    double *S = smem + Ls::DIAG;  // the caller stored the tile here, row-major with stride 17
    // this wave is the critical path of the workgroup: let it win instruction
    // issue over the other waves sharing its SIMD while it factors
    __builtin_amdgcn_s_setprio(3);
    wave_lds_sync();
    double R[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) R[c] = S[j * 17 + c];
    wave_lds_sync();

    const int base = 16 * t;
    const int jk = k - base;      // local index of row k (point i) if it lies in this tile
    const int jy = k + 1 - base;  // local index of row k+1 (observations) if it lies in this tile
    // Linv is built row by row alongside the factor.  Lane (g, j) keeps
    // W_j[4r + g] (r = 0..3), row j of the unit-scaled inverse: once column q
    // is known, W_j -= (L[j][q] / L[q][q]) W_q for the rows j below q, with
    // W_q broadcast from lane q; finally Linv[j][.] = W_j / L[j][j].  The
    // result is Linv in T-layout.
    double Wr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) Wr[r] = (j == 4 * r + g) ? 1.0 : 0.0;
    double myinv = 1.0;  // 1 / L[j][j], kept per lane as column j passes
    static_for<0, 16>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double piv = bcast_row<q>(R[q]);
        // no branch here: the pivot chain of the next column can then overlap
        // the trailing update of this one
        const double inv = rsqrt_refined(piv);
        // column q of L: L[j][q] below the diagonal, L[q][q] = piv inv in
        // lane q; the entries above the diagonal are never read
        const double lq = R[q] * inv;
        R[q] = lq;
        // trailing update first, it carries the next pivot:
        // R[c] -= L[j][q] L[c][q] with L[c][q] = lq of lane c
        static_for<q + 1, 16>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            fms_bcast_row<c, c == q + 1>(R[c], lq, lq);
        });
        myinv = (j == q) ? inv : myinv;
        // take the select here: sunk to the end it would keep all 16
        // inverses live through the factorisation
        asm volatile("" : "+v"(myinv));
        const double nlq_inv = (j > q) ? -(lq * inv) : 0.0;  // -L[j][q] / L[q][q]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == 0) fma_bcast_row_self<q, true>(Wr[r], nlq_inv);
            else fma_bcast_row_self<q, false>(Wr[r], nlq_inv);
        }
    });
#pragma unroll
    for (int r = 0; r < 4; ++r) Wr[r] *= myinv;
    // L_kk = 1 / (its refined reciprocal square-root pivot), within an ulp of
    // pivot * rsqrt(pivot)
    if (g == 0 && base <= k && k < base + 16 && j == jk) smem[Ls::SCAL + 0] = 1.0 / myinv;
    if (g == 0 && jy >= 0 && jy < 16 && j == jy) {
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < jy) smem[Ls::YP + base + c] = R[c];
    }
    double *Li = smem + Ls::CUR + (t & 1) * 256 + l * 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) Li[r] = Wr[r];
    __builtin_amdgcn_s_setprio(0);
}

// One conditional (modes as lds_conditional: qloc == NULL for the
// likelihood term of point i, else the prediction at qloc from row i of nbr).
template <int T, int W, int KC, bool GRAD>
__device__ __forceinline__ CondOut tile_conditional(const double *__restrict__ locs, const double *__restrict__ z,
                                    const int32_t *__restrict__ nbr, int64_t i, int64_t n, int32_t m,
                                    const double *qloc, const Params &P, double *smem) {
    constexpr bool GCD = kc_gcd(KC);
    using Ls = TileLds<T, GCD>;
    constexpr int NT = W * kWave;
    constexpr int NTW = tiles_per_wave(T, W);
    constexpr int NTILES = tile_count(T);
    constexpr int KP = Ls::KP;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int l = tid % kWave;
    const int g = l / 16, j = l % 16;
    const int64_t lim = qloc ? n : i;
    const int k = (int)(lim < m ? lim : m);
    double *XY = smem + Ls::XY;
    double *Z = smem + Ls::ZV;
    double *CLv = smem + Ls::CL;
    bool bad = false;

    // my tiles: slot s holds tile index w + W s; (R, C) packed as R * 32 + C, -1 if unused
    int sRC[NTW];
#pragma unroll
    for (int s = 0; s < NTW; ++s) {
        const int idx = w + W * s;
        int R_ = -1, C_ = -1;
        if (idx < NTILES) tile_rc(T, idx, R_, C_);
        sRC[s] = (R_ < 0) ? -1 : R_ * 32 + C_;
    }
#define SR(s) (sRC[s] < 0 ? -1 : (sRC[s] >> 5))
#define SC(s) (sRC[s] < 0 ? -1 : (sRC[s] & 31))

    __syncthreads();  // the previous conditional is done with smem
    // gather (Algorithm 1: s_{J_i}, y_{J_i}); indices are checked before use
    // and non-finite inputs flag the conditional (the covariance code below
    // assumes finite coordinates)
    for (int t = tid; t < KP; t += NT) {
        double x = 0.0, y = 0.0, zz = 0.0;
        if (t <= k) {
            int64_t jj = i;
            if (t < k) {
                const int32_t jn = nbr[i * (int64_t)m + t];
                const bool okj = (jn >= 0) && ((int64_t)jn < lim);
                bad |= !okj;
                jj = okj ? (int64_t)jn : 0;
            }
            if (t == k && qloc) {  // prediction point, observation taken as 0
                x = qloc[0];
                y = qloc[1];
            } else {
                const double2 p = *reinterpret_cast<const double2 *>(locs + 2 * jj);
                x = p.x;
                y = p.y;
                zz = z[jj];
            }
            bad |= !(isfinite(x) && isfinite(y) && isfinite(zz));
        }
        XY[2 * t] = x;
        XY[2 * t + 1] = y;
        Z[t] = zz;
        if constexpr (GCD) CLv[t] = cos(y * kDeg2Rad);
    }
    if (tid < kExpTableSize) {
        smem[Ls::EXPT + 2 * tid] = kExp2Frac64[tid].hi;
        smem[Ls::EXPT + 2 * tid + 1] = kExp2Frac64[tid].lo;
    }
    __syncthreads();

    // covariance generation straight into the register tiles.  Only tiles
    // that reach past row k (the observation row and the identity padding)
    // and diagonal tiles (the nugget) need per-entry cases; the branches on
    // them are uniform over the wavefront.  With the gradient, dC/dbeta is
    // kept in dtile from the same exponential when registers allow.
    constexpr bool KEEP_D = GRAD && keep_dbeta(T, W, GCD);
    const double *ET = smem + Ls::EXPT;
    dvec4 tile[NTW];
    dvec4 dtile[KEEP_D ? NTW : 1];
    const double s2b = P.sigma2 * P.inv_beta;
#pragma unroll
    for (int s = 0; s < NTW; ++s) {
        tile[s] = dvec4{0.0, 0.0, 0.0, 0.0};
        if constexpr (KEEP_D) dtile[s] = dvec4{0.0, 0.0, 0.0, 0.0};
        const int R_ = SR(s), C_ = SC(s);
        if (R_ < 0) continue;
        const int a = 16 * R_ + j;
        const double xa = XY[2 * a], ya = XY[2 * a + 1], ca = GCD ? CLv[a] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = 16 * C_ + 4 * r + g;
            double cv, db;
            cov_pair<KC, KEEP_D>(xa, ya, ca, XY[2 * b], XY[2 * b + 1], GCD ? CLv[b] : 0.0, P, s2b, ET, cv, db);
            tile[s][r] = cv;
            if constexpr (KEEP_D) dtile[s][r] = db;
        }
        if (R_ == C_) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (a == 16 * C_ + 4 * r + g) tile[s][r] += P.tau2;
        }
        if (16 * R_ + 15 > k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[s][r] = augment_value(a, 16 * C_ + 4 * r + g, k, tile[s][r], Z);
        }
        if (R_ == 0 && C_ == 0) store_diag<T>(tile[s], smem);
    }

    // blocked right-looking Cholesky
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
        // the lane's offset inside a tile slot, opaque to the compiler in every
        // step: otherwise it hoists one address register per slot out of the
        // loop, which at this register budget spill to scratch
        int lo = l * 4;
        asm volatile("" : "+v"(lo));
        // 1. diagonal tile t: fully updated, and stored to DIAG by its owner
        if (w == tile_index(T, t, t) % W) factor_diag<T>(t, k, smem);
        __syncthreads();
        // 2. tiles below: X = A Linv_t^T, published to the panel (T-layout).
        // With the gradient the register copy is kept in N-layout (the same
        // product with the operands swapped), the form the back substitution
        // feeds to the matrix cores.
        const double *Li = smem + Ls::CUR + (t & 1) * 256 + lo;
#pragma unroll
        for (int s = 0; s < NTW; ++s) {
            if (SC(s) == t && SR(s) > t) {
                const dvec4 li = *reinterpret_cast<const dvec4 *>(Li);
                dvec4 acc = {0.0, 0.0, 0.0, 0.0};
                dvec4 accn = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(li[q], tile[s][q], acc, 0, 0, 0);
                    if constexpr (GRAD) accn = __builtin_amdgcn_mfma_f64_16x16x4f64(tile[s][q], li[q], accn, 0, 0, 0);
                }
                *reinterpret_cast<dvec4 *>(smem + Ls::SLOT + SR(s) * 256 + lo) = acc;
                tile[s] = GRAD ? accn : acc;
            }
        }
        __syncthreads();
        // Linv_t has served its last TRSM: the back substitution wants it in
        // N-layout, copied by its owner to slot t (its panel tile X_t was
        // last read by the trailing update of column t - 1, before the
        // barriers above)
        if constexpr (GRAD) {
            if (w == tile_index(T, t, t) % W) linv_to_nlayout<T>(t, smem);
        }
        // 3. trailing update of the tiles right of column t
#pragma unroll
        for (int s = 0; s < NTW; ++s) {
            if (SC(s) > t) {
                const dvec4 xr = *reinterpret_cast<const dvec4 *>(smem + Ls::SLOT + SR(s) * 256 + lo);
                const dvec4 xc = *reinterpret_cast<const dvec4 *>(smem + Ls::SLOT + SC(s) * 256 + lo);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    tile[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xc[q], xr[q], tile[s], 0, 0, 0);
                // the next diagonal tile is now final: hand it to the factorisation
                if (SR(s) == t + 1 && SC(s) == t + 1) store_diag<T>(tile[s], smem);
            }
        }
    }
    // observation row k+1 from the tiles left of its diagonal tile: in
    // T-layout lane (g, jy) holds it, in N-layout register jy/4 of the lanes
    // of row group jy%4
    const int ty = (k + 1) / 16, jy = (k + 1) % 16;
#pragma unroll
    for (int s = 0; s < NTW; ++s) {
        if (SR(s) == ty && SC(s) < ty) {
            if constexpr (GRAD) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (4 * r + g == jy) smem[Ls::YP + 16 * SC(s) + j] = tile[s][r];
            } else {
                if (j == jy) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) smem[Ls::YP + 16 * SC(s) + 4 * r + g] = tile[s][r];
                }
            }
        }
    }
    __syncthreads();

    CondOut o;
    const double Lkk = smem[Ls::SCAL + 0];
    const double wv = smem[Ls::YP + k];
    o.ell = -0.5 * (kLog2Pi + 2.0 * log(Lkk) + wv * wv);
    o.g0 = o.g1 = o.g2 = 0.0;
    o.var = Lkk * Lkk;
    o.mean = Z[k] - wv * Lkk;

    if constexpr (GRAD) {
        const double c = Lkk * Lkk;
        const double rr = wv / Lkk;
        const double half = 0.5 * (rr * rr - 1.0 / c);
        // back substitution with L^T for both right-hand sides at once, on
        // the matrix cores.  A 16 x 16 operand in N-layout (lane (g, n),
        // register r holds M[4r + g][n]) enters a product as M^T when passed
        // first and as M when passed second, and the product comes out in
        // N-layout.  With the right-hand sides as columns 0 and 1 of X:
        // x_t = Linv_t^T q_t, then q_C -= L_tC^T x_t for the tiles of row t;
        // x_t leaves the first product already laid out as the second
        // operand of the next.  Every wave forms x_t itself, so one barrier
        // per step suffices.  Q holds (q_u, q_b) pairs, UB receives (u, b).
        double *Q = smem + Ls::Q, *UB = smem + Ls::UB;
        const double *YP = smem + Ls::YP;
        for (int t = tid; t < KP; t += NT) {
            Q[2 * t] = (t < k) ? rr * YP[t] : (t == k ? half * Lkk : 0.0);
            Q[2 * t + 1] = (t == k) ? Lkk : 0.0;
        }
        __syncthreads();
        const bool rhs_lane = j < 2;  // lanes of columns 0 and 1
#pragma unroll 1
        for (int t = T - 1; t >= 0; --t) {
            int qo = 2 * g + j;  // opaque per step, as in the factorisation loop
            asm volatile("" : "+v"(qo));
            const dvec4 li = *reinterpret_cast<const dvec4 *>(smem + Ls::SLOT + t * 256 + l * 4);
            dvec4 xq;
#pragma unroll
            for (int q = 0; q < 4; ++q) xq[q] = rhs_lane ? Q[2 * (16 * t + 4 * q + g) + j] : 0.0;
            dvec4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q) x = __builtin_amdgcn_mfma_f64_16x16x4f64(li[q], xq[q], x, 0, 0, 0);
            if (w == tile_index(T, t, t) % W && rhs_lane) {
#pragma unroll
                for (int r = 0; r < 4; ++r) UB[2 * (16 * t + 4 * r + g) + j] = x[r];
            }
#pragma unroll
            for (int s = 0; s < NTW; ++s) {
                if (SR(s) == t && SC(s) < t) {
                    dvec4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < 4; ++q) d = __builtin_amdgcn_mfma_f64_16x16x4f64(tile[s][q], x[q], d, 0, 0, 0);
                    if (rhs_lane) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) Q[32 * SC(s) + 8 * r + qo] -= d[r];
                    }
                }
            }
            __syncthreads();
        }
        // dl/dtau2 = u^T b; dl/dbeta = sum_{a > b} D_ab (u_a b_b + u_b b_a).
        // u and b vanish past row k, so entries there add exact zeros; in a
        // diagonal tile the symmetric pairs are both visited and weighted by
        // one half, and D_aa (zero in exact arithmetic, about 2^-500 sigma2 /
        // beta^2 after sqrt_pos) is set to zero.
        double ub = 0.0;
        for (int t = tid; t <= k; t += NT) ub += UB[2 * t] * UB[2 * t + 1];
        double gb = 0.0;
#pragma unroll
        for (int s = 0; s < NTW; ++s) {
            const int R_ = SR(s), C_ = SC(s);
            if (R_ < 0 || 16 * R_ > k) continue;
            const int a = 16 * R_ + j;
            const double2 uba = *reinterpret_cast<const double2 *>(UB + 2 * a);
            dvec4 db4;
            if constexpr (KEEP_D) {
                db4 = dtile[s];
            } else {
                const double xa = XY[2 * a], ya = XY[2 * a + 1], ca = GCD ? CLv[a] : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int b = 16 * C_ + 4 * r + g;
                    double cv, db;
                    cov_pair<KC, true>(xa, ya, ca, XY[2 * b], XY[2 * b + 1], GCD ? CLv[b] : 0.0, P, s2b, ET, cv,
                                       db);
                    db4[r] = db;
                }
            }
            double w = 1.0;
            if (R_ == C_) {  // wave-uniform: only diagonal tiles hold a == b
                w = 0.5;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (a == 16 * C_ + 4 * r + g) db4[r] = 0.0;
            }
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double2 ubb = *reinterpret_cast<const double2 *>(UB + 2 * (16 * C_ + 4 * r + g));
                acc = fma(db4[r], fma(uba.x, ubb.y, ubb.x * uba.y), acc);
            }
            gb = fma(w, acc, gb);
        }
        block_sum2<W>(ub, gb, smem + Ls::RED);
        o.g2 = ub;
        o.g0 = (0.5 * (rr * rr * c - 1.0) - P.tau2 * ub) / P.sigma2;
        o.g1 = gb;
    }
    const bool anybad = __syncthreads_or(bad ? 1 : 0) != 0;
    o.bad = anybad || !isfinite(o.ell) || !isfinite(o.g0) || !isfinite(o.g1) || !isfinite(o.g2);
    return o;
#undef SR
#undef SC
}

}  // namespace vecchia

// Tiled kernel: one workgroup of W wavefronts per conditional, the augmented
// block held in registers as 16x16 tiles, the Cholesky blocked by tile
// columns with its trailing updates on FP64 matrix cores and its triangular
// solves by substitution.
//
// Block layout (same augmented block as the unblocked kernel): rows 0..k-1
// neighbours, row k the point itself, row k+1 the observations, rows k+2..
// 16T-1 identity padding.  Factoring rows 0..k gives L_kk^2 = c_i and, in row
// k+1, the two forward solves of Algorithm 1 (POTRF + 2 TRSV, fused).
//
// Register tiles.  v_mfma_f64_16x16x4f64 leaves D[4r + l/16][l%16] in
// accumulator register r of lane l, and every tile M of the block is kept in
// that layout ("N-layout"): lane (g, n) = (l/16, l%16), register r holds
// M[4r + g][n].  The transposed form ("T-layout", register r of lane (g, j)
// holding M[j][4r + g]) is the one panel tiles take in LDS, because as
// either MFMA operand a T-layout tile X enters a product directly:
//   SYRK   A_RC -= X_R X_C^T   operands -X_R and X_C, register s of each,
//                              accumulating straight into the N-layout tile;
// and an N-layout tile passed as the first operand enters as its transpose,
// which is what the back substitution of the gradient needs (L_tC^T x).
//
// Per tile column t:
//   1. the owner of the diagonal tile factors it (one row per lane, 64-bit
//      DPP row broadcasts) and publishes the strictly lower factor and the
//      inverse pivots;
//   2. the owners of the tiles below solve X L_tt^T = A in registers by
//      forward substitution over the 16 columns (column c of an N-layout
//      tile lives in lane c of every 16-lane row, so each step is one DPP
//      broadcast FMA per register), and publish X to LDS in T-layout;
//   3. the owners of the trailing tiles subtract X_R X_C^T (4 MFMAs per
//      tile), the next diagonal tile first, so that its factorisation
//      overlaps the other updates of the column.
// Gradient: back substitution with L^T by tiles: x_t = L_tt^-T q_t by
// substitution (one wave), then q_C -= L_tC^T x_t on the matrix cores for
// the tiles of row t.  No step multiplies by an explicit inverse, so every
// solve is backward stable, as in the unblocked kernel.
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

// LDS layout of the tiled kernel, in doubles.  The great-circle codes add
// cos(latitude) of every row at the end; the other offsets do not depend on it.
//
// CUR[t % NPAR] receives diagonal tile t before its factorisation (row-major,
// row stride 17) and then its strictly lower factor, with 1 / L_jj in
// column 16 and again, contiguous, after the 16 x 17 block.  With several waves the buffer alternates by the parity of t:
// the one tile t + 1 is stored into served column t - 1, whose readers all
// passed a workgroup barrier since.  One array of T slots (DS doubles each)
// serves both the panel and, with the gradient, the factored diagonal tiles:
// while column t is processed, slot R > t holds the panel tile X_R (T-layout,
// lane-major), and slot t' <= t holds factor t' in the CUR format, copied
// there once every reader of X_t' has passed a barrier.
//
// A workgroup that evaluates G parameter vectors of one conditional in
// lockstep keeps G copies of everything that depends on the parameters (CUR,
// SLOT, YP, Q, UB, SCAL, RED); the gathered coordinates, observations and the
// exponential table are shared.  G = 1 is the one-vector layout.  With one
// wavefront per vector (INPLACE, also for G = 1) there is no CUR: the
// wavefront stores diagonal tile t + 1 into slot t + 1 once its trailing
// updates have read X_(t+1) there, and the tile is factored in place.
template <int T, int W, bool GRAD, bool GCD = false, int G = 1>
struct TileLds {
    static constexpr int KP = 16 * T;
    static constexpr int DS = 288;                        // a 16 x 17 tile, then 16 inverse pivots
    static constexpr bool INPLACE = W == 1;
    static constexpr int NPAR = (W > 1 && T > 1) ? 2 : 1;
    static constexpr int CUR = 0;                         // [G][NPAR][DS]  diagonal tile / its factor
    static constexpr int SLOT = CUR + (INPLACE ? 0 : G * NPAR * DS);  // [G][T][DS] panel tiles / factors
    static constexpr int XY = SLOT + G * T * DS;          // [KP][2]        coordinates
    static constexpr int ZV = XY + 2 * KP;                // [KP]           observations
    static constexpr int YP = ZV + KP;                    // [G][KP]        factor row k+1
    static constexpr int Q = YP + G * KP;                 // [G][KP][2]     back-substitution right-hand sides (gradient),
    static constexpr int UB = Q;                          //                overwritten in place by the solutions (u, b)
    static constexpr int SCAL = Q + (GRAD ? G * 2 * KP : 0);  // [G][16]    scalars: [0] L_kk
    static constexpr int RED = SCAL + G * 16;             // [G][2][4W]     reductions (two values, W waves x 4 rows)
    static constexpr int EXPT = RED + G * 8 * W;          // [64][2]        2^(j/64) as hi, lo for exp_neg_tab
    static constexpr int CL = EXPT + 2 * kExpTableSize;   // [KP]           cos(latitude) (great-circle codes only)
    static constexpr int TOTAL = CL + (GCD ? KP : 0);
    static constexpr size_t BYTES = (size_t)TOTAL * sizeof(double);
    // per-parameter-vector strides
    static constexpr int CUR_G = NPAR * DS, SLOT_G = T * DS, YP_G = KP, QUB_G = 2 * KP, SCAL_G = 16, RED_G = 8 * W;
};

// TileLds<T, W, grad, gcd, G>::TOTAL, for the occupancy estimate.
__host__ __device__ constexpr int tile_lds_doubles(int T, int W, bool grad, bool gcd, int G = 1) {
    return (W == 1 ? 0 : G * ((W > 1 && T > 1) ? 2 : 1) * 288) + G * T * 288 +
           16 * T * (3 + G * (1 + (grad ? 2 : 0)) + (gcd ? 1 : 0)) + G * (16 + 8 * W) + 2 * kExpTableSize;
}
static_assert(TileLds<8, 4, true, false>::TOTAL == tile_lds_doubles(8, 4, true, false), "LDS estimate out of date");
static_assert(TileLds<3, 1, false, true>::TOTAL == tile_lds_doubles(3, 1, false, true), "LDS estimate out of date");
static_assert(TileLds<4, 1, true, true, 4>::TOTAL == tile_lds_doubles(4, 1, true, true, 4), "LDS estimate out of date");
static_assert(TileLds<5, 2, false, false, 2>::TOTAL == tile_lds_doubles(5, 2, false, false, 2), "LDS estimate out of date");

// Parameter vectors a workgroup evaluates in lockstep, per shape: four for
// the one-wavefront shapes (up to five tile rows: six rows make 21 tiles,
// past the 20 one wavefront holds), where the four wavefronts share the
// gathered neighbours and the pair distances; other shapes keep one vector
// (G = 1).
// Only these group sizes are compiled.
__host__ __device__ constexpr int lockstep_group(int T, int W) { return (T <= 5 && W == 1) ? 4 : 1; }

// Shapes measured faster with one more workgroup per CU than the register
// estimate below allows, at the price of a small spill:
//   T = 8, W = 4 (m from 110 to 125): value + gradient 67.0 ms at four
//     workgroups (9-11 VGPRs spilled) against 79.3 ms at three for the
//     10^6-point, m = 120 field; a fifth workgroup (102 VGPRs) spilled more
//     and took 91 ms;
//   T = 10, W = 4 (m from 142 to 157): 32.5 ms at three workgroups against
//     41.7 ms at two (34.1 ms at four) for 250,000 uniform points, m = 150,
//     nu = 3/2, value + gradient;
//   T = 4, W = 2 (m from 47 to 62; LDS leaves room only without the
//     gradient): 2.82 ms at nine workgroups against 2.89 ms at eight for the
//     same points at m = 60, value only.
// T = 7 and 9 with W = 4, T = 2 to 4 with W = 1 and T = 3, 5, 6 with W = 2
// measured no faster one workgroup up.  Other shapes keep the estimate.
__host__ __device__ constexpr bool tile_measured_raise(int T, int W, bool gcd) {
    return ((T == 8 || T == 10) && W == 4 && !gcd) || (T == 4 && W == 2 && !gcd);
}

// Occupancy target (wavefronts per SIMD) the register allocation aims at.
// Workgroups per CU are limited by LDS and by registers: each lane holds 8
// VGPRs per tile (16 when the beta-derivative tiles are kept) plus about 72
// for the diagonal factorisation, the covariance code and addressing (the
// compiler reports 143 VGPRs for T = 8, W = 4 with the gradient, nine tiles).
// A lockstep workgroup (G parameter vectors) has G W wavefronts.
__host__ __device__ constexpr int tile_waves_per_simd(int T, int W, bool keep_d, bool grad, bool gcd = false,
                                                      int G = 1) {
    const int lds = tile_lds_doubles(T, W, grad, gcd, G) * 8;
    const int blocks_lds = 163840 / lds;
    const int need = 8 * tiles_per_wave(T, W) * (keep_d ? 2 : 1) + 72 + (gcd ? 16 : 0);
    const int wps_regs = 512 / need;                 // wavefronts per SIMD the registers allow
    const int blocks_regs = (wps_regs * 4) / (W * G);  // workgroups per CU the registers allow
    int blocks = blocks_lds < blocks_regs ? blocks_lds : blocks_regs;
    if (blocks < 1) blocks = 1;
    if (G == 1 && !keep_d && tile_measured_raise(T, W, gcd) && blocks + 1 <= blocks_lds) blocks += 1;
    int wps = (blocks * W * G + 3) / 4;
    if (wps < 1) wps = 1;
    if (wps > 8) wps = 8;
    return wps;
}

// Whether the gradient keeps the beta-derivative tiles in registers (one
// covariance evaluation per entry) or recomputes them after the solves.  For
// the Matern codes on Euclidean distances an evaluation is about 32
// instructions, and the tiles are kept only when the extra registers cost no
// occupancy.  The great-circle codes spend two sines, an arcsine and (power
// exponential) a logarithm and an exponential per entry: there the tiles are
// kept whenever two wavefronts per SIMD still fit (measured: the 250,000-point
// great-circle power-exponential gradient took 11.7 ms keeping them at two
// wavefronts per SIMD, 17.0 ms recomputing at three).  The one-wavefront
// shape of two tile rows keeps them as well (measured: 250,000 points,
// m = 30, value + gradient 1.25 ms keeping at four wavefronts per SIMD, 1.33
// ms recomputing at five).  Lockstep workgroups follow the one-vector
// decision: the two ways round the derivative contract their arithmetic
// differently, and the lockstep results must be the one-vector bits.
__host__ __device__ constexpr bool keep_dbeta(int T, int W, bool gcd = false) {
    return VECCHIA_KEEP_DBETA &&
           (tile_waves_per_simd(T, W, true, true, gcd) >= tile_waves_per_simd(T, W, false, true, gcd) ||
            (gcd && tile_waves_per_simd(T, W, true, true, gcd) >= 2) || (T == 2 && W == 1));
}

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

// Sums of two values over the W wavefronts of a parameter vector's group in a
// fixed order (rows, then rows of waves in ascending order); every thread of
// the group gets both totals.  `red` holds 2 * 4W doubles per group.  Every
// wavefront of the workgroup calls it together.
template <int W>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red) {
    const int l = threadIdx.x % kWave, w = (threadIdx.x / kWave) % W;
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

// Stores an N-layout tile (lane (g, n), register r: M[4r + g][n]) row-major
// with row stride 17 at D.
__device__ __forceinline__ void store_rowmajor17(const dvec4 &v, double *D) {
    const int l = threadIdx.x % kWave, g = l / 16, n = l % 16;
#pragma unroll
    for (int r = 0; r < 4; ++r) D[(4 * r + g) * 17 + n] = v[r];
}

// Writes an N-layout tile to a panel slot in T-layout, lane-major: the reader
// lane (g', j) finds M[j][4r' + g'] at slot[(16 g' + j) 4 + r'].  Element
// (4r + g, n) of this lane goes to reader lane (n % 4, 4r + g), register n / 4.
__device__ __forceinline__ void store_panel_tlayout(const dvec4 &v, double *slot) {
    const int l = threadIdx.x % kWave, g = l / 16, n = l % 16;
#pragma unroll
    for (int r = 0; r < 4; ++r) slot[(16 * (n % 4) + 4 * r + g) * 4 + n / 4] = v[r];
}

// Factors diagonal tile t, which the calling wave has stored row-major (stride
// 17) in D, in place: row j of D becomes the strictly lower part of row j of
// the factor (zeros from column j on) and D[j][16] = 1 / L_jj.  Records L_kk
// and the part of factor row k+1 that falls in this tile.  Every row is
// factored: the padding rows have pivot 1 and the observation row's diagonal
// is 2^600 (augment_value), so their pivots are positive and nothing past row
// k reaches rows up to k.  A pivot that is not positive and finite turns
// L_kk, and with it the conditional's value, into NaN, which the caller
// reports.
template <int T>
__device__ __forceinline__ void factor_diag(int t, int k, double *D, double *scal, double *yp) {
    int l = threadIdx.x % kWave;
    asm volatile("" : "+v"(l));  // keep the lane masks below inside the tile loop (no hoisting)
    const int g = l / 16, j = l % 16;
    // this wave is the critical path of the workgroup: let it win instruction
    // issue over the other waves sharing its SIMD while it factors
    __builtin_amdgcn_s_setprio(3);
    wave_lds_sync();
    double R[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) R[c] = D[j * 17 + c];
    wave_lds_sync();

    const int base = 16 * t;
    const int jk = k - base;      // local index of row k (point i) if it lies in this tile
    const int jy = k + 1 - base;  // local index of row k+1 (observations) if it lies in this tile
    double myinv = 1.0;           // 1 / L[j][j], kept per lane as column j passes
    static_for<0, 16>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double piv = bcast_row<q>(R[q]);
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
    });
    // L_kk = 1 / (its refined reciprocal square-root pivot), within an ulp of
    // pivot * rsqrt(pivot)
    if (g == 0 && j == jk) scal[0] = 1.0 / myinv;
    if (g == 0 && jy >= 0 && jy < 16 && j == jy) {
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < jy) yp[base + c] = R[c];
    }
    // publish: the four row groups hold the same rows and write a quarter of
    // the columns each
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (c % 4 == g) D[j * 17 + c] = (c < j) ? R[c] : 0.0;
    if (g == 0) D[j * 17 + 16] = myinv;
    if (g == 1) D[272 + j] = myinv;
    __builtin_amdgcn_s_setprio(0);
}

// Forward substitution X L^T = A for the N-layout tiles x[0..P) held in
// registers (row a of a tile in register a / 4 of row group a % 4, column n
// in lane n): with the strictly lower factor Ls and the inverse pivots in D
// (the CUR format), column c is final at step c, and column n > c loses
// A[.][c] L[n][c] / L[c][c].  Column c of every row group sits in lane c of
// that row, so each step is one DPP broadcast FMA per register; the inverse
// pivots scale the columns at the end.  Backward stable like any triangular
// substitution (no explicit inverse).  The weights of four steps are loaded
// while the previous four steps run.
template <int P>
__device__ __forceinline__ void panel_solve(dvec4 (&x)[P], const double *D) {
    const int n = threadIdx.x % 16;
    const double *Lrow = D + n * 17;  // row n of the strictly lower factor
    const double *dinv = D + 272;     // 1 / L_cc, contiguous
    double la[4], da[4], w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        la[q] = Lrow[q];
        da[q] = dinv[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = -(la[q] * da[q]);
    double xs[P][4];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) xs[p][r] = x[p][r];
    static_for<0, 4>([&](auto gc) {
        constexpr int G = decltype(gc)::value;
        if constexpr (G < 3) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                la[q] = Lrow[4 * G + 4 + q];
                da[q] = dinv[4 * G + 4 + q];
            }
        }
        static_for<0, 4>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr int c = 4 * G + q;
            static_for<0, P>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                // the first DPP read of a register follows its write by at least three instructions,
                // except at the very first step
                fma_bcast_row_self<c, c == 0 && p == 0>(xs[p][0], w[q]);
                fma_bcast_row_self<c, false>(xs[p][1], w[q]);
                fma_bcast_row_self<c, false>(xs[p][2], w[q]);
                fma_bcast_row_self<c, false>(xs[p][3], w[q]);
            });
        });
        if constexpr (G < 3) {
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = -(la[q] * da[q]);
        }
    });
    const double dn = dinv[n];
#pragma unroll
    for (int p = 0; p < P; ++p) x[p] = dvec4{xs[p][0] * dn, xs[p][1] * dn, xs[p][2] * dn, xs[p][3] * dn};
}

// One conditional (modes as lds_conditional: qloc == NULL for the
// likelihood term of point i, else the prediction at qloc from row i of nbr).
//
// With G > 1 (W = 1) the workgroup evaluates the conditional of point i for G
// parameter vectors at once (likelihood mode only): wavefront q takes vector
// q, passes its parameters in P and receives its result.  The wavefronts
// share the gather and the pair distances (each evaluates a G-th of them and
// exchanges them through LDS) and otherwise factor and solve their own
// vector, synchronising only with themselves.  Every vector's arithmetic is
// the one the single-vector form performs, in the same order, so the results
// are bitwise the same.  (Factoring the G diagonal tiles of a column in one
// wavefront, one tile per 16-lane row group, returned NaN now and then for
// the vectors held in row groups 1 and 3, in the first workgroups of small
// launches; each vector's wavefront factors its own tile instead.)
template <int T, int W, int KC, bool GRAD, int G = 1>
__device__ __forceinline__ CondOut tile_conditional(const double *__restrict__ locs, const double *__restrict__ z,
                                    const int32_t *__restrict__ nbr, int64_t i, int64_t n, int32_t m,
                                    const double *qloc, const Params &P, double *smem) {
    static_assert(G == 1 || G == 2 || G == 4, "one, two or four parameter vectors per workgroup");
    constexpr bool GCD = kc_gcd(KC);
    using Ls = TileLds<T, W, GRAD, GCD, G>;
    constexpr int NT = G * W * kWave;
    constexpr int NTG = W * kWave;  // threads per parameter vector
    constexpr int NTW = tiles_per_wave(T, W);
    constexpr int NTILES = tile_count(T);
    constexpr int KP = Ls::KP;
    constexpr int DS = Ls::DS;
    const int tid = threadIdx.x;
    const int wg = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int w = G > 1 ? wg % W : wg;   // wavefront within the vector's group
    const int wq = G > 1 ? wg / W : 0;   // the group's parameter vector
    const int tg = tid % NTG;            // thread within the group
    double *const CURq = smem + Ls::CUR + wq * Ls::CUR_G;
    double *const SLOTq = smem + Ls::SLOT + wq * Ls::SLOT_G;
    double *const YPq = smem + Ls::YP + wq * Ls::YP_G;
    double *const SCALq = smem + Ls::SCAL + wq * Ls::SCAL_G;
    // synchronisation of the wavefronts that share a vector's tiles: the whole
    // workgroup, except with one wavefront per vector, where each wavefront
    // works on its own vector alone (in lockstep groups, between the shared
    // phases: the gather, and the distance exchanges)
    auto group_sync = [&]() {
        if constexpr (W == 1)
            wave_lds_sync();
        else
            __syncthreads();
    };
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

    // covariance generation straight into the N-layout register tiles: lane
    // (g, n) register r of tile (R, C) is entry (16R + 4r + g, 16C + n).
    // Only tiles that reach past row k (the observation row and the identity
    // padding) and diagonal tiles (the nugget) need per-entry cases; the
    // branches on them are uniform over the wavefront.  With the gradient,
    // dC/dbeta is kept in dtile from the same exponential when registers allow.
    constexpr bool KEEP_D = GRAD && keep_dbeta(T, W, GCD);
    const double *ET = smem + Ls::EXPT;
    dvec4 tile[NTW];
    dvec4 dtile[KEEP_D ? NTW : 1];
    const double s2b = P.sigma2 * P.inv_beta;
    // With one wavefront per vector (INPLACE) every group needs the same
    // distances: each group's wavefront evaluates those of every G-th (tile,
    // register) pair, 64 lanes at a time, into the panel slots past slot 0,
    // which hold nothing yet (and nothing any more when the gradient's
    // contraction needs the distances again).
    constexpr bool SHARE_D = Ls::INPLACE && G > 1 && T >= 2;
    constexpr int DCH = SHARE_D ? ((T - 1) * DS) / kWave : 1;  // 64-double chunks per vector past slot 0
    static_assert(!SHARE_D || G * DCH >= 4 * NTW, "the shared distances fit in the panel slots");
    auto dslot = [&](int p) -> double * { return smem + Ls::SLOT + (p / DCH) * Ls::SLOT_G + DS + (p % DCH) * kWave; };
    if constexpr (SHARE_D) {
#pragma unroll
        for (int s = 0; s < NTW; ++s) {
            const int b = 16 * SC(s) + j;
            const double xb = XY[2 * b], yb = XY[2 * b + 1], cb = GCD ? CLv[b] : 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if ((4 * s + r) % G != wq) continue;  // wave-uniform
                const int a = 16 * SR(s) + 4 * r + g;
                dslot(4 * s + r)[l] = pair_dist_pow<KC>(XY[2 * a], XY[2 * a + 1], GCD ? CLv[a] : 0.0, xb, yb, cb, P,
                                                        ET);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < NTW; ++s) {
        tile[s] = dvec4{0.0, 0.0, 0.0, 0.0};
        if constexpr (KEEP_D) dtile[s] = dvec4{0.0, 0.0, 0.0, 0.0};
        const int R_ = SR(s), C_ = SC(s);
        if (R_ < 0) continue;
        const int b = 16 * C_ + j;
        const double xb = XY[2 * b], yb = XY[2 * b + 1], cb = GCD ? CLv[b] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = 16 * R_ + 4 * r + g;
            double cv, db;
            if constexpr (SHARE_D)
                cov_from_dist<KC, KEEP_D>(dslot(4 * s + r)[l], P, s2b, ET, cv, db);
            else
                cov_pair<KC, KEEP_D>(XY[2 * a], XY[2 * a + 1], GCD ? CLv[a] : 0.0, xb, yb, cb, P, s2b, ET, cv, db);
            tile[s][r] = cv;
            if constexpr (KEEP_D) dtile[s][r] = db;
        }
        if (R_ == C_) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (16 * R_ + 4 * r + g == b) tile[s][r] += P.tau2;
        }
        if (16 * R_ + 15 > k) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[s][r] = augment_value(16 * R_ + 4 * r + g, b, k, tile[s][r], Z);
        }
        if (R_ == 0 && C_ == 0) store_rowmajor17(tile[s], Ls::INPLACE ? SLOTq : CURq);
    }
    // every wavefront has read the shared distances before any writes a
    // panel tile over them
    if constexpr (SHARE_D) __syncthreads();

    // blocked right-looking Cholesky
#pragma unroll 1
    for (int t = 0; t < T; ++t) {
        // the lane's offset inside a tile slot, opaque to the compiler in every
        // step: otherwise it hoists one address register per slot out of the
        // loop, which at this register budget spill to scratch
        int lo = l * 4;
        asm volatile("" : "+v"(lo));
        const int par = Ls::INPLACE ? t * DS : (Ls::NPAR == 2 ? (t & 1) : 0) * DS;
        double *D = (Ls::INPLACE ? SLOTq : CURq) + par;
        const bool diag_owner = w == tile_index(T, t, t) % W;
        // 1. diagonal tile t (fully updated, stored to D by its owner)
        if (diag_owner) factor_diag<T>(t, k, D, SCALq, YPq);
        group_sync();
        // the factor goes to slot t for the back substitution: the panel tile
        // X_t it replaces was last read by the trailing update of column t - 1
        if constexpr (GRAD && !Ls::INPLACE) {
            if (diag_owner) {
                double *St = SLOTq + t * DS;
                for (int e = l; e < DS; e += kWave) St[e] = D[e];
            }
        }
        // 2. tiles below: X = A L_t^-T by substitution, kept in registers
        // (N-layout, the factor tile itself) and published in T-layout
#pragma unroll
        for (int s = 0; s < NTW; ++s) {
            if (SC(s) == t && SR(s) > t) {
                dvec4 one[1] = {tile[s]};
                panel_solve<1>(one, D);
                tile[s] = one[0];
                store_panel_tlayout(tile[s], SLOTq + SR(s) * DS);
            }
        }
        group_sync();
        // 3. trailing update of the tiles right of column t, the next diagonal
        // tile first: it is then handed to the factorisation
        double *Dn = CURq + (Ls::NPAR == 2 ? ((t + 1) & 1) : 0) * DS;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int s = 0; s < NTW; ++s) {
                const bool nextdiag = SR(s) == t + 1 && SC(s) == t + 1;
                if (SC(s) > t && (pass == 0) == nextdiag) {
                    const dvec4 xr = *reinterpret_cast<const dvec4 *>(SLOTq + SR(s) * DS + lo);
                    const dvec4 xc = *reinterpret_cast<const dvec4 *>(SLOTq + SC(s) * DS + lo);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        tile[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xr[q], xc[q], tile[s], 0, 0, 0);
                    if (nextdiag && !Ls::INPLACE) store_rowmajor17(tile[s], Dn);
                }
            }
        }
        if constexpr (Ls::INPLACE) {
            // X_(t+1) in slot t + 1 has had its last reader (this wavefront)
#pragma unroll
            for (int s = 0; s < NTW; ++s)
                if (SR(s) == t + 1 && SC(s) == t + 1) store_rowmajor17(tile[s], SLOTq + (t + 1) * DS);
        }
    }
    // observation row k+1 from the tiles left of its diagonal tile: row jy of
    // an N-layout tile is register jy / 4 of row group jy % 4
    const int ty = (k + 1) / 16, jy = (k + 1) % 16;
#pragma unroll
    for (int s = 0; s < NTW; ++s) {
        if (SR(s) == ty && SC(s) < ty) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (4 * r + g == jy) YPq[16 * SC(s) + j] = tile[s][r];
        }
    }
    group_sync();

    CondOut o;
    const double Lkk = SCALq[0];
    const double wv = YPq[k];
    o.ell = -0.5 * (kLog2Pi + 2.0 * log(Lkk) + wv * wv);
    o.g0 = o.g1 = o.g2 = 0.0;
    o.var = Lkk * Lkk;
    o.mean = Z[k] - wv * Lkk;

    if constexpr (GRAD) {
        const double c = Lkk * Lkk;
        const double rr = wv / Lkk;
        const double half = 0.5 * (rr * rr - 1.0 / c);
        // back substitution with L^T for both right-hand sides at once.  Q
        // holds (q_u, q_b) pairs, and (u, b) replace them in place (UB is
        // the same array): block t of q is read only by the solve that
        // writes block t of the solution, and later updates touch blocks
        // C < t only.  Per tile row t, from the last: the owner of the
        // diagonal tile solves L_tt^T x_t = q_t by substitution (lanes of row
        // groups 0 and 1 hold the two right-hand sides, lane n entry n), then
        // the owners of the tiles (t, C), C < t, subtract L_tC^T x_t from q_C
        // on the matrix cores: an N-layout tile as the first operand enters
        // as its transpose, and x_t as the second operand sits in lanes
        // (g, j < 2), register q holding x_j[4q + g].
        double *Q = smem + Ls::Q + wq * Ls::QUB_G, *UB = smem + Ls::UB + wq * Ls::QUB_G;
        const double *YP = YPq;
        for (int t = tg; t < KP; t += NTG) {
            Q[2 * t] = (t < k) ? rr * YP[t] : (t == k ? half * Lkk : 0.0);
            Q[2 * t + 1] = (t == k) ? Lkk : 0.0;
        }
        group_sync();
#pragma unroll 1
        for (int t = T - 1; t >= 0; --t) {
            const double *St = SLOTq + t * DS;  // strictly lower L_tt, 1 / L_jj in column 16
            if (w == tile_index(T, t, t) % W) {
                double qv = (g < 2) ? Q[2 * (16 * t + j) + g] : 0.0;
                // column c from the last: x_c = q_c / L_cc, then q_n -= L_cn x_c (n < c);
                // weights -L[c][n] / L[c][c] (zero for n >= c), four steps loaded ahead
                double la[4], da[4], wg[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    la[q] = St[(15 - q) * 17 + j];
                    da[q] = St[272 + 15 - q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) wg[q] = -(la[q] * da[q]);
                static_for<0, 4>([&](auto gc) {
                    constexpr int S = decltype(gc)::value;  // steps 4S .. 4S + 3 from the last column
                    if constexpr (S < 3) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            la[q] = St[(11 - 4 * S - q) * 17 + j];
                            da[q] = St[272 + 11 - 4 * S - q];
                        }
                    }
                    static_for<0, 4>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        fma_bcast_row_self<15 - 4 * S - q, true>(qv, wg[q]);
                    });
                    if constexpr (S < 3) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) wg[q] = -(la[q] * da[q]);
                    }
                });
                if (g < 2) UB[2 * (16 * t + j) + g] = qv * St[272 + j];
            }
            group_sync();
            if (t > 0) {
                int qo = 2 * g + j;  // opaque per step, as in the factorisation loop
                asm volatile("" : "+v"(qo));
                const bool rhs_lane = j < 2;
                dvec4 xq;
#pragma unroll
                for (int q = 0; q < 4; ++q) xq[q] = rhs_lane ? UB[2 * (16 * t + 4 * q + g) + j] : 0.0;
#pragma unroll
                for (int s = 0; s < NTW; ++s) {
                    if (SR(s) == t && SC(s) < t) {
                        dvec4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            d = __builtin_amdgcn_mfma_f64_16x16x4f64(tile[s][q], xq[q], d, 0, 0, 0);
                        if (rhs_lane) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) Q[32 * SC(s) + 8 * r + qo] -= d[r];
                        }
                    }
                }
                group_sync();
            }
        }
        // dl/dtau2 = u^T b; dl/dbeta = sum_{a > b} D_ab (u_a b_b + u_b b_a).
        // u and b vanish past row k, so entries there add exact zeros; in a
        // diagonal tile the symmetric pairs are both visited and weighted by
        // one half, and D_aa (zero in exact arithmetic, about 2^-500 sigma2 /
        // beta^2 after sqrt_pos) is set to zero.
        double ub = 0.0;
        for (int t = tg; t <= k; t += NTG) ub += UB[2 * t] * UB[2 * t + 1];
        if constexpr (SHARE_D && !KEEP_D) {
            // the distances again, shared as in the fill, once every wavefront
            // is past its back substitution (the last reader of its slots)
            __syncthreads();
#pragma unroll
            for (int s = 0; s < NTW; ++s) {
                if (16 * SR(s) > k) continue;
                const int b = 16 * SC(s) + j;
                const double xb = XY[2 * b], yb = XY[2 * b + 1], cb = GCD ? CLv[b] : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if ((4 * s + r) % G != wq) continue;  // wave-uniform
                    const int a = 16 * SR(s) + 4 * r + g;
                    dslot(4 * s + r)[l] = pair_dist_pow<KC>(XY[2 * a], XY[2 * a + 1], GCD ? CLv[a] : 0.0, xb, yb, cb,
                                                            P, ET);
                }
            }
            __syncthreads();
        }
        double gb = 0.0;
#pragma unroll
        for (int s = 0; s < NTW; ++s) {
            const int R_ = SR(s), C_ = SC(s);
            if (R_ < 0 || 16 * R_ > k) continue;
            const int b = 16 * C_ + j;
            const double2 ubb = *reinterpret_cast<const double2 *>(UB + 2 * b);
            dvec4 db4;
            if constexpr (KEEP_D) {
                db4 = dtile[s];
            } else {
                const double xb = XY[2 * b], yb = XY[2 * b + 1], cb = GCD ? CLv[b] : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = 16 * R_ + 4 * r + g;
                    double cv, db;
                    if constexpr (SHARE_D)
                        cov_from_dist<KC, true>(dslot(4 * s + r)[l], P, s2b, ET, cv, db);
                    else
                        cov_pair<KC, true>(XY[2 * a], XY[2 * a + 1], GCD ? CLv[a] : 0.0, xb, yb, cb, P, s2b, ET, cv,
                                           db);
                    db4[r] = db;
                }
            }
            double wt = 1.0;
            if (R_ == C_) {  // wave-uniform: only diagonal tiles hold a == b
                wt = 0.5;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (16 * R_ + 4 * r + g == b) db4[r] = 0.0;
            }
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double2 uba = *reinterpret_cast<const double2 *>(UB + 2 * (16 * R_ + 4 * r + g));
                acc = fma(db4[r], fma(uba.x, ubb.y, ubb.x * uba.y), acc);
            }
            gb = fma(wt, acc, gb);
        }
        block_sum2<W>(ub, gb, smem + Ls::RED + wq * Ls::RED_G);
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

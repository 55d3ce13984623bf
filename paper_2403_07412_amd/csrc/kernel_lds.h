// Unblocked LDS kernel: one workgroup (256 threads) per conditional, the
// whole augmented block packed in LDS.
//
// For point i with k = min(i, m) neighbours the block factored is the
// (k+2) x (k+2) lower triangle
//
//        [ Sigma_NN        .     . ]   rows 0..k-1: neighbours (nugget on the diagonal)
//   A =  [ v^T        Sigma_ii   . ]   row k: the point itself
//        [ y_N^T      y_i        * ]   row k+1: observations (its diagonal is never used)
//
// Factoring rows 0..k right-looking (Algorithm 1's POTRF) yields in row k the
// solve v' = L^{-1} v with L_kk^2 = c_i (the conditional variance), and in
// row k+1 the solve of [y_N; y_i] (both of Algorithm 1's TRSVs), whose last
// entry is (y_i - mu_i) / sqrt(c_i).  So
//   l_i = -1/2 (log 2 pi + 2 log L_kk + L_{k+1,k}^2).
//
// Gradient: with b = Sigma_aug^{-1} e_k c_i = [-Sigma_NN^{-1} v; 1] and
// s = [Sigma_NN^{-1} y_N; 0], r = (y_i - mu_i)/c_i, u = r s + (r^2 - 1/c)/2 b,
// every parameter derivative of l_i is u^T (dSigma_aug/dp) b.  Both b and u
// come from one back substitution with L_aug^T of
//   q_b = [0; sqrt(c)] and q_u = [r y'; (r^2 - 1/c) sqrt(c) / 2].
// Then  dl/dtau2 = u^T b,  dl/dsigma2 = ((r^2 c - 1)/2 - tau2 u^T b) / sigma2
// (Sigma_aug - tau2 I is proportional to sigma2 and Sigma_aug b = c e_k), and
// dl/dbeta = sum over a != b of u_a D_ab b_b with D = dC/dbeta recomputed.
#pragma once

#include "device_common.h"

namespace vecchia {

// Per-conditional results.  mean and var are the conditional mean and
// variance of the point's observation given its set (mu_i and c_i; with the
// point's own observation taken as 0 they are the kriging prediction).
struct CondOut {
    double ell, g0, g1, g2, mean, var;
    bool bad;
};

__host__ __device__ constexpr int64_t tri(int64_t a) { return a * (a + 1) / 2; }

// LDS bytes the unblocked kernel needs for conditioning sets of up to m points.
__host__ __device__ inline size_t lds_kernel_smem_bytes(int m) {
    int64_t rows = (int64_t)m + 2;
    return (size_t)(tri(rows) + 6 * (int64_t)(m + 2) + 16) * sizeof(double);
}

// One conditional.  Likelihood mode (qloc == NULL): point i of the n points,
// k = min(i, m) neighbours, all with indices below i.  Prediction mode: the
// point is the location qloc with observation 0, k = min(n, m) neighbours
// with indices below n, row i of nbr.
template <int KC, bool GRAD>
__device__ __forceinline__ CondOut lds_conditional(const double *__restrict__ locs, const double *__restrict__ z,
                                   const int32_t *__restrict__ nbr, int64_t i, int64_t n, int32_t m,
                                   const double *qloc, const Params &P, double *smem) {
    constexpr int NT = 256;
    constexpr int F = kc_family(KC);
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    const int64_t lim = qloc ? n : i;
    const int k = (int)(lim < m ? lim : m);
    const int rows = k + 2;  // rows 0..k+1
    double *A = smem;
    double *X = A + tri(m + 2);
    double *Y = X + (m + 2);
    double *Zv = Y + (m + 2);
    double *Q1 = Zv + (m + 2);
    double *Q2 = Q1 + (m + 2);
    double *CL = Q2 + (m + 2);   // cos(latitude), great-circle codes
    double *red = CL + (m + 2);  // reduction scratch
    bool mybad = false;

    __syncthreads();  // the previous conditional is done with smem
    // gather (Algorithm 1: s_{J_i}, y_{J_i}); every index is checked before use
    for (int t = tid; t <= k; t += NT) {
        int64_t j = i;
        if (t < k) {
            const int32_t jj = nbr[i * (int64_t)m + t];
            const bool okj = (jj >= 0) && ((int64_t)jj < lim);
            mybad |= !okj;
            j = okj ? (int64_t)jj : 0;
        }
        const bool self = t == k && qloc;
        X[t] = self ? qloc[0] : locs[2 * j];
        Y[t] = self ? qloc[1] : locs[2 * j + 1];
        Zv[t] = self ? 0.0 : z[j];
        if constexpr (kc_gcd(KC)) CL[t] = cos(Y[t] * kDeg2Rad);
        mybad |= !(isfinite(X[t]) && isfinite(Y[t]) && isfinite(Zv[t]));
    }
    __syncthreads();

    // covariance generation (batched-kernel step of Algorithm 1): rows by waves, columns by lanes
    for (int a = wave; a <= k + 1; a += NT / kWave) {
        double *row = A + tri(a);
        if (a <= k) {
            const double xa = X[a], ya = Y[a], ca = kc_gcd(KC) ? CL[a] : 0.0;
            for (int b = lane; b <= a; b += kWave) {
                const double r = cov_r<KC>(xa, ya, ca, X[b], Y[b], kc_gcd(KC) ? CL[b] : 0.0, P);
                const double c = matern_r<F>(r, P.sigma2);
                row[b] = (a == b) ? c + P.tau2 : c;
            }
        } else {
            for (int b = lane; b <= k; b += kWave) row[b] = Zv[b];
        }
    }

    // right-looking Cholesky of rows 0..k; row k+1 is carried along (the forward solves)
    for (int j = 0; j <= k; ++j) {
        __syncthreads();
        const double piv = A[tri(j) + j];
        mybad |= !(piv > 0.0) || !isfinite(piv);
        const double d = sqrt(piv);
        for (int r = j + 1 + tid; r < rows; r += NT) A[tri(r) + j] = A[tri(r) + j] / d;
        __syncthreads();
        if (tid == 0) A[tri(j) + j] = d;
        for (int r = j + 1 + wave; r < rows; r += NT / kWave) {
            const double arj = A[tri(r) + j];
            const int lmax = (r == k + 1) ? k : r;  // the observation row's diagonal is never needed
            for (int l = j + 1 + lane; l <= lmax; l += kWave) A[tri(r) + l] -= arj * A[tri(l) + j];
        }
    }
    __syncthreads();

    CondOut o;
    const double Lkk = A[tri(k) + k];
    const double w = A[tri(k + 1) + k];
    o.ell = -0.5 * (kLog2Pi + 2.0 * log(Lkk) + w * w);
    o.g0 = o.g1 = o.g2 = 0.0;
    o.var = Lkk * Lkk;
    o.mean = Zv[k] - w * Lkk;

    if constexpr (GRAD) {
        const double c = Lkk * Lkk;
        const double rr = w / Lkk;  // (y_i - mu_i) / c_i
        const double half = 0.5 * (rr * rr - 1.0 / c);
        for (int t = tid; t <= k; t += NT) {
            Q1[t] = (t < k) ? rr * A[tri(k + 1) + t] : half * Lkk;
            Q2[t] = (t < k) ? 0.0 : Lkk;
        }
        // back substitution L_aug^T x = q, column by column from k down to 0:
        // u goes to U (over the consumed observations), b over the consumed observation row of A
        double *U = Zv;
        double *Bv = A + tri(k + 1);
        for (int j = k; j >= 0; --j) {
            __syncthreads();
            const double ljj = A[tri(j) + j];
            const double x1 = Q1[j] / ljj;
            const double x2 = Q2[j] / ljj;
            for (int l = tid; l < j; l += NT) {
                const double ljl = A[tri(j) + l];
                Q1[l] -= ljl * x1;
                Q2[l] -= ljl * x2;
            }
            if (tid == 0) {
                U[j] = x1;
                Bv[j] = x2;
            }
        }
        __syncthreads();
        double ub = 0.0;
        for (int t = tid; t <= k; t += NT) ub += U[t] * Bv[t];
        // dl/dbeta = sum_{a > b} D_ab (u_a b_b + u_b b_a), D = dC/dbeta (zero on the diagonal)
        double gb = 0.0;
        const double s2b = P.sigma2 * P.inv_beta;
        for (int a = wave + 1; a <= k; a += NT / kWave) {
            const double xa = X[a], ya = Y[a], ua = U[a], ba = Bv[a], ca = kc_gcd(KC) ? CL[a] : 0.0;
            for (int b = lane; b < a; b += kWave) {
                const double r = cov_r<KC>(xa, ya, ca, X[b], Y[b], kc_gcd(KC) ? CL[b] : 0.0, P);
                gb += matern_dbeta_r<F>(r, s2b) * (ua * Bv[b] + U[b] * ba);
            }
        }
        ub = block_sum<NT / kWave>(ub, red);
        gb = block_sum<NT / kWave>(gb, red);
        o.g2 = ub;
        o.g0 = (0.5 * (rr * rr * c - 1.0) - P.tau2 * ub) / P.sigma2;
        o.g1 = gb;
    }
    const bool anybad = __syncthreads_or(mybad ? 1 : 0) != 0;
    o.bad = anybad || !isfinite(o.ell) || !isfinite(o.g0) || !isfinite(o.g1) || !isfinite(o.g2);
    return o;
}

}  // namespace vecchia

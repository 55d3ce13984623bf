/*
 * ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU evaluation of the Vecchia
 * approximated Gaussian-process log-likelihood and of its gradient with
 * respect to (sigma^2, beta, tau^2).  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the GPU library: it has its own covariance, Cholesky, solves and
 * summation.
 *
 * What it computes (Pan et al., "GPU-Accelerated Vecchia Approximations of
 * Gaussian Processes for Geospatial Data using Batched Matrix Computations"):
 *
 *   Eq. (7): log p(y) ~= sum_i log p(y_i | y_{J_i}), where J_i holds the
 *   min(i, m) nearest previously-ordered points of point i (0-based).  Each
 *   conditional is Gaussian with
 *       mean      mu_i = v^T Sigma_NN^{-1} y_N
 *       variance  c_i  = Sigma_ii - v^T Sigma_NN^{-1} v,
 *   formed as in Algorithm 1: covariance generation (sigma, Sigma, v), a
 *   Cholesky factor of Sigma_NN (POTRF), two triangular solves (TRSV) for
 *   v' = L^{-1} v and y' = L^{-1} y_N, the two dot products mu = v'.y' and
 *   v'.v', and the univariate Gaussian term, all summed.
 *
 *   Readings taken where the paper is silent or garbled:
 *   - The univariate term uses c_i as a VARIANCE (the algorithm subtracts a
 *     variance from a variance, so its "sigma" is a variance):
 *       l_i = -1/2 (log 2 pi + log c_i + (y_i - mu_i)^2 / c_i).
 *   - The first block is not a joint density over the first m points but the
 *     chain of short conditioning sets (k = i < m); by Eqs. (4)-(5) the two
 *     are equal.
 *   - Covariance, Eq. (2), with the distance scaled by beta alone (Table II's
 *     beta values give correlation 1/45 at the effective range under this
 *     scaling).  For nu = 1/2, 3/2, 5/2 the Bessel form reduces exactly to
 *       nu=0.5: s2 e^{-r};  nu=1.5: s2 (1+r) e^{-r};
 *       nu=2.5: s2 (1 + r + r^2/3) e^{-r},  r = ||s_a - s_b|| / beta.
 *   - A nugget tau^2 is added to the diagonal of Sigma_NN and to Sigma_ii
 *     (entries with equal indices), never to the cross vector v.
 *   - The gradient (not in the paper) is the derivative of each l_i:
 *       dl_i/dp = 1/2 (r^2 - 1/c) dc_p + r dmu_p,  r = (y_i - mu_i)/c_i,
 *       dc_p  = dSigma_ii/dp - 2 a^T dv/dp + a^T dSigma_NN/dp a,
 *       dmu_p = (dv/dp)^T s - a^T dSigma_NN/dp s,
 *     with a = Sigma_NN^{-1} v and s = Sigma_NN^{-1} y_N, each obtained by a
 *     back substitution with L^T.  dC/dsigma2 = C/sigma2 (nugget excluded),
 *     dSigma/dtau2 = I on Sigma_NN and 1 on Sigma_ii, dC/dbeta = -r/beta dC/dr.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp.  Per-conditional
 * results are stored per i and summed afterwards in ascending i with
 * Neumaier compensation, so totals do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORACLE_LOG_2PI 1.8378770664093454835606594728112

/* Error codes returned (negative) by the entry points. */
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* Matern covariance, Eq. (2), closed form for half-integer smoothness. */
static double matern(double d, double nu, double sigma2, double beta) {
    double r = d / beta;
    double e = exp(-r);
    if (nu == 0.5) return sigma2 * e;
    if (nu == 1.5) return sigma2 * (1.0 + r) * e;
    /* nu == 2.5 */
    return sigma2 * (1.0 + r + r * r / 3.0) * e;
}

/* d/dbeta of the covariance above: dC/dbeta = (dC/dr)(dr/dbeta), dr/dbeta = -r/beta. */
static double matern_dbeta(double d, double nu, double sigma2, double beta) {
    double r = d / beta;
    double e = exp(-r);
    double dcdr;
    if (nu == 0.5) dcdr = -sigma2 * e;
    else if (nu == 1.5) dcdr = sigma2 * (e - (1.0 + r) * e);
    else dcdr = sigma2 * ((1.0 + 2.0 * r / 3.0) * e - (1.0 + r + r * r / 3.0) * e);
    return dcdr * (-r / beta);
}

static double dist(const double *a, const double *b) {
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    return sqrt(dx * dx + dy * dy);
}

/*
 * Covariance model: family (0 Matern, Eq. (2); 1 power exponential, the
 * real-data model of Sec. V-C) and metric (0 Euclidean on (x, y); 1
 * great-circle on (longitude, latitude) in degrees, in kilometres).
 * smooth is nu for Matern and alpha for the power exponential.
 */
typedef struct {
    int family, metric;
    double smooth;
} cov_t;

#define ORACLE_EARTH_RADIUS_KM 6371.0
#define ORACLE_DEG2RAD 0.017453292519943295769236907684886

/*
 * Haversine value of two (lon, lat) points in degrees (Sec. V-C): with
 * phi the latitudes and lambda the longitudes in radians,
 *   hav(d / R) = hav(phi_a - phi_b) + cos phi_a cos phi_b hav(lambda_a - lambda_b),
 * hav(t) = sin^2(t / 2).  Differences are taken in degrees before the
 * conversion.  The result is clamped to [0, 1].
 */
static double haversine(const double *a, const double *b) {
    const double dlat = (a[1] - b[1]) * ORACLE_DEG2RAD;
    const double dlon = (a[0] - b[0]) * ORACLE_DEG2RAD;
    const double s1 = sin(0.5 * dlat), s2 = sin(0.5 * dlon);
    const double ca = cos(a[1] * ORACLE_DEG2RAD), cb = cos(b[1] * ORACLE_DEG2RAD);
    double h = s1 * s1 + (ca * cb) * (s2 * s2);
    if (h > 1.0) h = 1.0;
    return h;
}

/* great-circle distance in km: d = 2 R asin(sqrt(h)) */
static double gcd_km(const double *a, const double *b) {
    return 2.0 * ORACLE_EARTH_RADIUS_KM * asin(sqrt(haversine(a, b)));
}

static double cov_dist(const cov_t *cv, const double *a, const double *b) {
    return cv->metric == 1 ? gcd_km(a, b) : dist(a, b);
}

/* power exponential C(d) = sigma2 exp(-d^alpha / beta) and its beta-derivative C d^alpha / beta^2 */
static double powexp(double d, double alpha, double sigma2, double beta) {
    return sigma2 * exp(-pow(d, alpha) / beta);
}

static double powexp_dbeta(double d, double alpha, double sigma2, double beta) {
    const double u = pow(d, alpha) / beta;
    return sigma2 * exp(-u) * u / beta;
}

static double cov_fn(const cov_t *cv, double d, double sigma2, double beta) {
    return cv->family == 1 ? powexp(d, cv->smooth, sigma2, beta) : matern(d, cv->smooth, sigma2, beta);
}

static double cov_dbeta(const cov_t *cv, double d, double sigma2, double beta) {
    return cv->family == 1 ? powexp_dbeta(d, cv->smooth, sigma2, beta) : matern_dbeta(d, cv->smooth, sigma2, beta);
}

static int valid_cov(const cov_t *cv) {
    if (cv->metric != 0 && cv->metric != 1) return 0;
    if (cv->family == 0) return cv->smooth == 0.5 || cv->smooth == 1.5 || cv->smooth == 2.5;
    if (cv->family == 1) return cv->smooth > 0.0 && cv->smooth <= 2.0;
    return 0;
}

typedef struct {
    double *S, *L, *v, *yN, *vp, *yp, *a, *s, *Sp, *vpd;
} work_t;

static int work_alloc(work_t *w, int m) {
    size_t mm = (size_t)(m > 0 ? m : 1);
    w->S = (double *)malloc(mm * mm * sizeof(double));
    w->L = (double *)malloc(mm * mm * sizeof(double));
    w->Sp = (double *)malloc(mm * mm * sizeof(double));
    w->v = (double *)malloc(mm * sizeof(double));
    w->yN = (double *)malloc(mm * sizeof(double));
    w->vp = (double *)malloc(mm * sizeof(double));
    w->yp = (double *)malloc(mm * sizeof(double));
    w->a = (double *)malloc(mm * sizeof(double));
    w->s = (double *)malloc(mm * sizeof(double));
    w->vpd = (double *)malloc(mm * sizeof(double));
    return w->S && w->L && w->Sp && w->v && w->yN && w->vp && w->yp && w->a && w->s && w->vpd;
}

static void work_free(work_t *w) {
    free(w->S); free(w->L); free(w->Sp); free(w->v); free(w->yN);
    free(w->vp); free(w->yp); free(w->a); free(w->s); free(w->vpd);
}

/*
 * One conditional: l_i and (optionally) its gradient g[3] = dl_i/d(sigma2, beta, tau2).
 * Returns 0, or 1 when a pivot of the Cholesky factor or c_i is not positive
 * (or not finite).
 */
static int conditional(const double *locs, const double *z, const int32_t *nbr_row, int64_t i, int k,
                       const cov_t *cv, double sigma2, double beta, double tau2, work_t *w, double *ell,
                       double *g) {
    const double *si = locs + 2 * i;
    /* covariance generation (Algorithm 1, batched kernel step) */
    for (int a = 0; a < k; ++a) {
        const double *sa = locs + 2 * (int64_t)nbr_row[a];
        for (int b = 0; b < k; ++b) {
            const double *sb = locs + 2 * (int64_t)nbr_row[b];
            w->S[a * k + b] = cov_fn(cv, cov_dist(cv, sa, sb), sigma2, beta) + (a == b ? tau2 : 0.0);
        }
        w->v[a] = cov_fn(cv, cov_dist(cv, sa, si), sigma2, beta);
        w->yN[a] = z[nbr_row[a]];
    }
    double Sii = sigma2 + tau2;

    /* Cholesky-Banachiewicz, row by row (POTRF) */
    for (int r = 0; r < k; ++r) {
        for (int c = 0; c <= r; ++c) {
            double acc = w->S[r * k + c];
            for (int q = 0; q < c; ++q) acc -= w->L[r * k + q] * w->L[c * k + q];
            if (r == c) {
                if (!(acc > 0.0) || !isfinite(acc)) return 1;
                w->L[r * k + r] = sqrt(acc);
            } else {
                w->L[r * k + c] = acc / w->L[c * k + c];
            }
        }
    }
    /* forward substitutions (TRSV): v' = L^{-1} v, y' = L^{-1} y_N */
    for (int r = 0; r < k; ++r) {
        double av = w->v[r], ay = w->yN[r];
        for (int q = 0; q < r; ++q) {
            av -= w->L[r * k + q] * w->vp[q];
            ay -= w->L[r * k + q] * w->yp[q];
        }
        w->vp[r] = av / w->L[r * k + r];
        w->yp[r] = ay / w->L[r * k + r];
    }
    /* dot products: mu = v'.y', c = Sigma_ii - v'.v' */
    double mu = 0.0, vv = 0.0;
    for (int r = 0; r < k; ++r) {
        mu += w->vp[r] * w->yp[r];
        vv += w->vp[r] * w->vp[r];
    }
    double c = Sii - vv;
    if (!(c > 0.0) || !isfinite(c)) return 1;
    double res = z[i] - mu;
    *ell = -0.5 * (ORACLE_LOG_2PI + log(c) + res * res / c);
    if (!g) return 0;

    /* back substitutions with L^T: a = Sigma_NN^{-1} v, s = Sigma_NN^{-1} y_N */
    for (int r = k - 1; r >= 0; --r) {
        double aa = w->vp[r], ss = w->yp[r];
        for (int q = r + 1; q < k; ++q) {
            aa -= w->L[q * k + r] * w->a[q];
            ss -= w->L[q * k + r] * w->s[q];
        }
        w->a[r] = aa / w->L[r * k + r];
        w->s[r] = ss / w->L[r * k + r];
    }
    double rr = res / c;
    double half = 0.5 * (rr * rr - 1.0 / c);
    for (int p = 0; p < 3; ++p) {
        double Siip;
        /* derivative blocks: Sp = dSigma_NN/dp, vpd = dv/dp, Siip = dSigma_ii/dp */
        for (int a = 0; a < k; ++a) {
            const double *sa = locs + 2 * (int64_t)nbr_row[a];
            for (int b = 0; b < k; ++b) {
                const double *sb = locs + 2 * (int64_t)nbr_row[b];
                double d = cov_dist(cv, sa, sb);
                double val;
                if (p == 0) val = cov_fn(cv, d, sigma2, beta) / sigma2;
                else if (p == 1) val = cov_dbeta(cv, d, sigma2, beta);
                else val = (a == b) ? 1.0 : 0.0;
                w->Sp[a * k + b] = val;
            }
            double di = cov_dist(cv, sa, si);
            if (p == 0) w->vpd[a] = cov_fn(cv, di, sigma2, beta) / sigma2;
            else if (p == 1) w->vpd[a] = cov_dbeta(cv, di, sigma2, beta);
            else w->vpd[a] = 0.0;
        }
        Siip = (p == 1) ? 0.0 : 1.0;
        double aSa = 0.0, aSs = 0.0, av = 0.0, vs = 0.0;
        for (int a = 0; a < k; ++a) {
            double rowa = 0.0, rows = 0.0;
            for (int b = 0; b < k; ++b) {
                rowa += w->Sp[a * k + b] * w->a[b];
                rows += w->Sp[a * k + b] * w->s[b];
            }
            aSa += w->a[a] * rowa;
            aSs += w->a[a] * rows;
            av += w->a[a] * w->vpd[a];
            vs += w->vpd[a] * w->s[a];
        }
        double dc = Siip - 2.0 * av + aSa;
        double dmu = vs - aSs;
        g[p] = half * dc + rr * dmu;
    }
    return 0;
}

/* Neumaier-compensated sum of x[0..n) in ascending order. */
static double neumaier(const double *x, int64_t n, int64_t stride) {
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = x[i * stride];
        double t = s + v;
        if (fabs(s) >= fabs(v)) comp += (s - t) + v;
        else comp += (v - t) + s;
        s = t;
    }
    return s + comp;
}

static int valid_nu(double nu) { return nu == 0.5 || nu == 1.5 || nu == 2.5; }

/*
 * Per-conditional terms for the points listed in idx[0..nidx) (all points 0..n-1
 * when idx is NULL, then nidx must equal n).
 *   locs [n][2], z [n], nbr [n][m] int32 (row i: min(i,m) indices in [0,i), then -1)
 *   theta = {sigma2, beta, tau2}
 *   ell [nidx] receives l_i; grad [nidx][3] (may be NULL) receives dl_i/d(sigma2,beta,tau2).
 * Returns 0; a negative error code for bad arguments; or (i+1) for the smallest
 * listed point i whose conditional failed (its outputs are NaN).
 */
int64_t oracle_terms_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                         int32_t family, int32_t metric, double smooth, const double *theta, const int64_t *idx,
                         int64_t nidx, double *ell, double *grad, int32_t nthreads) {
    const cov_t cvs = {family, metric, smooth};
    const cov_t *cv = &cvs;
    if (!locs || !z || !theta || !ell || n < 0 || m < 0 || (m > 0 && !nbr) || nidx < 0) return ORACLE_EINVAL;
    if (!idx && nidx != n) return ORACLE_EINVAL;
    if (!valid_cov(cv) || !(theta[0] > 0) || !(theta[1] > 0) || !(theta[2] >= 0)) return ORACLE_EINVAL;
    for (int64_t t = 0; t < nidx; ++t) {
        int64_t i = idx ? idx[t] : t;
        if (i < 0 || i >= n) return ORACLE_EINVAL;
        int64_t k = i < m ? i : m;
        for (int64_t q = 0; q < k; ++q) {
            int32_t j = nbr[i * (int64_t)m + q];
            if (j < 0 || j >= i) return ORACLE_EINVAL;
        }
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t first_fail = INT64_MAX;
    int nomem = 0;
#pragma omp parallel
    {
        work_t w;
        int ok = work_alloc(&w, m);
        if (!ok) {
#pragma omp atomic write
            nomem = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nidx; ++t) {
            if (!ok) continue;
            int64_t i = idx ? idx[t] : t;
            int k = (int)(i < m ? i : m);
            double g[3] = {0, 0, 0};
            double e = 0.0;
            int bad = conditional(locs, z, nbr + i * (int64_t)m, i, k, cv, theta[0], theta[1], theta[2], &w, &e,
                                  grad ? g : NULL);
            if (bad) {
                e = NAN;
                g[0] = g[1] = g[2] = NAN;
#pragma omp critical
                {
                    if (i < first_fail) first_fail = i;
                }
            }
            ell[t] = e;
            if (grad) {
                grad[3 * t + 0] = g[0];
                grad[3 * t + 1] = g[1];
                grad[3 * t + 2] = g[2];
            }
        }
        work_free(&w);
    }
    if (nomem) return ORACLE_ENOMEM;
    return first_fail == INT64_MAX ? 0 : first_fail + 1;
}

/* Matern covariance with Euclidean distance (Eq. (2)): oracle_terms_cov with family 0, metric 0. */
int64_t oracle_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                     const double *theta, const int64_t *idx, int64_t nidx, double *ell, double *grad,
                     int32_t nthreads) {
    if (!valid_nu(nu)) return ORACLE_EINVAL;
    return oracle_terms_cov(locs, z, nbr, n, m, 0, 0, nu, theta, idx, nidx, ell, grad, nthreads);
}

/*
 * Whole log-likelihood: out[0] = sum_i l_i; grad[0..3) = sum_i dl_i/dp when grad != NULL.
 * Sums are Neumaier-compensated in ascending i.  Return value as oracle_terms.
 */
int64_t oracle_loglik_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                          int32_t family, int32_t metric, double smooth, const double *theta, double *out,
                          double *grad, int32_t nthreads) {
    if (!out || n < 0) return ORACLE_EINVAL;
    double *ell = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *g = grad ? (double *)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double)) : NULL;
    if (!ell || (grad && !g)) {
        free(ell); free(g);
        return ORACLE_ENOMEM;
    }
    int64_t rc = oracle_terms_cov(locs, z, nbr, n, m, family, metric, smooth, theta, NULL, n, ell, g, nthreads);
    if (rc >= 0) {
        out[0] = neumaier(ell, n, 1);
        if (grad)
            for (int p = 0; p < 3; ++p) grad[p] = neumaier(g + p, n, 3);
    }
    free(ell);
    free(g);
    return rc;
}

int64_t oracle_loglik(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                      const double *theta, double *out, double *grad, int32_t nthreads) {
    if (!valid_nu(nu)) return ORACLE_EINVAL;
    return oracle_loglik_cov(locs, z, nbr, n, m, 0, 0, nu, theta, out, grad, nthreads);
}

/* Covariance values and beta-derivatives of any model at distances d, for pins. */
int64_t oracle_cov_values(const double *d, int64_t n, int32_t family, int32_t metric, double smooth, double sigma2,
                          double beta, double *out, double *dbeta) {
    const cov_t cv = {family, metric, smooth};
    if (!valid_cov(&cv) || n < 0 || (n > 0 && (!d || !out))) return ORACLE_EINVAL;
    for (int64_t t = 0; t < n; ++t) {
        out[t] = cov_fn(&cv, d[t], sigma2, beta);
        if (dbeta) dbeta[t] = cov_dbeta(&cv, d[t], sigma2, beta);
    }
    return 0;
}

/* Pairwise distances a[t] to b[t] (n pairs of points) under a metric, for pins. */
int64_t oracle_distances(const double *a, const double *b, int64_t n, int32_t metric, double *out) {
    if (n < 0 || (metric != 0 && metric != 1) || (n > 0 && (!a || !b || !out))) return ORACLE_EINVAL;
    const cov_t cv = {0, metric, 0.5};
    for (int64_t t = 0; t < n; ++t) out[t] = cov_dist(&cv, a + 2 * t, b + 2 * t);
    return 0;
}

/* The covariance entries this oracle uses, exported so tests can pin them against Eq. (2). */
void oracle_matern(const double *d, int64_t n, double nu, double sigma2, double beta, double *out,
                   double *dbeta) {
    for (int64_t t = 0; t < n; ++t) {
        out[t] = matern(d[t], nu, sigma2, beta);
        if (dbeta) dbeta[t] = matern_dbeta(d[t], nu, sigma2, beta);
    }
}

/* Neumaier sum exported for tests. */
double oracle_sum(const double *x, int64_t n) { return neumaier(x, n, 1); }

/*
 * Ranking key of a candidate j for query point q: the squared Euclidean
 * distance dx*dx + dy*dy (each product rounded, no contraction) for metric 0,
 * the haversine value (monotone in the great-circle distance) for metric 1.
 */
static double knn_key(const double *q, const double *p, int metric) {
    if (metric == 1) return haversine(q, p);
    const double dx = q[0] - p[0];
    const double dy = q[1] - p[1];
    return dx * dx + dy * dy;
}

/*
 * The k = min(lim, m) candidates j in [0, lim) of ref nearest to q, ordered by
 * (key, index) ascending, into out[0..m) (-1 past k).  Brute force: every j is
 * compared with the current k-th best and inserted into a sorted list when it
 * beats it; j ascends, so among equal keys the earlier index wins.
 * bd and bj hold m entries.
 */
static void knn_one(const double *q, const double *ref, int64_t lim, int32_t m, int metric, double *bd,
                    int32_t *bj, int32_t *out) {
    const int32_t k = (int32_t)(lim < m ? lim : m);
    int32_t cnt = 0;
    for (int64_t j = 0; j < lim && k > 0; ++j) {
        const double d = knn_key(q, ref + 2 * j, metric);
        if (cnt == k && !(d < bd[k - 1])) continue;
        int32_t p = (cnt == k) ? k - 1 : cnt;
        while (p > 0 && d < bd[p - 1]) {
            bd[p] = bd[p - 1];
            bj[p] = bj[p - 1];
            --p;
        }
        bd[p] = d;
        bj[p] = (int32_t)j;
        if (cnt < k) ++cnt;
    }
    for (int32_t t = 0; t < m; ++t) out[t] = (t < cnt) ? bj[t] : -1;
}

/*
 * Conditioning sets by their definition (Sec. IV-B and the neighbour loop of
 * Algorithm 1; ties and the short sets as read here): for each requested
 * 0-based row i, the min(i, m) indices j < i closest to point i under the
 * metric (0 Euclidean, 1 great-circle on degrees), ordered by (key, index)
 * ascending; slots past min(i, m) are -1.  out is [nrows][m].  Returns 0, or
 * ORACLE_EINVAL / ORACLE_ENOMEM.
 */
int64_t oracle_knn_rows_metric(const double *locs, int64_t n, int32_t m, int32_t metric, const int64_t *rows,
                               int64_t nrows, int32_t *out, int32_t nthreads) {
    if (n < 0 || m < 0 || nrows < 0 || (nrows > 0 && (!rows || !out)) || (n > 0 && !locs)) return ORACLE_EINVAL;
    if (metric != 0 && metric != 1) return ORACLE_EINVAL;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n) return ORACLE_EINVAL;
    if (m == 0 || nrows == 0) return 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int failed = 0;
#pragma omp parallel
    {
        double *bd = (double *)malloc((size_t)m * sizeof(double));
        int32_t *bj = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        if (!bd || !bj) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!bd || !bj) continue;
            const int64_t i = rows[r];
            knn_one(locs + 2 * i, locs, i, m, metric, bd, bj, out + r * (int64_t)m);
        }
        free(bd);
        free(bj);
    }
    return failed ? ORACLE_ENOMEM : 0;
}

int64_t oracle_knn_rows(const double *locs, int64_t n, int32_t m, const int64_t *rows, int64_t nrows,
                        int32_t *out, int32_t nthreads) {
    return oracle_knn_rows_metric(locs, n, m, 0, rows, nrows, out, nthreads);
}

/*
 * Neighbour sets of prediction points: for each query q, the min(n_ref, m)
 * reference points nearest to it (all of them are candidates), ordered and
 * tie-broken as above.  out is [nq][m].  Returns 0, ORACLE_EINVAL or
 * ORACLE_ENOMEM.
 */
int64_t oracle_knn_query(const double *ref, int64_t n_ref, const double *q, int64_t nq, int32_t m, int32_t metric,
                         int32_t *out, int32_t nthreads) {
    if (n_ref < 0 || nq < 0 || m < 0 || (n_ref > 0 && !ref) || (nq > 0 && (!q || !out))) return ORACLE_EINVAL;
    if (metric != 0 && metric != 1) return ORACLE_EINVAL;
    if (m == 0 || nq == 0) return 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int failed = 0;
#pragma omp parallel
    {
        double *bd = (double *)malloc((size_t)m * sizeof(double));
        int32_t *bj = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        if (!bd || !bj) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < nq; ++t) {
            if (!bd || !bj) continue;
            knn_one(q + 2 * t, ref, n_ref, m, metric, bd, bj, out + t * (int64_t)m);
        }
        free(bd);
        free(bj);
    }
    return failed ? ORACLE_ENOMEM : 0;
}

/*
 * Vecchia kriging (Sec. V-C): the conditional Gaussian of the observation at
 * each prediction point given the observations at its neighbour set J
 * (nbr row t, min(n_ref, m) valid indices into the reference points):
 *   mean = v^T Sigma_JJ^{-1} y_J,   var = sigma2 + tau2 - v^T Sigma_JJ^{-1} v,
 * with Sigma_JJ the covariance of the neighbours (nugget on its diagonal) and
 * v the covariance between the neighbours and the point (no nugget).  The
 * solve is a Cholesky factorisation and two triangular substitutions.  var is
 * the variance of a new observation; the latent field's is var - tau2.
 * Returns 0, ORACLE_EINVAL, ORACLE_ENOMEM, or t + 1 for the first point whose
 * system is not positive definite or whose var is not positive (a point that
 * coincides with a neighbour when tau2 = 0); its outputs are NaN.
 */
int64_t oracle_predict(const double *ref, const double *zref, int64_t n_ref, const double *q, int64_t nq,
                       const int32_t *nbr, int32_t m, int32_t family, int32_t metric, double smooth,
                       const double *theta, double *mean, double *var, int32_t nthreads) {
    const cov_t cvs = {family, metric, smooth};
    const cov_t *cv = &cvs;
    if (n_ref < 0 || nq < 0 || m < 0 || !theta || (nq > 0 && (!q || !mean || !var))) return ORACLE_EINVAL;
    if (n_ref > 0 && (!ref || !zref)) return ORACLE_EINVAL;
    if (!valid_cov(cv) || !(theta[0] > 0) || !(theta[1] > 0) || !(theta[2] >= 0)) return ORACLE_EINVAL;
    const int32_t k = (int32_t)(n_ref < m ? n_ref : m);
    if (k > 0 && !nbr) return ORACLE_EINVAL;
    for (int64_t t = 0; t < nq; ++t)
        for (int32_t a = 0; a < k; ++a) {
            const int32_t j = nbr[t * (int64_t)m + a];
            if (j < 0 || j >= n_ref) return ORACLE_EINVAL;
        }
    const double sigma2 = theta[0], beta = theta[1], tau2 = theta[2];
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int64_t first_fail = INT64_MAX;
    int nomem = 0;
#pragma omp parallel
    {
        const size_t kk = (size_t)(k > 0 ? k : 1);
        double *L = (double *)malloc(kk * kk * sizeof(double));
        double *v = (double *)malloc(kk * sizeof(double));
        double *y = (double *)malloc(kk * sizeof(double));
        double *a = (double *)malloc(kk * sizeof(double));
        if (!L || !v || !y || !a) {
#pragma omp atomic write
            nomem = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nq; ++t) {
            if (!L || !v || !y || !a) continue;
            const int32_t *J = nbr + t * (int64_t)m;
            const double *sq = q + 2 * t;
            int bad = 0;
            /* Sigma_JJ (lower triangle, row-major), v and y_J */
            for (int32_t r = 0; r < k; ++r) {
                const double *sr = ref + 2 * (int64_t)J[r];
                for (int32_t c = 0; c <= r; ++c)
                    L[r * k + c] = cov_fn(cv, cov_dist(cv, sr, ref + 2 * (int64_t)J[c]), sigma2, beta) +
                                   (r == c ? tau2 : 0.0);
                v[r] = cov_fn(cv, cov_dist(cv, sr, sq), sigma2, beta);
                y[r] = zref[J[r]];
            }
            /* Cholesky in place */
            for (int32_t r = 0; r < k && !bad; ++r) {
                for (int32_t c = 0; c <= r; ++c) {
                    double acc = L[r * k + c];
                    for (int32_t p = 0; p < c; ++p) acc -= L[r * k + p] * L[c * k + p];
                    if (r == c) {
                        if (!(acc > 0.0) || !isfinite(acc)) {
                            bad = 1;
                            break;
                        }
                        L[r * k + r] = sqrt(acc);
                    } else {
                        L[r * k + c] = acc / L[c * k + c];
                    }
                }
            }
            double mu = NAN, vr = NAN;
            if (!bad) {
                /* a = Sigma_JJ^{-1} v: forward then back substitution */
                for (int32_t r = 0; r < k; ++r) {
                    double acc = v[r];
                    for (int32_t p = 0; p < r; ++p) acc -= L[r * k + p] * a[p];
                    a[r] = acc / L[r * k + r];
                }
                for (int32_t r = k - 1; r >= 0; --r) {
                    double acc = a[r];
                    for (int32_t p = r + 1; p < k; ++p) acc -= L[p * k + r] * a[p];
                    a[r] = acc / L[r * k + r];
                }
                double my = 0.0, mv = 0.0;
                for (int32_t r = 0; r < k; ++r) {
                    my += a[r] * y[r];
                    mv += a[r] * v[r];
                }
                mu = my;
                vr = sigma2 + tau2 - mv;
                if (!(vr > 0.0) || !isfinite(vr) || !isfinite(mu)) bad = 1;
            }
            if (bad) {
                mu = vr = NAN;
#pragma omp critical
                {
                    if (t < first_fail) first_fail = t;
                }
            }
            mean[t] = mu;
            var[t] = vr;
        }
        free(L);
        free(v);
        free(y);
        free(a);
    }
    if (nomem) return ORACLE_ENOMEM;
    return first_fail == INT64_MAX ? 0 : first_fail + 1;
}

/*
 * Morton (Z-order) ordering of the points (the ordering option of Sec. IV-A),
 * as read here: each coordinate is mapped to a 16-bit cell index
 * q = floor((x - min) / (max - min) * 65536) clamped to [0, 65535] over the
 * bounding box (a zero extent maps to 0), the code interleaves the bits with
 * x in the even and y in the odd positions, and perm lists the point indices
 * by ascending code, ties by ascending index.  Returns 0 or ORACLE_EINVAL /
 * ORACLE_ENOMEM.
 */
typedef struct {
    uint32_t code;
    int64_t idx;
} morton_key_t;

static int morton_cmp(const void *a, const void *b) {
    const morton_key_t *x = (const morton_key_t *)a, *y = (const morton_key_t *)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static uint32_t morton_cell(double v, double lo, double hi) {
    const double w = hi - lo;
    if (!(w > 0)) return 0;
    double q = floor((v - lo) / w * 65536.0);
    if (q < 0) q = 0;
    if (q > 65535) q = 65535;
    return (uint32_t)q;
}

int64_t oracle_morton_order(const double *locs, int64_t n, int64_t *perm) {
    if (n < 0 || (n > 0 && (!locs || !perm))) return ORACLE_EINVAL;
    if (n == 0) return 0;
    double xmin = locs[0], xmax = locs[0], ymin = locs[1], ymax = locs[1];
    for (int64_t i = 1; i < n; ++i) {
        if (locs[2 * i] < xmin) xmin = locs[2 * i];
        if (locs[2 * i] > xmax) xmax = locs[2 * i];
        if (locs[2 * i + 1] < ymin) ymin = locs[2 * i + 1];
        if (locs[2 * i + 1] > ymax) ymax = locs[2 * i + 1];
    }
    morton_key_t *keys = (morton_key_t *)malloc((size_t)n * sizeof(morton_key_t));
    if (!keys) return ORACLE_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t qx = morton_cell(locs[2 * i], xmin, xmax);
        const uint32_t qy = morton_cell(locs[2 * i + 1], ymin, ymax);
        uint32_t code = 0;
        for (int b = 0; b < 16; ++b) {
            code |= ((qx >> b) & 1u) << (2 * b);
            code |= ((qy >> b) & 1u) << (2 * b + 1);
        }
        keys[i].code = code;
        keys[i].idx = i;
    }
    qsort(keys, (size_t)n, sizeof(morton_key_t), morton_cmp);
    for (int64_t i = 0; i < n; ++i) perm[i] = keys[i].idx;
    free(keys);
    return 0;
}

/*
 * Approximate maxmin ordering (the ordering Sec. IV-A names as accurate but
 * too costly at scale), as defined for this library: points are elected in
 * rounds r = 0, 1, ... over grids of G = 2^l(r) x 2^l(r) square cells,
 * l(r) = min(r, Lmax), on the square box [x0, x0 + w] x [y0, y0 + w] with
 * (x0, y0) the lower-left of the bounding box and w its larger side (1 when
 * zero).  Lmax is the least L >= 0 with 4^L >= n, plus 1, at most 15.  A point's
 * cell is c = min(floor((x - x0) / w * G), G - 1) per axis; in each round
 * every cell elects, among its unselected points, the one with the least
 * squared distance to the cell centre (x0 + (c + 1/2) w / G, each product
 * and sum rounded, no contraction), ties by index.  The points elected in a
 * round follow all earlier rounds, in ascending order of
 * key(i) = mix64(seed XOR i) (a bijection on 64-bit words, the splitmix64
 * finaliser).  After Lmax + 33 rounds any points left follow in the same
 * key order.  perm receives the point indices in order.  Returns 0,
 * ORACLE_EINVAL or ORACLE_ENOMEM.
 */
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t key;
    int64_t idx;
} hkey_t;

static int hkey_cmp(const void *a, const void *b) {
    const hkey_t *x = (const hkey_t *)a, *y = (const hkey_t *)b;
    return (x->key > y->key) - (x->key < y->key);
}

static int64_t maxmin_cell(double v, double v0, double w, int64_t G) {
    double f = floor((v - v0) / w * (double)G);
    if (!(f >= 0)) f = 0; /* negative or NaN */
    if (f > (double)(G - 1)) f = (double)(G - 1);
    return (int64_t)f;
}

int64_t oracle_maxmin_order(const double *locs, int64_t n, uint64_t seed, int64_t *perm) {
    if (n < 0 || (n > 0 && (!locs || !perm))) return ORACLE_EINVAL;
    if (n == 0) return 0;
    double x0 = locs[0], x1 = locs[0], y0 = locs[1], y1 = locs[1];
    for (int64_t i = 1; i < n; ++i) {
        if (locs[2 * i] < x0) x0 = locs[2 * i];
        if (locs[2 * i] > x1) x1 = locs[2 * i];
        if (locs[2 * i + 1] < y0) y0 = locs[2 * i + 1];
        if (locs[2 * i + 1] > y1) y1 = locs[2 * i + 1];
    }
    double w = (x1 - x0 > y1 - y0) ? x1 - x0 : y1 - y0;
    if (!(w > 0)) w = 1.0;
    int lmax = 0;
    while (lmax < 14 && ((int64_t)1 << (2 * lmax)) < n) ++lmax;
    lmax += 1;
    const int64_t gmax = (int64_t)1 << lmax;
    char *sel = (char *)calloc((size_t)n, 1);
    double *bd = (double *)malloc((size_t)(gmax * gmax) * sizeof(double));
    int64_t *bi = (int64_t *)malloc((size_t)(gmax * gmax) * sizeof(int64_t));
    hkey_t *grp = (hkey_t *)malloc((size_t)n * sizeof(hkey_t));
    if (!sel || !bd || !bi || !grp) {
        free(sel); free(bd); free(bi); free(grp);
        return ORACLE_ENOMEM;
    }
    int64_t done = 0;
    for (int r = 0; done < n; ++r) {
        int64_t cnt = 0;
        if (r < lmax + 33) {
            const int l = r < lmax ? r : lmax;
            const int64_t G = (int64_t)1 << l;
            for (int64_t c = 0; c < G * G; ++c) bi[c] = -1;
            for (int64_t i = 0; i < n; ++i) {
                if (sel[i]) continue;
                const int64_t cx = maxmin_cell(locs[2 * i], x0, w, G);
                const int64_t cy = maxmin_cell(locs[2 * i + 1], y0, w, G);
                const double dx = locs[2 * i] - (x0 + ((double)cx + 0.5) * w / (double)G);
                const double dy = locs[2 * i + 1] - (y0 + ((double)cy + 0.5) * w / (double)G);
                const double d = dx * dx + dy * dy;
                const int64_t c = cy * G + cx;
                /* i ascends: among equal distances the earlier index stays */
                if (bi[c] < 0 || d < bd[c]) {
                    bd[c] = d;
                    bi[c] = i;
                }
            }
            for (int64_t c = 0; c < G * G; ++c)
                if (bi[c] >= 0) {
                    grp[cnt].key = mix64(seed ^ (uint64_t)bi[c]);
                    grp[cnt].idx = bi[c];
                    ++cnt;
                }
        } else {
            for (int64_t i = 0; i < n; ++i)
                if (!sel[i]) {
                    grp[cnt].key = mix64(seed ^ (uint64_t)i);
                    grp[cnt].idx = i;
                    ++cnt;
                }
        }
        qsort(grp, (size_t)cnt, sizeof(hkey_t), hkey_cmp);
        for (int64_t t = 0; t < cnt; ++t) {
            sel[grp[t].idx] = 1;
            perm[done + t] = grp[t].idx;
        }
        done += cnt;
    }
    free(sel); free(bd); free(bi); free(grp);
    return 0;
}

/*
 * Exact log-likelihood, Eq. (1): l = -1/2 (n log 2 pi + log det Sigma +
 * z^T Sigma^{-1} z) with Sigma the full covariance of all n points (the
 * covariance above, nugget on the diagonal), by a dense Cholesky-Banachiewicz
 * factorisation and one forward substitution; z == NULL means y = 0, the
 * reference term of the KL divergence of Eq. (9).  O(n^3 / 3) work.
 * Returns 0, ORACLE_EINVAL, ORACLE_ENOMEM or j + 1 for a non-positive pivot
 * in column j.
 */
int64_t oracle_exact_loglik(const double *locs, const double *z, int64_t n, double nu, const double *theta,
                            double *out) {
    if (!locs || !theta || !out || n < 1 || !valid_nu(nu)) return ORACLE_EINVAL;
    const double sigma2 = theta[0], beta = theta[1], tau2 = theta[2];
    if (!(sigma2 > 0) || !(beta > 0) || !(tau2 >= 0)) return ORACLE_EINVAL;
    double *L = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *logs = (double *)malloc((size_t)n * sizeof(double));
    if (!L || !w || !logs) {
        free(L); free(w); free(logs);
        return ORACLE_ENOMEM;
    }
    /* lower triangle, row-major */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j)
            L[i * n + j] = matern(dist(locs + 2 * i, locs + 2 * j), nu, sigma2, beta) + (i == j ? tau2 : 0.0);
    int64_t rc = 0;
    for (int64_t j = 0; j < n && rc == 0; ++j) {
        double d = L[j * n + j];
        for (int64_t p = 0; p < j; ++p) d -= L[j * n + p] * L[j * n + p];
        if (!(d > 0)) {
            rc = j + 1;
            break;
        }
        const double ljj = sqrt(d);
        L[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = L[i * n + j];
            for (int64_t p = 0; p < j; ++p) s -= L[i * n + p] * L[j * n + p];
            L[i * n + j] = s / ljj;
        }
    }
    if (rc == 0) {
        for (int64_t i = 0; i < n; ++i) logs[i] = 2.0 * log(L[i * n + i]);
        const double logdet = neumaier(logs, n, 1);
        double quad = 0.0;
        if (z) {
            for (int64_t i = 0; i < n; ++i) {
                double s = z[i];
                for (int64_t p = 0; p < i; ++p) s -= L[i * n + p] * w[p];
                w[i] = s / L[i * n + i];
                logs[i] = w[i] * w[i];
            }
            quad = neumaier(logs, n, 1);
        }
        out[0] = -0.5 * ((double)n * ORACLE_LOG_2PI + logdet + quad);
    }
    free(L);
    free(w);
    free(logs);
    return rc;
}

/*
 * Random ordering (Sec. IV-A orders the points at random before building the
 * conditioning sets), as defined for this library: perm lists the point
 * indices 0..n-1 by ascending key(i) = mix64(seed XOR i).  mix64 is a
 * bijection on 64-bit words, so the keys are distinct and the order is a
 * permutation.  Returns 0, ORACLE_EINVAL or ORACLE_ENOMEM.
 */
int64_t oracle_random_order(int64_t n, uint64_t seed, int64_t *perm) {
    if (n < 0 || (n > 0 && !perm)) return ORACLE_EINVAL;
    if (n == 0) return 0;
    hkey_t *k = (hkey_t *)malloc(sizeof(hkey_t) * (size_t)n);
    if (!k) return ORACLE_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        k[i].key = mix64(seed ^ (uint64_t)i);
        k[i].idx = i;
    }
    qsort(k, (size_t)n, sizeof(hkey_t), hkey_cmp);
    for (int64_t i = 0; i < n; ++i) perm[i] = k[i].idx;
    free(k);
    return 0;
}

/* The splitmix64 finaliser itself, for checking it against published outputs. */
uint64_t oracle_mix64(uint64_t z) { return mix64(z); }

/*
 * vecchia.h — C ABI of the MI355X (gfx950) library that evaluates the Vecchia
 * approximated Gaussian-process log-likelihood and its gradient in FP64.
 *
 * The method (Pan et al., "GPU-Accelerated Vecchia Approximations of Gaussian
 * Processes for Geospatial Data using Batched Matrix Computations"):
 *
 *   Eq. (7)       log p(y) ~= sum_{i=0}^{n-1} log p(y_i | y_{J_i})
 *   Algorithm 1   per point: covariance generation (sigma_i, Sigma_i, v_i),
 *                 Cholesky of Sigma_i, triangular solves for v_i and y_{J_i},
 *                 dot products giving the conditional mean and variance,
 *                 univariate Gaussian term, sum over points.
 *   Eq. (2)       Matern covariance with r = ||s_a - s_b|| / beta, here for
 *                 smoothness nu in {0.5, 1.5, 2.5} in closed form:
 *                 sigma2 e^-r, sigma2 (1+r) e^-r, sigma2 (1+r+r^2/3) e^-r.
 *
 * Additions that the paper does not have:
 *   - a nugget tau2 on the diagonal of Sigma_NN and on Sigma_ii (not on v);
 *   - the gradient dl/d(sigma2, beta, tau2) at fixed nu;
 *   - batched evaluation of many parameter vectors and many fields.
 *
 * Conventions shared by every entry point
 *   - Array pointers marked [dev] are DEVICE pointers owned by the caller.  The
 *     library never frees them and keeps no reference after the call.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     is asynchronous.  The likelihood entry points never synchronise the
 *     device and never allocate device memory; the autotuner, the orderings
 *     and the estimation drivers document their synchronisation.
 *   - locs  [dev] double [n][2]  row-major coordinates, already in the ordering.
 *   - z     [dev] double [n]     observations (zero mean).
 *   - nbr   [dev] int32  [n][m]  row i lists its min(i, m) conditioning points,
 *                                each in [0, i), in any order; other slots are
 *                                ignored (by convention -1).  Row 0 is empty.
 *   - theta [dev] double [3]     (sigma2 > 0, beta > 0, tau2 >= 0), all finite.
 *   - nu is 0.5, 1.5 or 2.5;  0 <= m <= VECCHIA_MAX_M.
 *   - status [dev] int64 per evaluation, written by the device:
 *         0                      success;
 *         VECCHIA_STATUS_THETA   theta invalid (outputs NaN);
 *         i + 1 (> 0)            point i is the smallest failing point: its
 *                                block is not numerically positive definite
 *                                (a pivot or the conditional variance is not
 *                                positive and finite), an input is not finite,
 *                                or a neighbour index is outside [0, i).
 *                                The outputs of that evaluation are NaN.
 *     The device checks every neighbour index before using it, so bad input
 *     never causes an out-of-bounds access.
 *   - Return value (synchronous): VECCHIA_OK or an error code below, for
 *     argument or launch problems detected on the host.
 *   - Results are deterministic: the same inputs give bitwise equal outputs,
 *     whatever the launch order of the work.
 */
#ifndef VECCHIA_H
#define VECCHIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VECCHIA_MAX_M 160
#define VECCHIA_MAX_FIELDS 4096
#define VECCHIA_STATUS_THETA (-1)

enum vecchia_error {
    VECCHIA_OK = 0,
    VECCHIA_EINVAL = 1,        /* null pointer, n < 0, m < 0, bad nu, bad sizes */
    VECCHIA_EUNSUPPORTED = 2,  /* m > VECCHIA_MAX_M, too many fields, unknown option */
    VECCHIA_EHIP = 3,          /* a HIP runtime call or kernel launch failed */
    VECCHIA_EWORKSPACE = 4     /* workspace missing or smaller than required */
};

/* Human-readable text for a return code. */
const char *vecchia_strerror(int code);

/* Library version string. */
const char *vecchia_version(void);

/*
 * Workspace (bytes) that vecchia_loglik / vecchia_loglik_grad need for n points
 * and m neighbours.  The caller allocates it on the device (256-byte aligned)
 * and may reuse it across calls on the same stream.
 */
size_t vecchia_workspace_size(int64_t n, int32_t m);

/*
 * Log-likelihood, Eq. (7): out[0] = sum_i l_i with
 *   l_i = -1/2 (log 2 pi + log c_i + (z_i - mu_i)^2 / c_i),
 * mu_i and c_i the conditional mean and variance of point i given its set.
 *   out      [dev] double[1]
 *   status   [dev] int64[1]
 *   ws       [dev] workspace of at least vecchia_workspace_size(n, m) bytes
 * n = 0 gives out = 0.  Returns VECCHIA_OK or an error code.
 */
int vecchia_loglik(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                   const double *theta, double *out, int64_t *status, void *ws, size_t ws_bytes, void *stream);

/*
 * Log-likelihood and its gradient with respect to (sigma2, beta, tau2) at fixed
 * nu (the derivative of every l_i, summed; not in the paper).
 *   out   [dev] double[1];  grad [dev] double[3] = (dl/dsigma2, dl/dbeta, dl/dtau2)
 * Factors are recomputed inside the kernel; nothing of size n*m^2 is stored.
 */
int vecchia_loglik_grad(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                        const double *theta, double *out, double *grad, int64_t *status, void *ws,
                        size_t ws_bytes, void *stream);

/*
 * vecchia_loglik_grad without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments and results as vecchia_loglik_grad
 * minus ws / ws_bytes, bitwise equal to it with the same kernel variant.  The
 * per-point rows live in a static device array of the library (about 10.6 MB
 * on every GPU it runs on, held until the process ends), which every call on
 * that GPU shares: calls that overlap on one GPU race and give wrong results.
 * Points are evaluated in slices of 2^18 through that array.
 *   n at most VECCHIA_NOALLOC_MAX_N; larger n returns VECCHIA_EUNSUPPORTED.
 * Returns VECCHIA_OK, VECCHIA_EINVAL, VECCHIA_EUNSUPPORTED or VECCHIA_EHIP.
 */
#define VECCHIA_NOALLOC_MAX_N (1 << 26)
int vecchia_loglik_grad_noalloc(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                                double nu, const double *theta, double *out, double *grad, int64_t *status,
                                void *stream);

/*
 * Per-point terms, for checking individual conditionals.
 *   idx    [dev] int64[nidx] points to evaluate, each in [0, n); NULL = all
 *          points (then nidx must equal n)
 *   terms  [dev] double[nidx]      l_i for idx[t]
 *   gterms [dev] double[nidx][3]   dl_i/d(sigma2, beta, tau2), or NULL
 *   status [dev] int64[1]          0; VECCHIA_STATUS_THETA; or t + 1 for the
 *                                  smallest position t whose point failed (as
 *                                  above) or whose index idx[t] is outside [0, n)
 * Failed positions hold NaN.
 */
int vecchia_loglik_terms(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                         double nu, const double *theta, const int64_t *idx, int64_t nidx, double *terms,
                         double *gterms, int64_t *status, void *stream);

/*
 * Covariance models beyond the Matern-with-Euclidean-distance calls above.
 *   family VECCHIA_MATERN   Eq. (2); smoothness = nu in {0.5, 1.5, 2.5}
 *          VECCHIA_POWEXP   the power exponential of the real-data study
 *                           (Sec. V-C), C(d) = sigma2 exp(-d^alpha / beta);
 *                           smoothness = alpha in (0, 2]
 *   metric VECCHIA_EUCLIDEAN     locs are (x, y)
 *          VECCHIA_GREAT_CIRCLE  locs are (longitude, latitude) in degrees and
 *                                d is the haversine great-circle distance in
 *                                km on a sphere of radius 6371 km (Sec. V-C)
 * The nugget tau2 is added to equal-index entries as for the Matern calls.
 */
enum vecchia_family { VECCHIA_MATERN = 0, VECCHIA_POWEXP = 1 };
enum vecchia_metric { VECCHIA_EUCLIDEAN = 0, VECCHIA_GREAT_CIRCLE = 1 };

typedef struct vecchia_cov {
    int32_t family;
    int32_t metric;
    double smoothness;
} vecchia_cov;

/*
 * vecchia_loglik / vecchia_loglik_grad under any covariance model: grad ==
 * NULL evaluates the value only, else also dl/d(sigma2, beta, tau2) at fixed
 * smoothness.  Arguments, workspace, status and return codes as above; an
 * invalid model is VECCHIA_EINVAL.
 */
int vecchia_loglik_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                       const vecchia_cov *cov, const double *theta, double *out, double *grad, int64_t *status,
                       void *ws, size_t ws_bytes, void *stream);

/* vecchia_loglik_terms under any covariance model. */
int vecchia_loglik_terms_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                             const vecchia_cov *cov, const double *theta, const int64_t *idx, int64_t nidx,
                             double *terms, double *gterms, int64_t *status, void *stream);

/*
 * Vecchia kriging (the prediction of Sec. V-C): for each prediction point t
 * the conditional mean and variance of its observation given the
 * observations at its neighbour set (row t of nbr):
 *   mean[t] = v^T Sigma_JJ^-1 z_J,   var[t] = sigma2 + tau2 - v^T Sigma_JJ^-1 v
 * (the variance of a new observation; the latent field's is var - tau2).
 *   locs, z  [dev] double[n][2], double[n]  the observed points
 *   qlocs    [dev] double[nq][2]            prediction points
 *   nbr      [dev] int32[nq][m]  row t: min(n, m) indices in [0, n) (any
 *                                order, e.g. from vecchia_knn_query)
 *   theta    [dev] double[3];  mean, var [dev] double[nq]
 *   status   [dev] int64[1]: 0; VECCHIA_STATUS_THETA; or t + 1 for the first
 *            point whose block is not positive definite or whose index is out
 *            of range (a prediction point on top of a neighbour with tau2 = 0
 *            has variance 0 and may land here); failed rows hold NaN.
 * No workspace.  Asynchronous on the stream.  Returns VECCHIA_OK,
 * VECCHIA_EINVAL, VECCHIA_EUNSUPPORTED (m > VECCHIA_MAX_M) or VECCHIA_EHIP.
 */
int vecchia_predict(const double *locs, const double *z, int64_t n, const double *qlocs, int64_t nq,
                    const int32_t *nbr, int32_t m, const vecchia_cov *cov, const double *theta, double *mean,
                    double *var, int64_t *status, void *stream);

/*
 * Kernel variants.  Every variant evaluates the same conditionals (Algorithm 1
 * fused per point); they differ in how a workgroup maps onto one conditional:
 *   VECCHIA_VARIANT_UNBLOCKED  256 threads, the block packed in LDS, unblocked
 *                              right-looking Cholesky;
 *   VECCHIA_VARIANT_TILE_W{1,2,4,8}
 *                              the block as 16x16 register tiles over 1, 2, 4
 *                              or 8 wavefronts, Cholesky blocked by tile columns
 *                              with FP64 matrix-core trailing updates.
 * VECCHIA_VARIANT_AUTO uses the per-(m, gradient) table below, or a built-in
 * default: one wavefront up to 62 neighbours with the gradient (and without
 * it for the Matern codes on Euclidean distances; two for the other codes
 * and for kriging from 31 to 62), two up to 94, four beyond.  A tile variant
 * is feasible when each wavefront holds at most 20 tiles;
 * vecchia_variant_feasible reports it.
 */
enum vecchia_variant {
    VECCHIA_VARIANT_AUTO = 0,
    VECCHIA_VARIANT_UNBLOCKED = 1,
    VECCHIA_VARIANT_TILE_W1 = 2,
    VECCHIA_VARIANT_TILE_W2 = 3,
    VECCHIA_VARIANT_TILE_W4 = 4,
    VECCHIA_VARIANT_TILE_W8 = 5
};

/* 1 if `variant` can run conditioning sets of size m, else 0. */
int vecchia_variant_feasible(int32_t m, int32_t variant);

/*
 * Sets the variant used by the entry points above for size m (0..VECCHIA_MAX_M)
 * with (with_grad != 0) or without the gradient; VECCHIA_VARIANT_AUTO restores
 * the default.  This host-side table is the library's only state; an
 * autotuner fills it.  Not thread-safe against concurrent launches.
 * Returns VECCHIA_OK, VECCHIA_EINVAL or VECCHIA_EUNSUPPORTED (infeasible).
 */
int vecchia_set_variant(int32_t m, int32_t with_grad, int32_t variant);

/* The variant the entry points use for (m, with_grad) under the Matern codes
 * on Euclidean distances; negative on bad m. */
int vecchia_get_variant(int32_t m, int32_t with_grad);

/*
 * vecchia_loglik (grad == NULL) or vecchia_loglik_grad (grad != NULL) with an
 * explicit variant; same arguments and results otherwise.
 */
int vecchia_loglik_variant(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                           double nu, const double *theta, int32_t variant, double *out, double *grad,
                           int64_t *status, void *ws, size_t ws_bytes, void *stream);

/* vecchia_loglik_terms with an explicit variant. */
int vecchia_loglik_terms_variant(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                                 double nu, const double *theta, int32_t variant, const int64_t *idx,
                                 int64_t nidx, double *terms, double *gterms, int64_t *status, void *stream);

/* ------------------------------------------------------------------ batched
 * Many parameter vectors and many fields of uneven n and m in one enqueue
 * (not in the paper; it evaluates one theta of one field per call).
 *
 * A field (host struct; its arrays are device arrays, layouts as above):   */
typedef struct vecchia_field {
    const double *locs;   /* [dev] [n][2] */
    const double *z;      /* [dev] [n]    */
    const int32_t *nbr;   /* [dev] [n][m] */
    int64_t n;            /* >= 0 */
    int32_t m;            /* 0..VECCHIA_MAX_M */
} vecchia_field;

/* Opaque plan (host object) and captured graph. */
typedef struct vecchia_plan vecchia_plan;
typedef struct vecchia_graph vecchia_graph;

/*
 * Plans the evaluation of nf fields (1..VECCHIA_MAX_FIELDS) under ntheta
 * parameter vectors each (nf * ntheta <= 2^31 - 1), at smoothness nu, with
 * (with_grad != 0) or without the gradient.  Evaluation e = f * ntheta + q is
 * field f under theta q.  Fields are grouped by tile class ceil((m+2)/16);
 * each class uses the kernel variant that the variant table (vecchia_set_variant
 * / vecchia_autotune) holds for the largest m of the class.  The plan is a host
 * object: planning allocates no device memory, creates no stream and does not
 * synchronise.  The field arrays must stay valid while the plan is used.
 * A class of up to five tile rows (m <= 78) whose ntheta is a multiple of 4
 * takes the one-wavefront variant instead, in lockstep groups
 * (vecchia_plan_class_group), unless the table holds the unblocked variant
 * or lockstep forms are off (vecchia_set_lockstep).  vecchia_plan_class_info
 * reports the variant a class uses; every result is bitwise equal to the
 * single call with that variant.
 * Returns VECCHIA_OK, VECCHIA_EINVAL, VECCHIA_EUNSUPPORTED (m, nf or
 * nf * ntheta too large).
 */
int vecchia_plan_create(const vecchia_field *fields, int32_t nf, int32_t ntheta, double nu, int32_t with_grad,
                        vecchia_plan **plan);

/* vecchia_plan_create under any covariance model (vecchia_cov; smoothness fixed). */
int vecchia_plan_create_cov(const vecchia_field *fields, int32_t nf, int32_t ntheta, const vecchia_cov *cov,
                            int32_t with_grad, vecchia_plan **plan);

/* Workspace (bytes) vecchia_plan_loglik needs: the device table of the plan
 * (64 bytes per field plus 12 per field and class), 36 bytes per (field,
 * theta, point) and a little for partial sums; 0 for a NULL plan. */
size_t vecchia_plan_workspace_size(const vecchia_plan *plan);

/* Number of tile classes of the plan, and the tile rows, variant, field count
 * and item count (points x thetas) of class c. */
int vecchia_plan_num_classes(const vecchia_plan *plan);
int vecchia_plan_class_info(const vecchia_plan *plan, int32_t c, int32_t *tile_rows, int32_t *variant,
                            int32_t *nfields, int64_t *items);

/* Parameter vectors one workgroup of class c evaluates together: 4 when the
 * class has at most five tile rows (m <= 78), a tiled variant and ntheta a
 * multiple of 4 (see vecchia_plan_create), else 1.  The four vectors of a
 * point share the gathered neighbours and the pair distances; each vector's
 * result is bitwise the single-vector one of the same variant.
 * -VECCHIA_EINVAL for a bad plan or class. */
int vecchia_plan_class_group(const vecchia_plan *plan, int32_t c);

/* Whether plans created from now on may use lockstep forms (default 1);
 * returns the previous setting.  Process-wide; for comparisons. */
int vecchia_set_lockstep(int32_t enable);

/* Releases the plan (host memory).  Not while a graph captured from it is used. */
int vecchia_plan_destroy(vecchia_plan *plan);

/*
 * Evaluates every (field, theta) of the plan:
 *   thetas [dev] double [nf][ntheta][3]   (sigma2, beta, tau2) per evaluation
 *   out    [dev] double [nf][ntheta]      log-likelihoods
 *   grad   [dev] double [nf][ntheta][3]   gradients (required iff the plan has them)
 *   status [dev] int64  [nf][ntheta]      per evaluation, as in the header notes
 *   ws     [dev] at least vecchia_plan_workspace_size(plan) bytes, 256-byte aligned
 * Everything is enqueued on `stream`, in order: a few small launches write
 * the plan's device table to the front of ws from their kernel arguments,
 * then one launch per tile class evaluates its (field, theta, point) items
 * (one workgroup per item, last points first), then the sums.  No allocation, no host copy, no synchronisation, no
 * memset: capturable.  Each evaluation's sum uses the same fixed order as
 * vecchia_loglik, so with the same variant the results are bitwise equal to
 * single calls.  Calls that share a workspace must not overlap.
 */
int vecchia_plan_loglik(const vecchia_plan *plan, const double *thetas, double *out, double *grad, int64_t *status,
                        void *ws, size_t ws_bytes, void *stream);

/*
 * The one-call batched form (Matern, Euclidean): plans on the host and
 * evaluates as vecchia_plan_loglik, with the same arguments and results.
 *   fields  [host] vecchia_field[nf]
 *   ws      [dev] at least vecchia_batched_workspace(fields, nf, ntheta) bytes
 * The plan lives only during the call: everything the device needs travels
 * in kernel arguments or is written into ws.  Returns as vecchia_plan_create
 * and vecchia_plan_loglik.
 */
size_t vecchia_batched_workspace(const vecchia_field *fields, int32_t nf, int32_t ntheta);
int vecchia_loglik_batched(const vecchia_field *fields, int32_t nf, const double *thetas, int32_t ntheta, double nu,
                           int32_t with_grad, double *out, double *grad, int64_t *status, void *ws, size_t ws_bytes,
                           void *stream);

/*
 * Captures vecchia_plan_loglik with these arguments into a HIP graph on
 * `stream` (not the null stream) and instantiates it.  Replays read the device
 * arrays in place, so new parameter vectors are written into `thetas` between
 * launches.  vecchia_batched_graph_launch replays it on `stream`.
 */
int vecchia_batched_graph_create(const vecchia_plan *plan, const double *thetas, double *out, double *grad,
                                 int64_t *status, void *ws, size_t ws_bytes, void *stream, vecchia_graph **graph);
int vecchia_batched_graph_launch(vecchia_graph *graph, void *stream);
int vecchia_batched_graph_destroy(vecchia_graph *graph);

/*
 * Autotuner: times every feasible variant on the last `sample` points of
 * `field` (points with full conditioning sets where possible), best of `reps`
 * runs, with (with_grad != 0) or without the gradient, and stores the fastest
 * in the variant table for (field->m, with_grad).
 *   theta        [dev] double[3]
 *   ws           [dev] at least 40 * field->n bytes
 *   best         [host] receives the chosen variant
 *   us_per_point [host] double[6] or NULL: microseconds per point for each
 *                variant (index = variant; -1 if infeasible; [0] = the best)
 * Synchronises the stream.  Returns VECCHIA_OK or an error code.
 */
int vecchia_autotune(const vecchia_field *field, double nu, int32_t with_grad, const double *theta, int64_t sample,
                     int32_t reps, void *ws, size_t ws_bytes, void *stream, int32_t *best, double *us_per_point);

/*
 * Preprocessing before the likelihood: conditioning sets and ordering
 * (Sec. IV-A/IV-B, the loop ahead of the likelihood in Algorithm 1).
 *
 * vecchia_knn: for each 0-based point i of locs (in the given order), the
 * min(i, m) points j < i nearest to it, as the likelihood's `nbr` input.
 *   locs  [dev] double[n][2], row-major, finite coordinates
 *   n     number of points, n >= 0
 *   m     set size, 0 <= m <= VECCHIA_MAX_M
 *   nbr   [dev] int32[n][m], written: row i holds the indices ordered by
 *         (squared distance, index) ascending, squared distances taken as
 *         dx*dx + dy*dy with each product rounded; slots past min(i, m) = -1
 *   ws    [dev] workspace of at least vecchia_knn_workspace_size(n) bytes
 *   stream  HIP stream (hipStream_t, NULL = default); asynchronous
 * Exact: equal to brute force over all j < i, independent of the device.
 * The search uses a uniform grid over the bounding box (about two points per
 * cell); non-finite coordinates give unspecified sets for the rows they touch.
 * Returns VECCHIA_OK, VECCHIA_EINVAL (null pointers, n < 0, m < 0, n > 2^31 - 1),
 * VECCHIA_EUNSUPPORTED (m > VECCHIA_MAX_M), VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
size_t vecchia_knn_workspace_size(int64_t n);
int vecchia_knn(const double *locs, int64_t n, int32_t m, int32_t *nbr, void *ws, size_t ws_bytes, void *stream);

/*
 * vecchia_knn under a metric: VECCHIA_EUCLIDEAN as vecchia_knn;
 * VECCHIA_GREAT_CIRCLE with locs as (longitude, latitude) in degrees, ranking
 * candidates by the haversine value sin^2(dlat/2) + cos lat_i cos lat_j
 * sin^2(dlon/2) (monotone in the great-circle distance of Sec. V-C, latitude
 * and longitude differences taken in degrees before conversion), ties by
 * index.  The search uses the grid of vecchia_knn over (longitude,
 * latitude) with a lower bound of the haversine value for unscanned rings;
 * latitudes must lie in [-90, 90], and a longitude span above 180 degrees
 * makes every query scan all cells.  The haversine value uses the device's
 * sine and cosine, so keys equal to the last bits may order differently
 * from another library's.  Other arguments and returns as vecchia_knn; an
 * unknown metric is VECCHIA_EINVAL.
 */
int vecchia_knn_metric(const double *locs, int64_t n, int32_t m, int32_t metric, int32_t *nbr, void *ws,
                       size_t ws_bytes, void *stream);

/*
 * Neighbour sets of prediction points for kriging (Sec. V-C): row t of nbr
 * receives the min(n, m) points of locs nearest to qlocs[t] (all n points are
 * candidates), ordered as vecchia_knn_metric orders them, -1 past min(n, m).
 *   locs   [dev] double[n][2];  qlocs [dev] double[nq][2];  nbr [dev] int32[nq][m]
 *   ws     [dev] at least vecchia_knn_workspace_size(n) bytes
 * Both metrics use the grid of vecchia_knn over locs (queries outside its
 * bounding box included), as vecchia_knn_metric.
 * Asynchronous.  Returns VECCHIA_OK, VECCHIA_EINVAL, VECCHIA_EUNSUPPORTED
 * (m > VECCHIA_MAX_M), VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
int vecchia_knn_query(const double *locs, int64_t n, const double *qlocs, int64_t nq, int32_t m, int32_t metric,
                      int32_t *nbr, void *ws, size_t ws_bytes, void *stream);

/*
 * vecchia_morton_order: the Morton (Z-order) ordering of Sec. IV-A.  Each
 * coordinate maps to a 16-bit cell floor((v - min) / (max - min) * 65536),
 * clamped to [0, 65535], over the bounding box (zero extent: cell 0); the code
 * interleaves x bits (even positions) and y bits (odd positions).
 *   locs  [dev] double[n][2], finite
 *   perm  [dev] int64[n], written: point indices by ascending code, ties by
 *         ascending index (locs[perm[0]] comes first in the new order)
 *   ws    [dev] at least vecchia_morton_workspace_size(n) bytes
 * Returns VECCHIA_OK, VECCHIA_EINVAL, VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
size_t vecchia_morton_workspace_size(int64_t n);
int vecchia_morton_order(const double *locs, int64_t n, int64_t *perm, void *ws, size_t ws_bytes, void *stream);

/*
 * vecchia_random_order: the random ordering of Sec. IV-A, reproducible from a
 * seed: perm lists 0..n-1 by ascending key(i) = mix64(seed XOR i), mix64 the
 * splitmix64 finaliser (a bijection on 64-bit words, so the keys are
 * distinct).  Device radix sort, kernel launches only (capturable).
 *   perm [dev] int64[n];  ws [dev] at least vecchia_random_order_workspace_size(n)
 * Returns VECCHIA_OK, VECCHIA_EINVAL (n < 0, n > 2^31 - 1, null perm),
 * VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
size_t vecchia_random_order_workspace_size(int64_t n);
int vecchia_random_order(int64_t n, uint64_t seed, int64_t *perm, void *ws, size_t ws_bytes, void *stream);

/*
 * Approximate maxmin ordering: maxmin orders points so that each one is as
 * far as possible from those before it, the ordering Sec. IV-A names as
 * accurate but too costly at scale.  This approximation elects points in
 * rounds over finer and finer grids:
 *   - Round r uses G x G square cells, G = 2^min(r, Lmax), on the square box
 *     whose lower-left corner is that of the bounding box and whose side w is
 *     the larger side of the bounding box (1 when zero).  Lmax is the least
 *     L >= 0 with 4^L >= n, plus 1, at most 15.
 *   - A point's cell per axis is min(floor((v - v0) / w * G), G - 1), or 0
 *     when negative or NaN.
 *   - Every cell elects its unselected point with the least squared distance
 *     to the cell centre v0 + (c + 1/2) w / G, taken as dx*dx + dy*dy with
 *     every operation rounded; ties go to the lower index.
 *   - A round's points follow all earlier rounds, in ascending
 *     mix64(seed XOR i), the splitmix64 finaliser (a bijection).
 *   - After Lmax + 33 rounds, the remaining points follow in that key order.
 * The first points of the ordering are thus spread over the domain at every
 * scale, as maxmin's are.
 *   locs [dev] double[n][2];  perm [dev] int64[n] receives the permutation
 *   ws   [dev] at least vecchia_maxmin_workspace_size(n) bytes: 12 bytes
 *        per cell of the finest grid (4 to 16 cells per point) plus sort
 *        buffers of about 40 bytes per point
 * Synchronises the stream once per round (at most Lmax + 34 rounds).  Exact:
 * equal to the definition.  Returns VECCHIA_OK, VECCHIA_EINVAL (n < 0,
 * n > 2^31 - 1, null pointers), VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
size_t vecchia_maxmin_workspace_size(int64_t n);
int vecchia_maxmin_order(const double *locs, int64_t n, uint64_t seed, int64_t *perm, void *ws, size_t ws_bytes,
                         void *stream);

/*
 * Maximum-likelihood fit of theta = (sigma2, beta, tau2) at fixed nu, the use
 * of the likelihood in Sec. V (the paper drives NLopt without derivatives;
 * this driver uses the fused gradient).  Projected limited-memory BFGS in
 * phi = log(theta) within [log lower, log upper], backtracking line search
 * with the Armijo condition, objective -l/n.  An evaluation that fails (a
 * non-positive pivot, non-finite value) counts as +infinity, so steps back
 * off from it.  Stops when the largest free component of d(-l/n)/dphi is
 * below gtol, after three steps that lower -l/n by at most
 * ftol * max(1, |l|/n), after max_iter iterations, or when no step along the
 * search direction decreases the objective.
 */
typedef struct vecchia_mle_options {
    int32_t max_iter;  /* iterations (default 200) */
    int32_t history;   /* BFGS pairs kept, 1..20 (default 8) */
    double gtol;       /* default 1e-7 */
    double ftol;       /* default 1e-13 */
    double lower[3];   /* bounds on theta, 0 < lower <= upper, finite (defaults 1e-8, 1e-8, 1e-10) */
    double upper[3];   /* (defaults 1e8 each) */
    int32_t trial_steps; /* step lengths the line search evaluates per device round trip, 1..8 (default 4) */
} vecchia_mle_options;

void vecchia_mle_default_options(vecchia_mle_options *opt);
size_t vecchia_mle_workspace_size(int64_t n, int32_t m);

/*
 *   locs, z, nbr, n, m, nu  as vecchia_loglik_grad (device arrays), n >= 1
 *   theta0      [host] double[3] start, each > 0 (clipped into the bounds)
 *   options     [host] or NULL for the defaults
 *   theta       [host] double[3] receives the estimate
 *   loglik      [host] double or NULL: l at the estimate
 *   grad        [host] double[3] or NULL: dl/dtheta at the estimate
 *   iterations, evaluations, round_trips  [host] int32 or NULL: iterations,
 *               parameter vectors evaluated, device round trips (launch,
 *               read-back and synchronisation)
 *   ws          [dev] at least vecchia_mle_workspace_size(n, m) bytes, 256-byte aligned
 * Each round trip evaluates a set of parameter vectors as the theta columns
 * of one batched launch (a host plan over the field): the line search tries
 * a quasi-Newton step alone, and once it backs off (or without curvature
 * information) the next trial_steps halvings of the step at once, taking
 * the longest that satisfies the Armijo condition, the step one-at-a-time
 * backtracking would take.  Round trips of four or eight vectors take the
 * plan's lockstep form, so at 63..78 neighbours their values and those of
 * single-vector round trips come from different kernel variants and may
 * differ in the last bits.  Synchronises the stream once per round trip.  Returns VECCHIA_OK,
 * VECCHIA_EINVAL (bad arguments or options, or theta0 does not evaluate),
 * VECCHIA_EUNSUPPORTED, VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
int vecchia_mle(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                const double *theta0, const vecchia_mle_options *options, double *theta, double *loglik,
                double *grad, int32_t *iterations, int32_t *evaluations, int32_t *round_trips, void *ws,
                size_t ws_bytes, void *stream);

/* vecchia_mle under any covariance model (smoothness fixed, as vecchia_loglik_cov). */
int vecchia_mle_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                    const vecchia_cov *cov, const double *theta0, const vecchia_mle_options *options, double *theta,
                    double *loglik, double *grad, int32_t *iterations, int32_t *evaluations, int32_t *round_trips,
                    void *ws, size_t ws_bytes, void *stream);

/*
 * Exact Gaussian-process log-likelihood, Eq. (1), for the KL divergence of
 * Eq. (9): KL(N_0 || N_a) = l_0(theta; 0) - l_a(theta; 0), the exact minus
 * the Vecchia log-likelihood at y = 0.  Accuracy harness, not the hot path:
 * the n x n covariance (Matern closed forms of Eq. (2), nugget on the
 * diagonal) is generated in the workspace and factored as in
 * vecchia_dense_logdet; l = -1/2 (n log 2 pi + log det Sigma + z^T Sigma^-1 z).
 *   locs    [dev] double[n][2];  z [dev] double[n], or NULL for y = 0
 *   n       1 <= n <= 2^30; in practice the 8 n^2-byte workspace bounds it
 *           (n = 180,000 needs 259 GB)
 *   theta   [dev] double[3] (sigma2, beta, tau2);  nu in {0.5, 1.5, 2.5}
 *   out     [dev] double[1];  status [dev] int64[1]: 0, VECCHIA_STATUS_THETA,
 *           or the 1-based column of the first non-positive pivot (out = NaN)
 *   ws      [dev] at least vecchia_exact_workspace_size(n) bytes (8 n^2 + small)
 * rocBLAS/rocSOLVER may allocate scratch of their own.  Synchronises the
 * stream.  Returns VECCHIA_OK, VECCHIA_EINVAL, VECCHIA_EUNSUPPORTED (n too
 * large), VECCHIA_EWORKSPACE or VECCHIA_EHIP.
 */
size_t vecchia_exact_workspace_size(int64_t n);
int vecchia_exact_loglik(const double *locs, const double *z, int64_t n, double nu, const double *theta, double *out,
                         int64_t *status, void *ws, size_t ws_bytes, void *stream);

/*
 * Log-determinant (and optionally z^T A^-1 z) of a dense symmetric positive
 * definite matrix: the two terms of the Gaussian log-density of Eq. (1).  A is
 * overwritten by its Cholesky factor (lower triangle; the strict upper
 * triangle is not read) by a left-looking blocked factorisation: 1024-column
 * diagonal blocks factored by rocSOLVER, panel updates by rocBLAS GEMM calls
 * whose inner dimension is at most 8192, panel solves by rocBLAS TRSM.
 *   A       [dev] double, column-major, n x n with leading dimension lda >= n
 *   z       [dev] double[n] or NULL;  quad [dev] double[1], required with z
 *   logdet  [dev] double[1]
 *   status  [dev] int64[1]: 0, or the 1-based column of the first
 *           non-positive pivot, or n when a result is not finite (then
 *           logdet and quad are NaN)
 *   ws      [dev] at least vecchia_dense_logdet_workspace_size(n) bytes
 * Synchronises the stream.  Returns VECCHIA_OK, VECCHIA_EINVAL,
 * VECCHIA_EUNSUPPORTED (n or lda above 2^30), VECCHIA_EWORKSPACE or
 * VECCHIA_EHIP.
 */
size_t vecchia_dense_logdet_workspace_size(int64_t n);
int vecchia_dense_logdet(double *A, int64_t n, int64_t lda, const double *z, double *logdet, double *quad,
                         int64_t *status, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VECCHIA_H */

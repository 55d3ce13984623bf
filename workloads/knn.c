/*
 * m nearest previously-ordered neighbours (the conditioning sets J_i of the
 * Vecchia approximation, Sec. IV-B, Eq. (7); the preprocessing loop of
 * Algorithm 1).  This is INPUT PREPARATION shared by the oracle and the GPU
 * path: it decides which points condition which, and holds none of the
 * likelihood arithmetic.
 *
 * For 0-based point i (in the given order) the row out[i][0..m) receives the
 * min(i, m) indices j < i with the smallest Euclidean distance to point i,
 * sorted by (squared distance, index) ascending; the remaining slots are -1.
 * Distances are compared as dx*dx + dy*dy in IEEE double without FMA
 * contraction (build with -ffp-contract=off), so the result does not depend on
 * the machine or the thread count.
 *
 * Search: a uniform grid of about two points per cell over the bounding box;
 * each cell lists its points in ascending index, so the points before i are a
 * prefix of every list.  Rings of cells around point i are scanned until the
 * nearest unscanned cell is farther than the current m-th best.  Points with
 * small i are handled by brute force over 0..i-1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int32_t m, cnt;
    double *d;   /* [m] squared distances, ascending */
    int32_t *ix; /* [m] matching indices */
} topm_t;

static inline int topm_less(double d1, int32_t i1, double d2, int32_t i2) {
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

static inline void topm_push(topm_t *t, double d, int32_t j) {
    if (t->cnt == t->m) {
        if (!topm_less(d, j, t->d[t->m - 1], t->ix[t->m - 1])) return;
        t->cnt--; /* drop the current worst */
    }
    int32_t p = t->cnt;
    while (p > 0 && topm_less(d, j, t->d[p - 1], t->ix[p - 1])) {
        t->d[p] = t->d[p - 1];
        t->ix[p] = t->ix[p - 1];
        p--;
    }
    t->d[p] = d;
    t->ix[p] = j;
    t->cnt++;
}

static inline double sqdist(const double *a, const double *b) {
    double dx = a[0] - b[0];
    double dy = a[1] - b[1];
    return dx * dx + dy * dy;
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure. */
int knn_previous(const double *locs, int64_t n, int32_t m, int32_t *out, int32_t nthreads) {
    if (n < 0 || m < 0 || (n > 0 && (!locs || !out))) return -1;
    if (n == 0) return 0;
    if (m == 0) return 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);

    double xmin = locs[0], xmax = locs[0], ymin = locs[1], ymax = locs[1];
    for (int64_t i = 1; i < n; ++i) {
        double x = locs[2 * i], y = locs[2 * i + 1];
        if (x < xmin) xmin = x;
        if (x > xmax) xmax = x;
        if (y < ymin) ymin = y;
        if (y > ymax) ymax = y;
    }
    int64_t g = (int64_t)ceil(sqrt((double)n / 2.0));
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    double wx = (xmax - xmin), wy = (ymax - ymin);
    double w = wx > wy ? wx : wy;
    if (!(w > 0)) w = 1.0;
    double h = w / (double)g * (1.0 + 1e-12);

    int64_t ncell = g * g;
    int64_t *start = (int64_t *)calloc((size_t)(ncell + 1), sizeof(int64_t));
    int32_t *cellof = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *list = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!start || !cellof || !list) {
        free(start); free(cellof); free(list);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = (int64_t)((locs[2 * i] - xmin) / h);
        int64_t cy = (int64_t)((locs[2 * i + 1] - ymin) / h);
        if (cx >= g) cx = g - 1;
        if (cy >= g) cy = g - 1;
        if (cx < 0) cx = 0;
        if (cy < 0) cy = 0;
        cellof[i] = (int32_t)(cy * g + cx);
        start[cellof[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
        if (!fill) { free(start); free(cellof); free(list); return -2; }
        memcpy(fill, start, (size_t)ncell * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) list[fill[cellof[i]]++] = (int32_t)i; /* ascending i */
        free(fill);
    }

    const int64_t brute_below = 4 * (int64_t)m + 64;
    int failed = 0;
#pragma omp parallel
    {
        topm_t t;
        t.m = m;
        t.d = (double *)malloc((size_t)m * sizeof(double));
        t.ix = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        if (!t.d || !t.ix) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            if (failed) continue;
            int32_t *row = out + i * (int64_t)m;
            const double *p = locs + 2 * i;
            t.cnt = 0;
            int32_t want = (int32_t)(i < m ? i : m);
            if (i < brute_below) {
                for (int64_t j = 0; j < i; ++j) topm_push(&t, sqdist(p, locs + 2 * j), (int32_t)j);
            } else {
                int64_t cx = cellof[i] % g, cy = cellof[i] / g;
                for (int64_t R = 0;; ++R) {
                    int64_t x0 = cx - R, x1 = cx + R, y0 = cy - R, y1 = cy + R;
                    for (int64_t yy = y0; yy <= y1; ++yy) {
                        if (yy < 0 || yy >= g) continue;
                        int edge_row = (yy == y0 || yy == y1);
                        for (int64_t xx = x0; xx <= x1; ++xx) {
                            if (xx < 0 || xx >= g) continue;
                            if (!edge_row && xx != x0 && xx != x1) continue;
                            int64_t c = yy * g + xx;
                            for (int64_t q = start[c]; q < start[c + 1]; ++q) {
                                int32_t j = list[q];
                                if (j >= i) break;
                                topm_push(&t, sqdist(p, locs + 2 * (int64_t)j), j);
                            }
                        }
                    }
                    if (x0 <= 0 && y0 <= 0 && x1 >= g - 1 && y1 >= g - 1) break; /* whole grid seen */
                    if (t.cnt == want) {
                        /* nearest point of any cell outside the scanned (2R+1)^2 block */
                        double bx0 = xmin + (double)x0 * h, bx1 = xmin + (double)(x1 + 1) * h;
                        double by0 = ymin + (double)y0 * h, by1 = ymin + (double)(y1 + 1) * h;
                        double gap = p[0] - bx0;
                        if (bx1 - p[0] < gap) gap = bx1 - p[0];
                        if (p[1] - by0 < gap) gap = p[1] - by0;
                        if (by1 - p[1] < gap) gap = by1 - p[1];
                        if (gap > 0 && gap * gap > t.d[t.cnt - 1]) break;
                    }
                }
            }
            for (int32_t q = 0; q < m; ++q) row[q] = q < t.cnt ? t.ix[q] : -1;
        }
        free(t.d);
        free(t.ix);
    }
    free(start);
    free(cellof);
    free(list);
    return failed ? -2 : 0;
}

// Batched evaluation: many parameter vectors and many fields of uneven n and
// m in one enqueue (or one graph launch), and the autotuner that picks the
// kernel variant per conditioning-set size.
//
// A plan groups the fields by tile class T = ceil((m+2)/16).  Items of a class
// are (field, theta, point) triples; one launch per class evaluates all of
// them with the class's variant.  The classes run concurrently on plan-owned
// streams forked from and joined back into the caller's stream.  A segmented
// reduction then forms every evaluation (field, theta) with the same
// fixed-order sum as the single-evaluation entry points, so a batched result
// is bitwise equal to the single call with the same variant.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "launch.h"
#include "reduce.h"
#include "vecchia.h"

using namespace vecchia;

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// One evaluation: its rows of the per-point arrays and its reduce blocks.
struct EvalDev {
    int64_t vals0;  // first row
    int64_t n;      // rows (points of the field)
    int64_t pb0;    // first reduce block
    int64_t nb;     // reduce blocks
};

struct ClassPlan {
    int T = 0;
    int variant = 0;
    int32_t m_max = 0;
    std::vector<int32_t> fidx;   // fields of the class
    std::vector<int64_t> item0;  // prefix sums of ntheta * n over fidx (size nfc + 1)
    size_t off_fidx = 0, off_item0 = 0;
};

__global__ void __launch_bounds__(kReduceThreads) batched_reduce_kernel(const double *__restrict__ vals,
                                                                        const int32_t *__restrict__ flags,
                                                                        const EvalDev *__restrict__ evals,
                                                                        int32_t nevals,
                                                                        double *__restrict__ partial,
                                                                        int64_t *__restrict__ pfail) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nevals;
    while (hi - lo > 1) {  // last evaluation whose first block is <= b
        const int mid = (lo + hi) >> 1;
        if (evals[mid].pb0 <= b) lo = mid;
        else hi = mid;
    }
    // evaluations with n = 0 own no block; skip to the one that owns b
    while (lo + 1 < nevals && evals[lo].nb == 0) ++lo;
    const EvalDev E = evals[lo];
    reduce_segment_block(vals + 4 * E.vals0, flags + E.vals0, E.n, b - E.pb0, partial + 8 * b, pfail + b);
}

__global__ void __launch_bounds__(kFinalizeThreads) batched_finalize_kernel(const double *__restrict__ partial,
                                                                            const int64_t *__restrict__ pfail,
                                                                            const EvalDev *__restrict__ evals,
                                                                            const double *__restrict__ thetas,
                                                                            double *__restrict__ out,
                                                                            double *__restrict__ grad,
                                                                            int64_t *__restrict__ status) {
    const int64_t e = blockIdx.x;
    const EvalDev E = evals[e];
    finalize_segment(partial + 8 * E.pb0, pfail + E.pb0, E.nb, thetas + 3 * e, out + e, grad ? grad + 3 * e : nullptr,
                     status + e);
}

}  // namespace

struct vecchia_plan {
    int32_t nf = 0, ntheta = 0;
    int nuc = 0;         // covariance code (launch_any)
    double alpha = 1.0;  // power-exponential exponent
    bool grad = false;
    std::vector<FieldDev> fields;
    std::vector<EvalDev> evals;
    std::vector<ClassPlan> classes;
    int64_t total_rows = 0, total_pblocks = 0;
    char *d_buf = nullptr;  // device copy of fields, evals and the class tables
    size_t off_fields = 0, off_evals = 0;
    std::vector<hipStream_t> streams;  // one per class after the first
    std::vector<hipEvent_t> events;    // fork event + one join event per extra class
    size_t ws_vals = 0, ws_flags = 0, ws_partial = 0, ws_pfail = 0, ws_bytes = 0;
};

struct vecchia_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void plan_release(vecchia_plan *p) {
    if (!p) return;
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    for (hipStream_t s : p->streams) (void)hipStreamDestroy(s);
    if (p->d_buf) (void)hipFree(p->d_buf);
    delete p;
}

int run_batched(const vecchia_plan *p, const double *thetas, double *out, double *grad, int64_t *status, void *ws,
                size_t ws_bytes, hipStream_t s) {
    if (!p || !thetas || !out || !status || (p->grad && !grad)) return VECCHIA_EINVAL;
    if (!ws || ws_bytes < p->ws_bytes) return VECCHIA_EWORKSPACE;
    char *w = (char *)ws;
    double *vals = (double *)(w + p->ws_vals);
    int32_t *flags = (int32_t *)(w + p->ws_flags);
    double *partial = (double *)(w + p->ws_partial);
    int64_t *pfail = (int64_t *)(w + p->ws_pfail);
    const FieldDev *dfields = (const FieldDev *)(p->d_buf + p->off_fields);
    const EvalDev *devals = (const EvalDev *)(p->d_buf + p->off_evals);

    const size_t nc = p->classes.size();
    if (nc > 1) {
        if (hipEventRecord(p->events[0], s) != hipSuccess) return VECCHIA_EHIP;
        for (size_t c = 1; c < nc; ++c)
            if (hipStreamWaitEvent(p->streams[c - 1], p->events[0], 0) != hipSuccess) return VECCHIA_EHIP;
    }
    for (size_t c = 0; c < nc; ++c) {
        const ClassPlan &C = p->classes[c];
        hipStream_t cs = (c == 0) ? s : p->streams[c - 1];
        EvalArgs a{};
        a.k.theta = thetas;
        a.k.fields = dfields;
        a.k.fidx = (const int32_t *)(p->d_buf + C.off_fidx);
        a.k.item0 = (const int64_t *)(p->d_buf + C.off_item0);
        a.k.nfc = (int32_t)C.fidx.size();
        a.k.ell = vals;
        a.k.ell_stride = 4;
        a.k.g = vals + 1;
        a.k.g_stride = 4;
        a.k.flags = flags;
        a.k.alpha = p->alpha;
        a.t_begin = 0;
        a.t_end = C.item0.back();
        a.m_max = C.m_max;
        const int rc = launch_any(p->nuc, p->grad, C.variant, a, cs);
        if (rc != VECCHIA_OK) return rc;
    }
    if (nc > 1) {
        for (size_t c = 1; c < nc; ++c) {
            if (hipEventRecord(p->events[c], p->streams[c - 1]) != hipSuccess) return VECCHIA_EHIP;
            if (hipStreamWaitEvent(s, p->events[c], 0) != hipSuccess) return VECCHIA_EHIP;
        }
    }
    if (p->total_pblocks > 0)
        hipLaunchKernelGGL(batched_reduce_kernel, dim3((unsigned)p->total_pblocks), dim3(kReduceThreads), 0, s, vals,
                           flags, devals, (int32_t)p->evals.size(), partial, pfail);
    hipLaunchKernelGGL(batched_finalize_kernel, dim3((unsigned)p->evals.size()), dim3(kFinalizeThreads), 0, s,
                       partial, pfail, devals, thetas, out, p->grad ? grad : nullptr, status);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

}  // namespace

extern "C" {

int vecchia_plan_create(const vecchia_field *fields, int32_t nf, int32_t ntheta, double nu, int32_t with_grad,
                        vecchia_plan **plan) {
    const vecchia_cov cov{VECCHIA_MATERN, VECCHIA_EUCLIDEAN, nu};
    return vecchia_plan_create_cov(fields, nf, ntheta, &cov, with_grad, plan);
}

int vecchia_plan_create_cov(const vecchia_field *fields, int32_t nf, int32_t ntheta, const vecchia_cov *cov,
                            int32_t with_grad, vecchia_plan **plan) {
    if (!plan) return VECCHIA_EINVAL;
    *plan = nullptr;
    double alpha = 1.0;
    const int kc = cov_code(cov, &alpha);
    if (!fields || nf < 1 || ntheta < 1 || kc < 0) return VECCHIA_EINVAL;
    if (nf > VECCHIA_MAX_FIELDS) return VECCHIA_EUNSUPPORTED;
    for (int32_t f = 0; f < nf; ++f) {
        const vecchia_field &F = fields[f];
        if (F.n < 0 || F.m < 0) return VECCHIA_EINVAL;
        if (F.m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
        if (F.n > 0 && (!F.locs || !F.z)) return VECCHIA_EINVAL;
        if (F.n > 1 && F.m > 0 && !F.nbr) return VECCHIA_EINVAL;
    }
    vecchia_plan *p = new (std::nothrow) vecchia_plan();
    if (!p) return VECCHIA_EINVAL;
    p->nf = nf;
    p->ntheta = ntheta;
    p->nuc = kc;
    p->alpha = alpha;
    p->grad = with_grad != 0;
    int64_t rows = 0, pblocks = 0;
    for (int32_t f = 0; f < nf; ++f) {
        FieldDev d{};
        d.locs = fields[f].locs;
        d.z = fields[f].z;
        d.nbr = fields[f].nbr;
        d.n = fields[f].n;
        d.m = fields[f].m;
        d.eval0 = f * ntheta;
        d.vals0 = rows;
        p->fields.push_back(d);
        for (int32_t q = 0; q < ntheta; ++q) {
            EvalDev e{};
            e.vals0 = rows + (int64_t)q * d.n;
            e.n = d.n;
            e.pb0 = pblocks;
            e.nb = num_reduce_blocks(d.n);
            pblocks += e.nb;
            p->evals.push_back(e);
        }
        rows += (int64_t)ntheta * d.n;
    }
    p->total_rows = rows;
    p->total_pblocks = pblocks;
    // tile classes, largest first so the longest launch starts first
    for (int T = (VECCHIA_MAX_M + 2 + 15) / 16; T >= 1; --T) {
        ClassPlan C;
        C.T = T;
        C.item0.push_back(0);
        for (int32_t f = 0; f < nf; ++f) {
            if (tile_rows(fields[f].m) != T || fields[f].n == 0) continue;
            C.fidx.push_back(f);
            C.item0.push_back(C.item0.back() + (int64_t)ntheta * fields[f].n);
            C.m_max = std::max(C.m_max, fields[f].m);
        }
        if (C.fidx.empty()) continue;
        C.variant = resolve_variant(C.m_max, p->grad, 0);
        p->classes.push_back(C);
    }
    // device tables
    size_t off = 0;
    p->off_fields = off;
    off = align256(off + sizeof(FieldDev) * p->fields.size());
    p->off_evals = off;
    off = align256(off + sizeof(EvalDev) * p->evals.size());
    for (ClassPlan &C : p->classes) {
        C.off_fidx = off;
        off = align256(off + sizeof(int32_t) * C.fidx.size());
        C.off_item0 = off;
        off = align256(off + sizeof(int64_t) * C.item0.size());
    }
    std::vector<char> host(off, 0);
    std::copy((const char *)p->fields.data(), (const char *)(p->fields.data() + p->fields.size()),
              host.data() + p->off_fields);
    std::copy((const char *)p->evals.data(), (const char *)(p->evals.data() + p->evals.size()),
              host.data() + p->off_evals);
    for (const ClassPlan &C : p->classes) {
        std::copy((const char *)C.fidx.data(), (const char *)(C.fidx.data() + C.fidx.size()), host.data() + C.off_fidx);
        std::copy((const char *)C.item0.data(), (const char *)(C.item0.data() + C.item0.size()),
                  host.data() + C.off_item0);
    }
    if (hipMalloc((void **)&p->d_buf, std::max<size_t>(off, 256)) != hipSuccess ||
        hipMemcpy(p->d_buf, host.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
        plan_release(p);
        return VECCHIA_EHIP;
    }
    // streams and events for running the classes concurrently (default priority)
    for (size_t c = 1; c < p->classes.size(); ++c) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            plan_release(p);
            return VECCHIA_EHIP;
        }
        p->streams.push_back(st);
    }
    for (size_t c = 0; c < std::max<size_t>(p->classes.size(), 1); ++c) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            plan_release(p);
            return VECCHIA_EHIP;
        }
        p->events.push_back(ev);
    }
    // workspace layout
    size_t w = 0;
    p->ws_vals = w;
    w = align256(w + (size_t)rows * 4 * sizeof(double));
    p->ws_flags = w;
    w = align256(w + (size_t)rows * sizeof(int32_t));
    p->ws_partial = w;
    w = align256(w + (size_t)pblocks * 8 * sizeof(double));
    p->ws_pfail = w;
    w = align256(w + (size_t)pblocks * sizeof(int64_t));
    p->ws_bytes = w + 256;
    *plan = p;
    return VECCHIA_OK;
}

size_t vecchia_plan_workspace_size(const vecchia_plan *plan) { return plan ? plan->ws_bytes : 0; }

int vecchia_plan_num_classes(const vecchia_plan *plan) { return plan ? (int)plan->classes.size() : -VECCHIA_EINVAL; }

int vecchia_plan_class_info(const vecchia_plan *plan, int32_t c, int32_t *tile_rows_out, int32_t *variant,
                            int32_t *nfields, int64_t *items) {
    if (!plan || c < 0 || c >= (int32_t)plan->classes.size()) return VECCHIA_EINVAL;
    const ClassPlan &C = plan->classes[c];
    if (tile_rows_out) *tile_rows_out = C.T;
    if (variant) *variant = C.variant;
    if (nfields) *nfields = (int32_t)C.fidx.size();
    if (items) *items = C.item0.back();
    return VECCHIA_OK;
}

int vecchia_plan_destroy(vecchia_plan *plan) {
    if (!plan) return VECCHIA_EINVAL;
    plan_release(plan);
    return VECCHIA_OK;
}

int vecchia_loglik_batched(const vecchia_plan *plan, const double *thetas, double *out, double *grad,
                           int64_t *status, void *ws, size_t ws_bytes, void *stream) {
    return run_batched(plan, thetas, out, grad, status, ws, ws_bytes, (hipStream_t)stream);
}

int vecchia_batched_graph_create(const vecchia_plan *plan, const double *thetas, double *out, double *grad,
                                 int64_t *status, void *ws, size_t ws_bytes, void *stream, vecchia_graph **graph) {
    if (!graph) return VECCHIA_EINVAL;
    *graph = nullptr;
    if (!stream) return VECCHIA_EINVAL;  // the null stream cannot be captured
    hipStream_t s = (hipStream_t)stream;
    vecchia_graph *g = new (std::nothrow) vecchia_graph();
    if (!g) return VECCHIA_EINVAL;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete g;
        return VECCHIA_EHIP;
    }
    const int rc = run_batched(plan, thetas, out, grad, status, ws, ws_bytes, s);
    const hipError_t e1 = hipStreamEndCapture(s, &g->graph);
    if (rc != VECCHIA_OK || e1 != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return rc != VECCHIA_OK ? rc : VECCHIA_EHIP;
    }
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return VECCHIA_EHIP;
    }
    *graph = g;
    return VECCHIA_OK;
}

int vecchia_batched_graph_launch(vecchia_graph *graph, void *stream) {
    if (!graph || !graph->exec) return VECCHIA_EINVAL;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

int vecchia_batched_graph_destroy(vecchia_graph *graph) {
    if (!graph) return VECCHIA_EINVAL;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return VECCHIA_OK;
}

int vecchia_autotune(const vecchia_field *field, double nu, int32_t with_grad, const double *theta, int64_t sample,
                     int32_t reps, void *ws, size_t ws_bytes, void *stream, int32_t *best, double *us_per_point) {
    if (!field || !theta || !best || nu_code(nu) < 0 || reps < 1 || sample < 1) return VECCHIA_EINVAL;
    const int64_t n = field->n;
    const int32_t m = field->m;
    if (m < 0 || n < 1) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    if (!field->locs || !field->z || (m > 0 && n > 1 && !field->nbr)) return VECCHIA_EINVAL;
    // time rows [t_begin, n): the last `sample` points, starting no earlier than m (full sets) when possible
    int64_t t_begin = n - sample;
    if (t_begin < 0) t_begin = 0;
    if (t_begin < m && m < n) t_begin = m;
    if (!ws || ws_bytes < (size_t)n * 5 * sizeof(double)) return VECCHIA_EWORKSPACE;
    double *vals = (double *)ws;
    hipStream_t s = (hipStream_t)stream;
    const bool grad = with_grad != 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return VECCHIA_EHIP;
    int32_t chosen = 0;
    double chosen_us = 0.0;
    int rc = VECCHIA_OK;
    for (int32_t v = V_UNBLOCKED; v <= V_TILE_W8 && rc == VECCHIA_OK; ++v) {
        double t_us = -1.0;
        if (variant_feasible(v, m)) {
            EvalArgs a{};
            a.k.locs = field->locs;
            a.k.z = field->z;
            a.k.nbr = field->nbr;
            a.k.n = n;
            a.k.m = m;
            a.k.theta = theta;
            a.k.ell = vals;
            a.k.ell_stride = 4;
            a.k.g = vals + 1;
            a.k.g_stride = 4;
            a.k.flags = (int32_t *)(vals + 4 * n);
            a.t_begin = t_begin;
            a.t_end = n;
            a.m_max = m;
            rc = launch_any(nu_code(nu), grad, v, a, s);  // warm-up
            double best_ms = 1e300;
            for (int32_t r = 0; r < reps && rc == VECCHIA_OK; ++r) {
                (void)hipEventRecord(e0, s);
                rc = launch_any(nu_code(nu), grad, v, a, s);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) rc = VECCHIA_EHIP;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                best_ms = std::min(best_ms, (double)ms);
            }
            if (rc == VECCHIA_OK) {
                t_us = best_ms * 1e3 / (double)(n - t_begin);
                if (chosen == 0 || t_us < chosen_us) {
                    chosen = v;
                    chosen_us = t_us;
                }
            }
        }
        if (us_per_point) us_per_point[v] = t_us;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != VECCHIA_OK) return rc;
    if (us_per_point) us_per_point[0] = chosen_us;
    g_variant[grad ? 1 : 0][m] = chosen;
    *best = chosen;
    return VECCHIA_OK;
}

}  // extern "C"

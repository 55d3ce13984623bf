// Batched evaluation: many parameter vectors and many fields of uneven n and
// m in one enqueue (or one graph launch), and the autotuner that picks the
// kernel variant per conditioning-set size.
//
// A plan (host memory only) groups the fields by tile class
// T = ceil((m+2)/16).  Items of a class are (field, theta, point) triples;
// one launch per class evaluates all of them with the class's variant, one
// workgroup per item, last points first (their conditioning sets are the
// full ones), so the short sets of the first points fill the tail.  Where the
// variant has a lockstep form and ntheta is a multiple of its group size G,
// one workgroup takes G consecutive items instead: one point, G parameter
// vectors (same arithmetic per vector, so the same bits).  The
// classes run one after the other on the caller's stream.  A segmented reduction then forms every evaluation (field, theta)
// with the same fixed-order sum as the single-evaluation entry points, so a
// batched result is bitwise equal to the single call with the same variant.
//
// The device table the kernels read (fields, per-class field lists and item
// offsets) lives at the front of the caller's workspace.  Each call writes it
// there with small kernels that carry the bytes in their arguments, so the
// library allocates no device memory, creates no streams and issues no host
// copies: a call is only kernel launches, which graph capture records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <vector>

#include "launch.h"
#include "reduce.h"
#include "vecchia.h"

using namespace vecchia;

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

std::atomic<bool> g_lockstep{true};  // plans use lockstep forms where they exist

constexpr int kPutWords = 256;  // 8-byte words of table one writing launch carries (2 KB of kernel arguments)

struct PutChunk {
    uint64_t word0;  // first destination word
    uint32_t nwords;
    uint32_t pad;
    uint64_t w[kPutWords];
};

// Copies a chunk of the host-built table from the kernel arguments to the workspace.
__global__ void __launch_bounds__(kPutWords) put_words_kernel(uint64_t *__restrict__ dst, const PutChunk c) {
    const uint32_t t = threadIdx.x;
    if (t < c.nwords) dst[c.word0 + t] = c.w[t];
}

struct ClassPlan {
    int T = 0;
    int variant = 0;
    int group = 1;               // parameter vectors per workgroup (lockstep form when > 1)
    int32_t m_max = 0;
    std::vector<int32_t> fidx;   // fields of the class, larger m first
    std::vector<int64_t> item0;  // prefix sums of ntheta * n over fidx (size nfc + 1)
    size_t off_fidx = 0, off_item0 = 0;
};

// Last field whose first reduce block is <= b: the field owning block b
// (fields without points own no block and share their successor's pb0).
__device__ __forceinline__ int field_of_block(const FieldDev *__restrict__ fields, int nf, int64_t b) {
    int lo = 0, hi = nf;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (fields[mid].pb0 <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kReduceThreads) batched_reduce_kernel(const double *__restrict__ vals,
                                                                        const int32_t *__restrict__ flags,
                                                                        const FieldDev *__restrict__ fields,
                                                                        int32_t nf, double *__restrict__ partial,
                                                                        int64_t *__restrict__ pfail) {
    const int64_t b = blockIdx.x;
    const FieldDev F = fields[field_of_block(fields, nf, b)];
    const int64_t q = (b - F.pb0) / F.nb;
    const int64_t v0 = F.vals0 + q * F.n;
    reduce_segment_block(vals + 4 * v0, flags + v0, F.n, b - F.pb0 - q * F.nb, partial + 8 * b, pfail + b);
}

__global__ void __launch_bounds__(kFinalizeThreads) batched_finalize_kernel(const double *__restrict__ partial,
                                                                            const int64_t *__restrict__ pfail,
                                                                            const FieldDev *__restrict__ fields,
                                                                            int32_t ntheta,
                                                                            const double *__restrict__ thetas,
                                                                            double *__restrict__ out,
                                                                            double *__restrict__ grad,
                                                                            int64_t *__restrict__ status) {
    const int64_t e = blockIdx.x;
    const FieldDev F = fields[e / ntheta];
    const int64_t q = e % ntheta;
    const int64_t p0 = F.pb0 + q * F.nb;
    finalize_segment(partial + 8 * p0, pfail + p0, F.nb, thetas + 3 * e, out + e, grad ? grad + 3 * e : nullptr,
                     status + e);
}

}  // namespace

struct vecchia_plan {
    int32_t nf = 0, ntheta = 0;
    int nuc = 0;         // covariance code (launch_any)
    double alpha = 1.0;  // power-exponential exponent
    bool grad = false;
    std::vector<FieldDev> fields;
    std::vector<ClassPlan> classes;
    int64_t total_rows = 0, total_pblocks = 0;
    std::vector<uint64_t> table;  // host image of the device table (fields, class lists), 8-byte words
    size_t ws_vals = 0, ws_flags = 0, ws_partial = 0, ws_pfail = 0, ws_bytes = 0;
};

struct vecchia_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int run_batched(const vecchia_plan *p, const double *thetas, double *out, double *grad, int64_t *status, void *ws,
                size_t ws_bytes, hipStream_t s) {
    if (!p || !thetas || !out || !status || (p->grad && !grad)) return VECCHIA_EINVAL;
    if (!ws || ws_bytes < p->ws_bytes) return VECCHIA_EWORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return VECCHIA_EINVAL;
    char *w = (char *)ws;
    uint64_t *table = (uint64_t *)w;
    double *vals = (double *)(w + p->ws_vals);
    int32_t *flags = (int32_t *)(w + p->ws_flags);
    double *partial = (double *)(w + p->ws_partial);
    int64_t *pfail = (int64_t *)(w + p->ws_pfail);
    const FieldDev *dfields = (const FieldDev *)w;  // the field array opens the table

    // 1. the device table, from the kernel arguments of a few small launches
    for (size_t w0 = 0; w0 < p->table.size(); w0 += kPutWords) {
        PutChunk c;
        c.word0 = w0;
        c.nwords = (uint32_t)std::min<size_t>(kPutWords, p->table.size() - w0);
        c.pad = 0;
        std::copy(p->table.begin() + w0, p->table.begin() + w0 + c.nwords, c.w);
        hipLaunchKernelGGL(put_words_kernel, dim3(1), dim3(kPutWords), 0, s, table, c);
    }
    const int nc = (int)p->classes.size();
    // 2. one launch per tile class
    for (int c = 0; c < nc; ++c) {
        const ClassPlan &C = p->classes[c];
        EvalArgs a{};
        a.k.ell = vals;
        a.k.ell_stride = 4;
        a.k.g = vals + 1;
        a.k.g_stride = 4;
        a.k.flags = flags;
        a.k.alpha = p->alpha;
        if (C.fidx.size() == 1 && p->ntheta == 1 && C.group == 1) {
            // one field and one vector: nothing to batch, the single-field
            // launch (rows offset by the field's)
            const FieldDev &F = p->fields[C.fidx[0]];
            a.k.locs = F.locs;
            a.k.z = F.z;
            a.k.nbr = F.nbr;
            a.k.n = F.n;
            a.k.m = (int32_t)F.m;
            a.k.theta = thetas + 3 * F.eval0;
            a.k.row0 = -F.vals0;
            a.t_begin = 0;
            a.t_end = F.n;
        } else {
            a.k.theta = thetas;
            a.k.fields = dfields;
            a.k.fidx = (const int32_t *)(w + C.off_fidx);
            a.k.item0 = (const int64_t *)(w + C.off_item0);
            a.k.nfc = (int32_t)C.fidx.size();
            a.k.ntheta = p->ntheta;
            a.t_begin = 0;
            a.t_end = C.item0.back();
        }
        a.m_max = C.m_max;
        a.group = C.group;
        const int rc = launch_any(p->nuc, p->grad, C.variant, a, s);
        if (rc != VECCHIA_OK) return rc;
    }
    // 3. fixed-order sums per evaluation
    if (p->total_pblocks > 0)
        hipLaunchKernelGGL(batched_reduce_kernel, dim3((unsigned)p->total_pblocks), dim3(kReduceThreads), 0, s, vals,
                           flags, dfields, p->nf, partial, pfail);
    hipLaunchKernelGGL(batched_finalize_kernel, dim3((unsigned)((int64_t)p->nf * p->ntheta)), dim3(kFinalizeThreads),
                       0, s, partial, pfail, dfields, p->ntheta, thetas, out, p->grad ? grad : nullptr, status);
    return hipGetLastError() == hipSuccess ? VECCHIA_OK : VECCHIA_EHIP;
}

template <class V>
void append_words(std::vector<uint64_t> &table, size_t byte_off, const V *data, size_t count) {
    const size_t bytes = sizeof(V) * count;
    const size_t words = (byte_off + bytes + 7) / 8;
    if (table.size() < words) table.resize(words, 0);
    std::copy((const char *)data, (const char *)data + bytes, (char *)table.data() + byte_off);
}

// Host-side planning: no device memory, no streams, no synchronisation.
int plan_build(const vecchia_field *fields, int32_t nf, int32_t ntheta, const vecchia_cov *cov, int32_t with_grad,
               vecchia_plan **plan) {
    if (!plan) return VECCHIA_EINVAL;
    *plan = nullptr;
    double alpha = 1.0;
    const int kc = cov_code(cov, &alpha);
    if (!fields || nf < 1 || ntheta < 1 || kc < 0) return VECCHIA_EINVAL;
    if (nf > VECCHIA_MAX_FIELDS) return VECCHIA_EUNSUPPORTED;
    if ((int64_t)nf * ntheta > (int64_t)INT32_MAX) return VECCHIA_EUNSUPPORTED;  // one finalize block per evaluation
    for (int32_t f = 0; f < nf; ++f) {
        const vecchia_field &F = fields[f];
        if (F.n < 0 || F.m < 0) return VECCHIA_EINVAL;
        if (F.m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
        if (F.n > 0 && (!F.locs || !F.z)) return VECCHIA_EINVAL;
        if (F.n > 1 && F.m > 0 && !F.nbr) return VECCHIA_EINVAL;
        if (F.n > (int64_t)INT32_MAX * kChunk) return VECCHIA_EUNSUPPORTED;
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
        d.eval0 = (int64_t)f * ntheta;
        d.vals0 = rows;
        d.pb0 = pblocks;
        d.nb = num_reduce_blocks(d.n);
        pblocks += (int64_t)ntheta * d.nb;
        rows += (int64_t)ntheta * d.n;
        p->fields.push_back(d);
    }
    p->total_rows = rows;
    p->total_pblocks = pblocks;
    if (pblocks > (int64_t)INT32_MAX) {
        delete p;
        return VECCHIA_EUNSUPPORTED;
    }
    // tile classes, largest first; within a class, fields by descending m
    for (int T = (VECCHIA_MAX_M + 2 + 15) / 16; T >= 1; --T) {
        ClassPlan C;
        C.T = T;
        for (int32_t f = 0; f < nf; ++f)
            if (tile_rows(fields[f].m) == T && fields[f].n > 0) C.fidx.push_back(f);
        if (C.fidx.empty()) continue;
        std::stable_sort(C.fidx.begin(), C.fidx.end(),
                         [&](int32_t x, int32_t y) { return fields[x].m > fields[y].m; });
        C.item0.push_back(0);
        for (int32_t f : C.fidx) {
            C.item0.push_back(C.item0.back() + (int64_t)ntheta * fields[f].n);
            C.m_max = std::max(C.m_max, fields[f].m);
        }
        C.variant = resolve_variant(C.m_max, p->grad, 0, p->nuc);
        // Several parameter vectors of a point share one workgroup (lockstep)
        // when they divide into groups of four and the class fits the
        // one-wavefront form (up to five tile rows).  That form replaces any
        // tiled variant the table holds for single calls: on 64 vectors at
        // 10^5 points it took 36.1 against 44.7 ms (m = 40), 60.7 against
        // 71.8 ms (m = 60) and 105.2 against 115.7 ms (m = 75) without the
        // gradient, 158.5 against 183.0 ms (m = 75) with it, each against
        // one vector per workgroup of the table's two-wavefront variant.
        const int G1 = lockstep_group(T, 1);
        if (g_lockstep.load() && variant_waves(C.variant) > 0 && G1 > 1 && ntheta % G1 == 0 &&
            variant_feasible(V_TILE_W1, C.m_max)) {
            C.variant = V_TILE_W1;
            C.group = G1;
        }
        p->classes.push_back(C);
    }
    // device table: the field array, then per class its field list and item offsets
    size_t off = align256(sizeof(FieldDev) * p->fields.size());
    for (ClassPlan &C : p->classes) {
        C.off_fidx = off;
        off = align256(off + sizeof(int32_t) * C.fidx.size());
        C.off_item0 = off;
        off = align256(off + sizeof(int64_t) * C.item0.size());
    }
    p->table.assign(off / 8, 0);
    append_words(p->table, 0, p->fields.data(), p->fields.size());
    for (const ClassPlan &C : p->classes) {
        append_words(p->table, C.off_fidx, C.fidx.data(), C.fidx.size());
        append_words(p->table, C.off_item0, C.item0.data(), C.item0.size());
    }
    // workspace layout: table, per-row values and flags, reduce partials
    size_t w = off;
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

}  // namespace

extern "C" {

int vecchia_plan_create(const vecchia_field *fields, int32_t nf, int32_t ntheta, double nu, int32_t with_grad,
                        vecchia_plan **plan) {
    const vecchia_cov cov{VECCHIA_MATERN, VECCHIA_EUCLIDEAN, nu};
    return plan_build(fields, nf, ntheta, &cov, with_grad, plan);
}

int vecchia_plan_create_cov(const vecchia_field *fields, int32_t nf, int32_t ntheta, const vecchia_cov *cov,
                            int32_t with_grad, vecchia_plan **plan) {
    return plan_build(fields, nf, ntheta, cov, with_grad, plan);
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

int vecchia_plan_class_group(const vecchia_plan *plan, int32_t c) {
    if (!plan || c < 0 || c >= (int32_t)plan->classes.size()) return -VECCHIA_EINVAL;
    return plan->classes[c].group;
}

int vecchia_set_lockstep(int32_t enable) { return g_lockstep.exchange(enable != 0) ? 1 : 0; }

int vecchia_plan_destroy(vecchia_plan *plan) {
    if (!plan) return VECCHIA_EINVAL;
    delete plan;
    return VECCHIA_OK;
}

int vecchia_plan_loglik(const vecchia_plan *plan, const double *thetas, double *out, double *grad, int64_t *status,
                        void *ws, size_t ws_bytes, void *stream) {
    return run_batched(plan, thetas, out, grad, status, ws, ws_bytes, (hipStream_t)stream);
}

size_t vecchia_batched_workspace(const vecchia_field *fields, int32_t nf, int32_t ntheta) {
    const vecchia_cov cov{VECCHIA_MATERN, VECCHIA_EUCLIDEAN, 0.5};
    vecchia_plan *p = nullptr;
    if (plan_build(fields, nf, ntheta, &cov, 0, &p) != VECCHIA_OK) return 0;
    const size_t bytes = p->ws_bytes;
    delete p;
    return bytes;
}

int vecchia_loglik_batched(const vecchia_field *fields, int32_t nf, const double *thetas, int32_t ntheta, double nu,
                           int32_t with_grad, double *out, double *grad, int64_t *status, void *ws, size_t ws_bytes,
                           void *stream) {
    const vecchia_cov cov{VECCHIA_MATERN, VECCHIA_EUCLIDEAN, nu};
    vecchia_plan *p = nullptr;
    const int rc = plan_build(fields, nf, ntheta, &cov, with_grad, &p);
    if (rc != VECCHIA_OK) return rc;
    // the launches carry everything they need in their arguments: the host
    // plan can go as soon as they are enqueued
    const int rc2 = run_batched(p, thetas, out, grad, status, ws, ws_bytes, (hipStream_t)stream);
    delete p;
    return rc2;
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

// Maximum-likelihood estimation of (sigma2, beta, tau2) at fixed smoothness,
// for any covariance model: the use the Vecchia log-likelihood is built for
// (Sec. V fits the Matern and power-exponential parameters by maximising it).
// The paper drives a derivative-free NLopt search; here the fused value +
// gradient evaluation feeds a projected limited-memory BFGS in
// log-parameters, phi = log theta, inside bounds.
//
// Host code driving the batched evaluation: every device round trip
// evaluates a set of parameter vectors as the theta columns of one host plan
// (vecchia_plan_loglik, one launch per round trip), reads back their values,
// gradients and statuses in one copy and synchronises once.  A line search
// tries a quasi-Newton step alone first (it is usually accepted as it
// stands); once it backs off, and from the first step of a search without
// curvature information, it evaluates K = trial_steps step lengths (the next
// K halvings) per round trip and takes the longest one that satisfies the
// Armijo condition, the step sequential backtracking would take.  Round
// trips never exceed those of one-at-a-time backtracking.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "vecchia.h"

namespace {

constexpr int kNp = 3;            // sigma2, beta, tau2
constexpr int kMaxHistory = 20;
constexpr int kMaxTrials = 8;     // step lengths per round trip, at most
constexpr size_t kScratch = 2048; // device scratch at the front of ws: thetas, outputs, statuses of one round trip

struct Eval {
    double f;          // -l / n (+inf when the evaluation failed)
    double g[kNp];     // d f / d phi
    double ll;         // l
    double gth[kNp];   // dl / dtheta
    bool ok;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Problem {
    vecchia_plan *plan[kMaxTrials + 1] = {};  // plan[k]: k parameter vectors per launch, made when first needed
    vecchia_field field{};
    vecchia_cov cov{};
    int64_t n;
    char *ws;
    size_t ws_bytes;
    hipStream_t s;
    int evals = 0, trips = 0;

    ~Problem() {
        for (vecchia_plan *p : plan)
            if (p) vecchia_plan_destroy(p);
    }

    // Evaluates the k parameter vectors phi[0..k) (log theta) in one launch and one round trip.
    int eval(const double (*phi)[kNp], int k, Eval *e) {
        double th[kMaxTrials][kNp];
        for (int q = 0; q < k; ++q)
            for (int p = 0; p < kNp; ++p) th[q][p] = std::exp(phi[q][p]);
        double *d_theta = (double *)ws;                     // [k][3]
        double *d_out = d_theta + 3 * kMaxTrials;           // [k]  then grad [k][3]
        double *d_grad = d_out + kMaxTrials;
        int64_t *d_status = (int64_t *)(d_grad + 3 * kMaxTrials);
        if (!plan[k]) {
            const int prc = vecchia_plan_create_cov(&field, 1, k, &cov, 1, &plan[k]);
            if (prc != VECCHIA_OK) return prc;
        }
        if (hipMemcpyAsync(d_theta, th, sizeof(double) * kNp * k, hipMemcpyHostToDevice, s) != hipSuccess)
            return VECCHIA_EHIP;
        const int rc = vecchia_plan_loglik(plan[k], d_theta, d_out, d_grad, d_status, ws + kScratch,
                                           ws_bytes - kScratch, s);
        if (rc != VECCHIA_OK) return rc;
        // outputs, gradients and statuses are contiguous: one copy back
        double host[kMaxTrials * 5];
        if (hipMemcpyAsync(host, d_out, sizeof(double) * kMaxTrials * 5, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return VECCHIA_EHIP;
        ++trips;
        evals += k;
        const double scale = n > 0 ? 1.0 / (double)n : 1.0;
        for (int q = 0; q < k; ++q) {
            int64_t status;
            std::memcpy(&status, &host[4 * kMaxTrials + q], sizeof(status));
            Eval &x = e[q];
            x.ll = host[q];
            x.ok = status == 0 && std::isfinite(x.ll);
            x.f = x.ok ? -x.ll * scale : INFINITY;
            for (int p = 0; p < kNp; ++p) {
                x.gth[p] = host[kMaxTrials + 3 * q + p];
                x.g[p] = -x.gth[p] * th[q][p] * scale;  // chain rule through theta = e^phi
                x.ok = x.ok && std::isfinite(x.g[p]);
            }
            if (!x.ok) x.f = INFINITY;
        }
        return VECCHIA_OK;
    }
};

double dot(const double *a, const double *b) {
    double s = 0;
    for (int p = 0; p < kNp; ++p) s += a[p] * b[p];
    return s;
}

}  // namespace

extern "C" void vecchia_mle_default_options(vecchia_mle_options *opt) {
    if (!opt) return;
    opt->max_iter = 200;
    opt->history = 8;
    opt->gtol = 1e-7;
    opt->ftol = 1e-13;
    opt->lower[0] = 1e-8;
    opt->lower[1] = 1e-8;
    opt->lower[2] = 1e-10;
    opt->upper[0] = 1e8;
    opt->upper[1] = 1e8;
    opt->upper[2] = 1e8;
    opt->trial_steps = 4;
}

extern "C" size_t vecchia_mle_workspace_size(int64_t n, int32_t m) {
    if (n < 0 || m < 0 || m > VECCHIA_MAX_M) return 0;
    // the largest plan: one field with kMaxTrials parameter vectors
    const vecchia_field f{(const double *)16, (const double *)16, (const int32_t *)16, n, m};
    const size_t plan_ws = vecchia_batched_workspace(&f, 1, kMaxTrials);
    return plan_ws ? kScratch + plan_ws : 0;
}

extern "C" int vecchia_mle_cov(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m,
                               const vecchia_cov *cov, const double *theta0, const vecchia_mle_options *options,
                               double *theta, double *loglik, double *grad, int32_t *iterations,
                               int32_t *evaluations, int32_t *round_trips, void *ws, size_t ws_bytes, void *stream) {
    if (!cov || !theta0 || !theta || !locs || !z || (m > 0 && !nbr) || n < 1 || m < 0) return VECCHIA_EINVAL;
    if (m > VECCHIA_MAX_M) return VECCHIA_EUNSUPPORTED;
    vecchia_mle_options opt;
    if (options) {
        opt = *options;
    } else {
        vecchia_mle_default_options(&opt);
    }
    if (opt.max_iter < 0 || opt.history < 1 || opt.history > kMaxHistory || !(opt.gtol >= 0) || !(opt.ftol >= 0) ||
        opt.trial_steps < 1 || opt.trial_steps > kMaxTrials)
        return VECCHIA_EINVAL;
    const int K = opt.trial_steps;
    double lo[kNp], hi[kNp], phi[kNp];
    for (int p = 0; p < kNp; ++p) {
        if (!(opt.lower[p] > 0) || !(opt.upper[p] >= opt.lower[p]) || !std::isfinite(opt.upper[p]) ||
            !(theta0[p] > 0) || !std::isfinite(theta0[p]))
            return VECCHIA_EINVAL;
        lo[p] = std::log(opt.lower[p]);
        hi[p] = std::log(opt.upper[p]);
        phi[p] = std::min(hi[p], std::max(lo[p], std::log(theta0[p])));
    }
    if (!ws || ws_bytes < vecchia_mle_workspace_size(n, m) || ((uintptr_t)ws & 255) != 0) return VECCHIA_EWORKSPACE;
    Problem pb;
    pb.field = vecchia_field{locs, z, nbr, n, m};
    pb.cov = *cov;
    pb.n = n;
    pb.ws = (char *)ws;
    pb.ws_bytes = ws_bytes;
    pb.s = (hipStream_t)stream;

    Eval cur;
    int rc = pb.eval(&phi, 1, &cur);
    if (rc != VECCHIA_OK) return rc;
    if (!cur.ok) return VECCHIA_EINVAL;  // the starting point itself does not evaluate

    // limited-memory BFGS pairs (s, y) in phi
    double S[kMaxHistory][kNp], Y[kMaxHistory][kNp], rho[kMaxHistory];
    int hist = 0, head = 0, iter = 0, small_steps = 0;

    // a variable is held at a bound while the gradient pushes it outward
    auto free_var = [&](int p, const double *g) {
        const double tol = 1e-12 * (1.0 + std::fabs(phi[p]));
        if (phi[p] <= lo[p] + tol && g[p] > 0) return false;
        if (phi[p] >= hi[p] - tol && g[p] < 0) return false;
        return true;
    };
    auto proj_gnorm = [&](const double *g) {
        double m_ = 0;
        for (int p = 0; p < kNp; ++p)
            if (free_var(p, g)) m_ = std::max(m_, std::fabs(g[p]));
        return m_;
    };

    while (iter < opt.max_iter && proj_gnorm(cur.g) > opt.gtol) {
        // search direction: two-loop recursion on the free variables
        double d[kNp], q[kNp], alpha[kMaxHistory];
        bool fr[kNp];
        for (int p = 0; p < kNp; ++p) {
            fr[p] = free_var(p, cur.g);
            q[p] = fr[p] ? cur.g[p] : 0.0;
        }
        for (int t = 0; t < hist; ++t) {
            const int idx = (head - 1 - t + kMaxHistory) % kMaxHistory;
            alpha[t] = rho[idx] * dot(S[idx], q);
            for (int p = 0; p < kNp; ++p) q[p] -= alpha[t] * Y[idx][p];
        }
        double gamma = 1.0;
        if (hist > 0) {
            const int last = (head - 1 + kMaxHistory) % kMaxHistory;
            gamma = dot(S[last], Y[last]) / dot(Y[last], Y[last]);
        }
        for (int p = 0; p < kNp; ++p) q[p] *= gamma;
        for (int t = hist - 1; t >= 0; --t) {
            const int idx = (head - 1 - t + kMaxHistory) % kMaxHistory;
            const double b = rho[idx] * dot(Y[idx], q);
            for (int p = 0; p < kNp; ++p) q[p] += S[idx][p] * (alpha[t] - b);
        }
        for (int p = 0; p < kNp; ++p) d[p] = fr[p] ? -q[p] : 0.0;
        double slope = dot(cur.g, d);
        if (!(slope < 0)) {  // not a descent direction: restart from steepest descent
            hist = 0;
            for (int p = 0; p < kNp; ++p) d[p] = fr[p] ? -cur.g[p] : 0.0;
            slope = dot(cur.g, d);
            if (!(slope < 0)) break;
        }
        // first step without curvature information: at most one unit in phi
        double step = 1.0;
        if (hist == 0) {
            double dmax = 0;
            for (int p = 0; p < kNp; ++p) dmax = std::max(dmax, std::fabs(d[p]));
            if (dmax > 1.0) step = 1.0 / dmax;
        }
        // projected backtracking line search with the Armijo condition: a
        // quasi-Newton step alone first, then the next K halvings of the step
        // per round trip, the longest acceptable one taken
        Eval nxt{};
        double phin[kNp];
        bool accepted = false;
        for (int ls = 0; ls < 40 && !accepted;) {
            const int k = std::min((ls == 0 && hist > 0) ? 1 : K, 40 - ls);
            double cand[kMaxTrials][kNp];
            Eval ev[kMaxTrials];
            double st = step;
            for (int q = 0; q < k; ++q, st *= 0.5)
                for (int p = 0; p < kNp; ++p) cand[q][p] = std::min(hi[p], std::max(lo[p], phi[p] + st * d[p]));
            rc = pb.eval(cand, k, ev);
            if (rc != VECCHIA_OK) return rc;
            for (int q = 0; q < k; ++q) {
                double dphi[kNp];
                for (int p = 0; p < kNp; ++p) dphi[p] = cand[q][p] - phi[p];
                if (ev[q].ok && ev[q].f <= cur.f + 1e-4 * dot(cur.g, dphi)) {
                    std::memcpy(phin, cand[q], sizeof(phin));
                    nxt = ev[q];
                    accepted = true;
                    break;
                }
            }
            step = st;
            ls += k;
        }
        if (!accepted) break;
        double s[kNp], y[kNp];
        for (int p = 0; p < kNp; ++p) {
            s[p] = phin[p] - phi[p];
            y[p] = nxt.g[p] - cur.g[p];
        }
        const double sy = dot(s, y);
        if (sy > 1e-12 * std::sqrt(dot(s, s) * dot(y, y))) {
            std::memcpy(S[head], s, sizeof(s));
            std::memcpy(Y[head], y, sizeof(y));
            rho[head] = 1.0 / sy;
            head = (head + 1) % kMaxHistory;
            hist = std::min(hist + 1, opt.history);
        }
        const double fdrop = cur.f - nxt.f;
        std::memcpy(phi, phin, sizeof(phi));
        cur = nxt;
        ++iter;
        small_steps = (fdrop <= opt.ftol * std::max(1.0, std::fabs(cur.f))) ? small_steps + 1 : 0;
        if (small_steps >= 3) break;
    }
    for (int p = 0; p < kNp; ++p) theta[p] = std::exp(phi[p]);
    if (loglik) *loglik = cur.ll;
    if (grad)
        for (int p = 0; p < kNp; ++p) grad[p] = cur.gth[p];
    if (iterations) *iterations = iter;
    if (evaluations) *evaluations = pb.evals;
    if (round_trips) *round_trips = pb.trips;
    return VECCHIA_OK;
}

extern "C" int vecchia_mle(const double *locs, const double *z, const int32_t *nbr, int64_t n, int32_t m, double nu,
                           const double *theta0, const vecchia_mle_options *options, double *theta, double *loglik,
                           double *grad, int32_t *iterations, int32_t *evaluations, int32_t *round_trips, void *ws,
                           size_t ws_bytes, void *stream) {
    const vecchia_cov cov{VECCHIA_MATERN, VECCHIA_EUCLIDEAN, nu};
    return vecchia_mle_cov(locs, z, nbr, n, m, &cov, theta0, options, theta, loglik, grad, iterations, evaluations,
                           round_trips, ws, ws_bytes, stream);
}

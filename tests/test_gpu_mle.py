"""Maximum-likelihood driver against the same fit done on the oracle.

The reference maximises the oracle's log-likelihood with scipy's L-BFGS-B in
log-parameters under the same bounds; both must reach the same maximum of a
field drawn from a known Matern process.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v():
    import paper_2403_07412_amd as v
    v.library()
    return v


def reference_fit(f, theta0, lower, upper):
    from scipy.optimize import minimize

    n = f.n

    def fun(phi):
        th = np.exp(phi)
        try:
            ell, g = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, th, with_grad=True, threads=16)
        except oracle.OracleError:
            return np.inf, np.zeros(3)
        return -ell / n, -g * th / n

    res = minimize(fun, np.log(theta0), jac=True, method="L-BFGS-B",
                   bounds=list(zip(np.log(lower), np.log(upper))),
                   options={"maxiter": 1000, "ftol": 1e-16, "gtol": 1e-11})
    return np.exp(res.x), -res.fun * n


@pytest.mark.parametrize("nu,truth", [(1.5, (1.0, 0.08, 0.02)), (0.5, (2.0, 0.15, 0.05))])
def test_mle_matches_oracle_fit(v, nu, truth):
    import torch
    rng = np.random.default_rng(500 + int(nu * 10))
    n, m = 1500, 30
    locs = wl.uniform_locations(rng, n)[rng.permutation(n)]
    z = wl.exact_gp_draw(rng, locs, nu, *truth)
    nbr = wl.nearest_previous_neighbours(locs, m)
    f = wl.Field(locs, z, nbr, m, nu, np.atleast_2d(truth))
    theta0 = np.array([0.5, 0.3, 0.2])
    opt = v.mle_default_options()
    lower = np.array(opt.lower[:])
    upper = np.array(opt.upper[:])
    dev = torch.device("cuda:0")
    res = v.vecchia_mle(torch.from_numpy(locs).to(dev), torch.from_numpy(z).to(dev), torch.from_numpy(nbr).to(dev),
                        m, nu, theta0)
    print("gpu fit", res, flush=True)
    th_ref, ll_ref = reference_fit(f, theta0, lower, upper)
    print("oracle fit", th_ref, ll_ref, flush=True)
    # the reported value is the likelihood at the reported estimate
    ll_at = oracle.loglik(locs, z, nbr, m, nu, res["theta"])
    assert abs(res["loglik"] - ll_at) <= 1e-10 * abs(ll_at)
    # the same maximum
    assert res["loglik"] >= ll_ref - 1e-9 * abs(ll_ref)
    np.testing.assert_allclose(res["theta"], th_ref, rtol=2e-3)
    # and a stationary point: the log-parameter gradient is small
    assert np.max(np.abs(res["grad"] * res["theta"])) <= 1e-3


def test_mle_rejects_bad_start(v):
    import torch
    rng = np.random.default_rng(600)
    f = wl.small_field(rng, 200, 10, 0.5, (1.0, 0.1, 0.01))
    dev = torch.device("cuda:0")
    args = (torch.from_numpy(f.locs).to(dev), torch.from_numpy(f.z).to(dev), torch.from_numpy(f.nbr).to(dev), 10, 0.5)
    with pytest.raises(v.VecchiaError):
        v.vecchia_mle(*args, (-1.0, 0.1, 0.01))
    opt = v.mle_default_options()
    opt.history = 0
    with pytest.raises(v.VecchiaError):
        v.vecchia_mle(*args, (1.0, 0.1, 0.01), options=opt)


def test_mle_power_exponential_great_circle_matches_oracle_fit(v):
    """The real-data model of Sec. V-C: power exponential on great-circle distances, alpha fixed."""
    import torch
    from sklearn.metrics.pairwise import haversine_distances
    rng = np.random.default_rng(620)
    n, m, alpha = 1200, 25, 0.9
    locs = np.column_stack([rng.uniform(-95.0, -85.0, n), rng.uniform(30.0, 40.0, n)])
    D = oracle.EARTH_RADIUS_KM * haversine_distances(np.radians(locs[:, ::-1]))
    truth = (1.5, 80.0, 0.05)
    S = truth[0] * np.exp(-D ** alpha / truth[1]) + truth[2] * np.eye(n)
    z = np.linalg.cholesky(S) @ rng.standard_normal(n)
    cov = (oracle.POWEXP, oracle.GREAT_CIRCLE, alpha)
    nbr = oracle.knn_rows(locs, m, metric=oracle.GREAT_CIRCLE)
    theta0 = np.array([0.5, 30.0, 0.2])
    dev = torch.device("cuda:0")
    res = v.vecchia_mle(torch.from_numpy(locs).to(dev), torch.from_numpy(z).to(dev), torch.from_numpy(nbr).to(dev),
                        m, 0.0, theta0, cov=cov)
    print("gpu fit", res, flush=True)
    opt = v.mle_default_options()
    lower, upper = np.array(opt.lower[:]), np.array(opt.upper[:])
    from scipy.optimize import minimize

    def fun(phi):
        th = np.exp(phi)
        try:
            ell, g = oracle.loglik_cov(locs, z, nbr, m, cov, th, with_grad=True, threads=16)
        except oracle.OracleError:
            return np.inf, np.zeros(3)
        return -ell / n, -g * th / n

    ref = minimize(fun, np.log(theta0), jac=True, method="L-BFGS-B", bounds=list(zip(np.log(lower), np.log(upper))),
                   options={"maxiter": 1000, "ftol": 1e-16, "gtol": 1e-11})
    th_ref, ll_ref = np.exp(ref.x), -ref.fun * n
    print("oracle fit", th_ref, ll_ref, flush=True)
    ll_at = oracle.loglik_cov(locs, z, nbr, m, cov, res["theta"])
    assert abs(res["loglik"] - ll_at) <= 1e-10 * abs(ll_at)
    assert res["loglik"] >= ll_ref - 1e-9 * abs(ll_ref)
    np.testing.assert_allclose(res["theta"], th_ref, rtol=2e-3)


def test_batched_line_search_takes_the_same_steps_in_no_more_round_trips(v):
    """Trial step lengths evaluated as theta columns of one batched launch once a line search backs off
    (a quasi-Newton step is tried alone first): the line search accepts the step one-at-a-time
    backtracking accepts (batched evaluations are bitwise equal to single ones), so the fit is bitwise
    the same, in no more device round trips."""
    import time

    import torch
    rng = np.random.default_rng(630)
    n, m, nu = 3000, 30, 1.5
    locs = wl.uniform_locations(rng, n)[rng.permutation(n)]
    z = wl.exact_gp_draw(rng, locs, nu, 1.2, 0.1, 0.03)
    nbr = wl.nearest_previous_neighbours(locs, m)
    dev = torch.device("cuda:0")
    args = (torch.from_numpy(locs).to(dev), torch.from_numpy(z).to(dev), torch.from_numpy(nbr).to(dev), m, nu)
    theta0 = (0.3, 0.5, 0.3)  # far from the truth: the early steps back off
    fits = {}
    for k in (1, 4, 8):
        opt = v.mle_default_options()
        opt.trial_steps = k
        t0 = time.perf_counter()
        fits[k] = v.vecchia_mle(*args, theta0, options=opt)
        fits[k]["seconds"] = time.perf_counter() - t0
        print("trial_steps", k, fits[k], flush=True)
    for k in (4, 8):
        assert np.array_equal(fits[k]["theta"], fits[1]["theta"]), k
        assert fits[k]["loglik"] == fits[1]["loglik"]
        assert fits[k]["iterations"] == fits[1]["iterations"]
        assert fits[k]["round_trips"] <= fits[1]["round_trips"]
        assert fits[k]["evaluations"] >= fits[1]["evaluations"]
    assert fits[1]["round_trips"] == fits[1]["evaluations"]
    # the start is poor enough that some line searches back off
    assert fits[1]["evaluations"] > fits[1]["iterations"] + 1
    opt = v.mle_default_options()
    opt.trial_steps = 9
    with pytest.raises(v.VecchiaError):
        v.vecchia_mle(*args, theta0, options=opt)

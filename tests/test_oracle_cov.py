"""Pins of the oracle's real-data covariance model and of its kriging (Sec. V-C).

Power exponential C(d) = sigma2 exp(-d^alpha / beta) with Euclidean or
great-circle distance (haversine, R = 6371 km, (longitude, latitude) in
degrees).  The pins are independent of the oracle's code: closed-form
distances and covariance values, scikit-learn's haversine distances, the
identity between a Vecchia chain with complete conditioning sets and the
exact joint density (scipy's multivariate normal), central differences for
the gradient, numpy brute-force neighbour sets, and dense kriging with numpy.
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist
from scipy.stats import multivariate_normal
from sklearn.metrics.pairwise import haversine_distances

import oracle

R = oracle.EARTH_RADIUS_KM


def gcd_matrix(a, b):
    """Great-circle distances (km) by scikit-learn; it takes (lat, lon) in radians."""
    return R * haversine_distances(np.radians(a[:, ::-1]), np.radians(b[:, ::-1]))


def lonlat(rng, n, lon=(-95.0, -85.0), lat=(30.0, 40.0)):
    return np.column_stack([rng.uniform(*lon, n), rng.uniform(*lat, n)])


def full_sets(n):
    """Conditioning sets holding every earlier point (m = n - 1)."""
    m = max(n - 1, 1)
    nbr = -np.ones((n, m), dtype=np.int32)
    for i in range(n):
        nbr[i, :i] = np.arange(i)
    return nbr, m


def test_great_circle_closed_forms():
    a = np.array([[0.0, 0.0], [0.0, 0.0], [30.0, 45.0], [-120.0, 10.0], [170.0, -5.0]])
    b = np.array([[1.0, 0.0], [180.0, 0.0], [30.0, -45.0], [-120.0, 10.0], [-170.0, -5.0]])
    d = oracle.distances(a, b, oracle.GREAT_CIRCLE)
    want = [R * np.pi / 180, R * np.pi, R * np.pi / 2, 0.0]
    np.testing.assert_allclose(d[:4], want, rtol=1e-14, atol=0)
    # across the antimeridian: 20 degrees of longitude at latitude -5
    lat = np.radians(5.0)
    np.testing.assert_allclose(d[4], 2 * R * np.arcsin(np.cos(lat) * np.sin(np.radians(10.0))), rtol=1e-13)
    # symmetric
    np.testing.assert_array_equal(oracle.distances(b, a, oracle.GREAT_CIRCLE), d)


def test_great_circle_against_sklearn():
    rng = np.random.default_rng(900)
    a = np.column_stack([rng.uniform(-180, 180, 500), rng.uniform(-89, 89, 500)])
    b = a + rng.normal(0, 0.05, size=a.shape)          # nearby pairs: the case that matters
    c = np.column_stack([rng.uniform(-180, 180, 500), rng.uniform(-89, 89, 500)])
    for x, y in ((a, b), (a, c)):
        got = oracle.distances(x, y, oracle.GREAT_CIRCLE)
        want = np.diag(gcd_matrix(x, y))
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-9)


def test_power_exponential_values():
    d = np.array([0.0, 0.5, 1.0, 2.0, 7.5])
    for alpha, beta in ((1.0, 0.3), (0.5, 2.0), (2.0, 1.7), (1.37, 0.9)):
        c = oracle.cov_values(d, (oracle.POWEXP, 0, alpha), 2.5, beta)
        assert c[0] == 2.5
        # at d = beta^(1/alpha) the exponent is exactly -1
        c1 = oracle.cov_values([beta ** (1 / alpha)], (oracle.POWEXP, 0, alpha), 2.5, beta)
        np.testing.assert_allclose(c1, 2.5 * np.exp(-1.0), rtol=1e-15)
        assert np.all(np.diff(c) < 0)
    # alpha = 1 is the exponential (Matern nu = 1/2) covariance
    c = oracle.cov_values(d, (oracle.POWEXP, 0, 1.0), 1.3, 0.4)
    np.testing.assert_allclose(c, oracle.matern(d, 0.5, 1.3, 0.4), rtol=1e-15)


def test_power_exponential_dbeta_by_differences():
    d = np.array([0.0, 0.1, 0.7, 1.5, 4.0])
    for alpha in (0.6, 1.0, 1.9):
        beta, h = 0.8, 1e-6
        _, db = oracle.cov_values(d, (oracle.POWEXP, 1, alpha), 1.7, beta, with_dbeta=True)
        fd = (oracle.cov_values(d, (oracle.POWEXP, 1, alpha), 1.7, beta + h)
              - oracle.cov_values(d, (oracle.POWEXP, 1, alpha), 1.7, beta - h)) / (2 * h)
        np.testing.assert_allclose(db, fd, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("metric,alpha", [(0, 1.3), (1, 0.8), (1, 1.0)])
def test_full_chain_equals_joint_density(metric, alpha):
    """Eqs. (4)-(5): with every earlier point conditioned on, the chain is the exact joint density."""
    rng = np.random.default_rng(910 + metric)
    n = 60
    if metric == 0:
        locs = rng.uniform(size=(n, 2))
        D = cdist(locs, locs)
        theta = (1.3, 0.2, 1e-3)
    else:
        locs = lonlat(rng, n)
        D = gcd_matrix(locs, locs)
        theta = (1.3, 150.0 ** alpha, 1e-3)
    np.fill_diagonal(D, 0.0)
    S = theta[0] * np.exp(-D ** alpha / theta[1]) + theta[2] * np.eye(n)
    z = np.linalg.cholesky(S) @ rng.standard_normal(n)
    nbr, m = full_sets(n)
    got = oracle.loglik_cov(locs, z, nbr, m, (oracle.POWEXP, metric, alpha), theta)
    want = multivariate_normal(np.zeros(n), S).logpdf(z)
    assert abs(got - want) <= 1e-10 * abs(want)


def test_gradient_by_differences():
    rng = np.random.default_rng(920)
    n, m = 300, 12
    locs = lonlat(rng, n)
    z = rng.standard_normal(n)
    nbr = oracle.knn_rows(locs, m, metric=oracle.GREAT_CIRCLE)
    cov = (oracle.POWEXP, oracle.GREAT_CIRCLE, 0.9)
    theta = np.array([1.1, 60.0, 0.05])
    _, g = oracle.loglik_cov(locs, z, nbr, m, cov, theta, with_grad=True)
    for p in range(3):
        h = 1e-5 * theta[p]
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (oracle.loglik_cov(locs, z, nbr, m, cov, tp) - oracle.loglik_cov(locs, z, nbr, m, cov, tm)) / (2 * h)
        assert abs(g[p] - fd) <= 1e-6 * max(1.0, abs(fd)), (p, g[p], fd)


def brute_sets(key, lim, m):
    """Row of the m smallest keys among the first lim candidates, ties by index."""
    order = np.lexsort((np.arange(lim), key[:lim]))[:min(lim, m)]
    return np.concatenate([order, -np.ones(m - order.size, dtype=np.int64)])


def test_great_circle_sets_against_numpy():
    rng = np.random.default_rng(930)
    n, m = 400, 15
    locs = lonlat(rng, n)
    got = oracle.knn_rows(locs, m, metric=oracle.GREAT_CIRCLE)
    D = gcd_matrix(locs, locs)
    for i in range(n):
        np.testing.assert_array_equal(got[i], brute_sets(D[i], i, m))


def test_query_sets_against_numpy():
    rng = np.random.default_rng(931)
    ref = rng.uniform(size=(700, 2))
    q = rng.uniform(size=(90, 2))
    q[:5] = ref[[3, 50, 200, 650, 699]]     # queries on top of reference points
    for metric, D in ((0, cdist(q, ref, "sqeuclidean")), (1, None)):
        if metric == 1:
            ref_g, q_g = lonlat(rng, 700), lonlat(rng, 90)
            D = gcd_matrix(q_g, ref_g)
            got = oracle.knn_query(ref_g, q_g, 20, metric)
        else:
            got = oracle.knn_query(ref, q, 20, metric)
        for t in range(got.shape[0]):
            np.testing.assert_array_equal(got[t], brute_sets(D[t], D.shape[1], 20))
    # fewer reference points than m: all of them, then -1
    small = oracle.knn_query(ref[:7], q[:3], 10)
    assert (small[:, 7:] == -1).all() and (np.sort(small[:, :7], axis=1) == np.arange(7)).all()


@pytest.mark.parametrize("metric", [0, 1])
def test_kriging_with_all_points_is_dense_kriging(metric):
    rng = np.random.default_rng(940 + metric)
    n, nq = 150, 40
    if metric == 0:
        ref, q = rng.uniform(size=(n, 2)), rng.uniform(size=(nq, 2))
        Drr, Dqr = cdist(ref, ref), cdist(q, ref)
        theta, alpha = (0.9, 0.15, 0.01), 1.5
    else:
        ref, q = lonlat(rng, n), lonlat(rng, nq)
        Drr, Dqr = gcd_matrix(ref, ref), gcd_matrix(q, ref)
        theta, alpha = (0.9, 90.0, 0.01), 0.7
    np.fill_diagonal(Drr, 0.0)
    S = theta[0] * np.exp(-Drr ** alpha / theta[1]) + theta[2] * np.eye(n)
    V = theta[0] * np.exp(-Dqr ** alpha / theta[1])
    zref = np.linalg.cholesky(S) @ rng.standard_normal(n)
    W = np.linalg.solve(S, V.T)
    want_mean = W.T @ zref
    want_var = theta[0] + theta[2] - np.sum(V.T * W, axis=0)
    nbr = np.tile(np.arange(n, dtype=np.int32), (nq, 1))
    mean, var = oracle.predict(ref, zref, q, nbr, n, (oracle.POWEXP, metric, alpha), theta)
    np.testing.assert_allclose(mean, want_mean, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(var, want_var, rtol=1e-9)


def test_kriging_reproduces_the_conditional_terms():
    """The conditional of point i given J_i is the prediction at s_i from the earlier points."""
    rng = np.random.default_rng(950)
    n, m = 200, 10
    locs = lonlat(rng, n)
    z = rng.standard_normal(n)
    cov = (oracle.POWEXP, oracle.GREAT_CIRCLE, 1.2)
    theta = (1.4, 40.0 ** 1.2, 0.02)
    nbr = oracle.knn_rows(locs, m, metric=oracle.GREAT_CIRCLE)
    terms = oracle.terms_cov(locs, z, nbr, m, cov, theta)
    for i in (m, m + 1, 77, n - 1):
        mean, var = oracle.predict(locs[:i], z[:i], locs[i:i + 1], nbr[i:i + 1], m, cov, theta)
        ell = -0.5 * (np.log(2 * np.pi) + np.log(var[0]) + (z[i] - mean[0]) ** 2 / var[0])
        assert abs(ell - terms[i]) <= 1e-12 * max(1.0, abs(terms[i]))


def test_kriging_failure_and_errors():
    ref = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    zref = np.array([1.0, 2.0, 3.0])
    nbr = np.array([[0, 1, 2]], dtype=np.int32)
    # a repeated neighbour with no nugget makes the neighbour block singular (pivot exactly 0): reported
    dup = np.array([[0, 1, 2], [0, 0, 1]], dtype=np.int32)
    q = np.array([[0.5, 0.5], [0.3, 0.2]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.predict(ref, zref, q, dup, 3, (oracle.POWEXP, 0, 1.0), (1.0, 0.5, 0.0))
    assert e.value.code == 2
    mean, var = oracle.predict(ref, zref, q, dup, 3, (oracle.POWEXP, 0, 1.0), (1.0, 0.5, 0.0),
                               raise_on_fail=False)
    assert np.isfinite(mean[0]) and np.isnan(mean[1]) and np.isnan(var[1])
    with pytest.raises(oracle.OracleError):
        oracle.predict(ref, zref, ref[:1], np.array([[0, 1, 3]], dtype=np.int32), 3, (oracle.POWEXP, 0, 1.0),
                       (1.0, 0.5, 0.1))
    with pytest.raises(oracle.OracleError):   # alpha outside (0, 2]
        oracle.cov_values([1.0], (oracle.POWEXP, 0, 2.5), 1.0, 1.0)

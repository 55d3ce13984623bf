"""Pins for the oracle: each test checks it against something other than itself.

Sources of truth: the exact Gaussian log-likelihood, Eq. (1), via LAPACK; the
general Bessel form of the Matern covariance, Eq. (2), via scipy; Table II of
the paper; the chain rule, Eqs. (4)-(5); brute-force conditional densities;
the KL identity, Eq. (9); homogeneity of the covariance in (sigma2, tau2);
finite differences; and 50-digit arithmetic.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.special import gamma, kv

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LOG2PI = math.log(2 * math.pi)


def dense_cov(locs, nu, sigma2, beta, tau2):
    d = np.sqrt(((locs[:, None, :] - locs[None, :, :]) ** 2).sum(-1))
    return wl.matern_bessel(d, nu, sigma2, beta) + tau2 * np.eye(len(locs))


def exact_loglik(locs, z, nu, theta):
    """Eq. (1) with LAPACK: -n/2 log 2 pi - 1/2 log|Sigma| - 1/2 z^T Sigma^{-1} z."""
    S = dense_cov(locs, nu, *theta)
    sign, logdet = np.linalg.slogdet(S)
    assert sign > 0
    return -0.5 * len(z) * LOG2PI - 0.5 * logdet - 0.5 * z @ np.linalg.solve(S, z)


def dbeta_complex_step(d, nu, sigma2, beta, h=1e-30):
    """dC/dbeta of the Bessel form by the complex step (exact to rounding)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    pos = d > 0
    r = d[pos] / (beta + 1j * h)
    val = sigma2 * (2.0 ** (1.0 - nu) / gamma(nu)) * r ** nu * kv(nu, r)
    out[pos] = val.imag / h
    return out


def field(seed, n, m, nu, theta, grid=False):
    return wl.small_field(np.random.default_rng(seed), n, m, nu, theta, grid=grid)


NUS = [0.5, 1.5, 2.5]


# ------------------------------------------------------------------ P8: kernel
@pytest.mark.parametrize("nu", NUS)
def test_closed_forms_equal_bessel_form(nu):
    d = np.concatenate([[0.0], np.geomspace(1e-8, 3.0, 400)])
    for sigma2, beta in [(1.0, 0.1), (1.7, 0.03), (0.6, 0.3)]:
        got, gb = oracle.matern(d, nu, sigma2, beta, with_dbeta=True)
        ref = wl.matern_bessel(d, nu, sigma2, beta)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15 * sigma2)
        refb = dbeta_complex_step(d, nu, sigma2, beta)
        np.testing.assert_allclose(gb, refb, rtol=1e-10, atol=1e-13 * sigma2 / beta)


def test_table2_effective_range_correlation():
    rows = np.loadtxt(os.path.join(GOLDEN, "table2_beta.txt"))
    for eff, nu, printed, read in rows:
        corr = oracle.matern([eff], nu, 1.0, read)[0]
        assert abs(corr * 45.0 - 1.0) < 2e-4, (eff, nu, read, corr)
        if printed != read:
            # the printed duplicate does not give 1/45: it is a typo
            assert abs(oracle.matern([eff], nu, 1.0, printed)[0] * 45.0 - 1.0) > 0.5


def test_table2_rejects_sqrt2nu_scaling():
    # The alternative scaling r = sqrt(2 nu) d / beta does not reproduce Table II.
    rows = np.loadtxt(os.path.join(GOLDEN, "table2_beta.txt"))
    for eff, nu, _, read in rows:
        if nu == 0.5:
            continue
        corr = oracle.matern([math.sqrt(2 * nu) * eff], nu, 1.0, read)[0]
        assert abs(corr * 45.0 - 1.0) > 0.5


# ----------------------------------------------------- P1: empty conditioning
@pytest.mark.parametrize("nu", NUS)
def test_m0_is_independent_normals(nu):
    f = field(11, 500, 0, nu, (1.3, 0.07, 2e-3))
    theta = f.thetas[0]
    got = oracle.loglik(f.locs, f.z, f.nbr, 0, nu, theta)
    ref = stats.norm.logpdf(f.z, 0.0, math.sqrt(theta[0] + theta[2])).sum()
    assert got == pytest.approx(ref, rel=1e-13)
    ell, g = oracle.terms(f.locs, f.z, f.nbr, 0, nu, theta, with_grad=True)
    c = theta[0] + theta[2]
    # d/dc of log N(z; 0, c) is (z^2/c - 1)/(2c), the same for sigma2 and tau2; beta does not enter.
    np.testing.assert_allclose(g[:, 0], (f.z ** 2 / c - 1) / (2 * c), rtol=1e-13)
    np.testing.assert_allclose(g[:, 2], (f.z ** 2 / c - 1) / (2 * c), rtol=1e-13)
    assert np.all(g[:, 1] == 0.0)


# ------------------------------------------- P2: full conditioning is exact
@pytest.mark.parametrize("nu", NUS)
@pytest.mark.parametrize("tau2", [0.0, 1e-3])
def test_full_conditioning_equals_exact_likelihood(nu, tau2):
    n = 90
    theta = (1.2, 0.08, tau2)
    f = field(21 + int(nu * 2), n, n - 1, nu, theta)
    got = oracle.loglik(f.locs, f.z, f.nbr, n - 1, nu, theta)
    ref = exact_loglik(f.locs, f.z, nu, theta)
    assert got == pytest.approx(ref, rel=1e-10, abs=1e-9)


def test_full_conditioning_exact_gp_draw():
    # the small parity workload's recipe (exact GP draw, nu=0.5, tau2=0) at a size LAPACK takes instantly
    rng = np.random.default_rng(5)
    n = 300
    locs = rng.uniform(size=(n, 2))[rng.permutation(n)]
    z = wl.exact_gp_draw(rng, locs, 0.5, 1.0, 0.1)
    nbr = wl.nearest_previous_neighbours(locs, n - 1)
    got = oracle.loglik(locs, z, nbr, n - 1, 0.5, (1.0, 0.1, 0.0))
    ref = exact_loglik(locs, z, 0.5, (1.0, 0.1, 0.0))
    assert got == pytest.approx(ref, rel=1e-10)


# --------------------------------------------------- P3: first block = joint
@pytest.mark.parametrize("nu", NUS)
def test_short_sets_equal_joint_first_block(nu):
    m = 40
    theta = (0.9, 0.12, 5e-4)
    f = field(31, 400, m, nu, theta)
    ell = oracle.terms(f.locs, f.z, f.nbr, m, nu, theta)
    S = dense_cov(f.locs[:m], nu, *theta)
    joint = stats.multivariate_normal(mean=np.zeros(m), cov=S).logpdf(f.z[:m])
    assert ell[:m].sum() == pytest.approx(joint, rel=1e-11)


# ----------------------------------------- P10: brute-force conditionals
@pytest.mark.parametrize("nu", NUS)
def test_brute_force_conditionals_tiny(nu):
    rng = np.random.default_rng(41)
    for n, m in [(12, 3), (10, 9), (12, 5)]:
        theta = (rng.uniform(0.5, 2), rng.uniform(0.05, 0.4), rng.uniform(0, 1e-2))
        f = wl.small_field(rng, n, m, nu, theta)
        ell = oracle.terms(f.locs, f.z, f.nbr, m, nu, theta)
        for i in range(n):
            # brute-force neighbours, O(n^2)
            d = np.sqrt(((f.locs[:i] - f.locs[i]) ** 2).sum(1))
            J = list(np.lexsort((np.arange(i), d))[:min(i, m)])
            assert J == list(f.nbr[i, :len(J)])
            idx = J + [i]
            S = dense_cov(f.locs[idx], nu, *theta)
            lp_joint = stats.multivariate_normal(np.zeros(len(idx)), S).logpdf(f.z[idx])
            lp_cond = lp_joint - (stats.multivariate_normal(np.zeros(len(J)), S[:-1, :-1]).logpdf(f.z[J])
                                  if J else 0.0)
            assert ell[i] == pytest.approx(lp_cond, rel=1e-11, abs=1e-12)


# ---------------------------------------------------- P4: exact gradient
@pytest.mark.parametrize("nu", NUS)
def test_full_conditioning_gradient_equals_exact(nu):
    n = 70
    theta = (1.1, 0.09, 2e-3)
    f = field(51, n, n - 1, nu, theta)
    _, g = oracle.loglik(f.locs, f.z, f.nbr, n - 1, nu, theta, with_grad=True)
    K = dense_cov(f.locs, nu, *theta)
    d = np.sqrt(((f.locs[:, None, :] - f.locs[None, :, :]) ** 2).sum(-1))
    Ks = (K - theta[2] * np.eye(n)) / theta[0]
    Kb = dbeta_complex_step(d, nu, theta[0], theta[1])
    Kt = np.eye(n)
    Kinv = np.linalg.inv(K)
    alpha = Kinv @ f.z
    ref = [0.5 * alpha @ Kp @ alpha - 0.5 * np.trace(Kinv @ Kp) for Kp in (Ks, Kb, Kt)]
    np.testing.assert_allclose(g, ref, rtol=1e-8)


# -------------------------------------------------- P5: homogeneity (Euler)
@pytest.mark.parametrize("nu", NUS)
def test_euler_identity_sigma2_tau2(nu):
    m = 25
    theta = np.array([1.4, 0.06, 3e-3])
    f = field(61, 1500, m, nu, theta)
    l1, g = oracle.loglik(f.locs, f.z, f.nbr, m, nu, theta, with_grad=True)
    l2 = oracle.loglik(f.locs, f.z, f.nbr, m, nu, theta * np.array([2.0, 1.0, 2.0]))
    n = f.n
    # scaling Sigma by 2 keeps every conditional mean and doubles every conditional variance:
    # l(2) = l(1) - n/2 log 2 + 1/4 Q with Q = sum (y_i - mu_i)^2 / c_i
    Q = 4.0 * (l2 - l1 + 0.5 * n * math.log(2.0))
    lhs = theta[0] * g[0] + theta[2] * g[2]
    assert lhs == pytest.approx(-0.5 * n + 0.5 * Q, rel=1e-9)


# -------------------------------------------------- P9: finite differences
@pytest.mark.parametrize("nu", NUS)
def test_gradient_central_differences(nu):
    m = 20
    theta = np.array([1.3, 0.07, 4e-3])
    f = field(71, 600, m, nu, theta)
    _, g = oracle.loglik(f.locs, f.z, f.nbr, m, nu, theta, with_grad=True)
    for p in range(3):
        h = 1e-5 * theta[p]
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd = (oracle.loglik(f.locs, f.z, f.nbr, m, nu, tp) - oracle.loglik(f.locs, f.z, f.nbr, m, nu, tm)) / (2 * h)
        assert g[p] == pytest.approx(fd, rel=1e-5), p


# ------------------------------------------------- P6: KL >= 0, monotone in m
@pytest.mark.parametrize("nu", NUS)
def test_kl_nonnegative_and_monotone_in_m(nu):
    n = 200
    theta = (1.0, 0.1, 1e-3)
    rng = np.random.default_rng(81)
    locs = rng.uniform(size=(n, 2))[rng.permutation(n)]
    zero = np.zeros(n)
    l0 = exact_loglik(locs, zero, nu, theta)
    prev = -np.inf
    for m in [0, 1, 2, 5, 10, 20, 40, 80, n - 1]:
        nbr = wl.nearest_previous_neighbours(locs, m)
        la = oracle.loglik(locs, zero, nbr, m, nu, theta)
        assert la <= l0 + 1e-9 * abs(l0)           # Eq. (9): KL = l0 - la >= 0
        assert la >= prev - 1e-9 * abs(la)          # nested sets: conditional variances shrink
        prev = la
    assert prev == pytest.approx(l0, rel=1e-10)     # m = n-1: KL = 0


# --------------------------------------- P7: order within each set is irrelevant
def test_neighbour_order_invariance():
    m = 30
    theta = (1.0, 0.05, 1e-6)
    f = field(91, 2500, m, 1.5, theta, grid=True)
    rng = np.random.default_rng(0)
    nbr2 = f.nbr.copy()
    for i in range(f.n):
        k = min(i, m)
        nbr2[i, :k] = nbr2[i, rng.permutation(k)]
    a, ga = oracle.loglik(f.locs, f.z, f.nbr, m, 1.5, theta, with_grad=True)
    b, gb = oracle.loglik(f.locs, f.z, nbr2, m, 1.5, theta, with_grad=True)
    assert a == pytest.approx(b, rel=1e-11)
    np.testing.assert_allclose(ga, gb, rtol=1e-8)


# ---------------------------------------------- P11: 50-digit arithmetic
def test_mpmath_conditionals():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    m = 20
    theta = (1.0, 0.05, 1e-6)
    f = field(101, 900, m, 1.5, theta, grid=True)
    idx = np.array([0, 1, 7, 19, 20, 333, 899])
    ell, g = oracle.terms(f.locs, f.z, f.nbr, m, 1.5, theta, idx=idx, with_grad=True)
    s2, beta, tau2 = [mpmath.mpf(x) for x in theta]

    def C(a, b):
        d = mpmath.sqrt((mpmath.mpf(a[0]) - b[0]) ** 2 + (mpmath.mpf(a[1]) - b[1]) ** 2)
        r = d / beta
        return s2 * (1 + r) * mpmath.exp(-r)

    for t, i in enumerate(idx):
        J = [int(j) for j in f.nbr[i, :min(i, m)]]
        pts = [f.locs[j] for j in J]
        si = f.locs[i]
        if J:
            S = mpmath.matrix(len(J), len(J))
            for a in range(len(J)):
                for b in range(len(J)):
                    S[a, b] = C(pts[a], pts[b]) + (tau2 if a == b else 0)
            v = mpmath.matrix([C(p, si) for p in pts])
            y = mpmath.matrix([mpmath.mpf(f.z[j]) for j in J])
            a_ = mpmath.lu_solve(S, v)
            mu = (a_.T * y)[0]
            c = s2 + tau2 - (a_.T * v)[0]
        else:
            mu, c = 0, s2 + tau2
        e = mpmath.mpf(f.z[i]) - mu
        ref = -(mpmath.log(2 * mpmath.pi) + mpmath.log(c) + e * e / c) / 2
        assert ell[t] == pytest.approx(float(ref), rel=1e-9, abs=1e-9)


def test_compensated_sum():
    x = np.array([1e16, 1.0, -1e16, 1.0] * 10)
    assert oracle.compensated_sum(x) == 20.0


def test_failure_reports_first_point():
    # duplicated locations with no nugget give a singular block
    rng = np.random.default_rng(3)
    locs = rng.uniform(size=(50, 2))
    locs[30] = locs[10]
    locs[40] = locs[10]
    z = rng.standard_normal(50)
    nbr = wl.nearest_previous_neighbours(locs, 10)
    with pytest.raises(oracle.OracleError) as e:
        oracle.loglik(locs, z, nbr, 10, 0.5, (1.0, 0.1, 0.0))
    assert e.value.code - 1 in (30, 40)
    ell = oracle.terms(locs, z, nbr, 10, 0.5, (1.0, 0.1, 0.0), raise_on_fail=False)
    assert np.isnan(ell[40]) and np.isfinite(ell[:30]).all()


def test_invalid_arguments():
    rng = np.random.default_rng(4)
    locs = rng.uniform(size=(20, 2))
    z = rng.standard_normal(20)
    nbr = wl.nearest_previous_neighbours(locs, 5)
    for bad_theta in [(0.0, 0.1, 0.0), (1.0, -0.1, 0.0), (1.0, 0.1, -1e-3)]:
        with pytest.raises(oracle.OracleError):
            oracle.loglik(locs, z, nbr, 5, 0.5, bad_theta)
    with pytest.raises(oracle.OracleError):
        oracle.loglik(locs, z, nbr, 5, 1.0, (1.0, 0.1, 0.0))
    bad = nbr.copy()
    bad[7, 0] = 7  # not a previous point
    with pytest.raises(oracle.OracleError):
        oracle.loglik(locs, z, bad, 5, 0.5, (1.0, 0.1, 0.0))


def test_arbitrary_precision_term_agrees_with_the_fp64_oracle():
    """The mpmath evaluation used to adjudicate rounding: equal to the FP64 oracle on well-conditioned
    conditionals, stable when the precision grows, and the more accurate of the two on a near-singular one."""
    import workloads as wl
    rng = np.random.default_rng(1900)
    f = wl.small_field(rng, 400, 12, 1.5, (1.0, 0.05, 1e-2))
    theta = (1.0, 0.05, 1e-2)
    rows = [0, 1, 5, 12, 13, 200, 399]
    fp = oracle.terms(f.locs, f.z, f.nbr, f.m, 1.5, theta, idx=rows)
    for r, t in zip(rows, fp):
        mp50 = oracle.term_mp(f.locs, f.z, f.nbr, f.m, 1.5, theta, r, dps=50)
        assert abs(mp50 - t) <= 1e-12 * max(1.0, abs(t))
        assert oracle.term_mp(f.locs, f.z, f.nbr, f.m, 1.5, theta, r, dps=80) == mp50
    # a conditional made nearly singular (a tiny nugget, smooth kernel, long range): FP64 loses digits,
    # the 50-digit value does not move at 80 digits
    g = wl.small_field(rng, 300, 30, 2.5, (1.0, 0.4, 1e-9))
    th = (1.0, 0.4, 1e-9)
    a = oracle.term_mp(g.locs, g.z, g.nbr, g.m, 2.5, th, 299, dps=50)
    b = oracle.term_mp(g.locs, g.z, g.nbr, g.m, 2.5, th, 299, dps=80)
    assert abs(a - b) <= 1e-14 * abs(b)

"""Pins of the oracle's conditioning sets (Sec. IV-B) and Morton ordering (Sec. IV-A).

The brute-force neighbour oracle is checked against hand-worked cases with
exact ties, against scipy's k-d tree on random points (a library routine of
its own), and against the workload generator's grid search; the Morton
oracle against the quadrant structure of the Z curve.
"""
import numpy as np
import pytest

import oracle
import workloads as wl


def test_hand_worked_rows_with_ties():
    # unit square corners, then its centre: the centre ties all four corners
    locs = np.array([(0, 0), (1, 0), (0, 1), (1, 1), (0.5, 0.5)], dtype=float)
    got = oracle.knn_rows(locs, 3)
    want = np.array([[-1, -1, -1],
                     [0, -1, -1],
                     [0, 1, -1],
                     [1, 2, 0],      # (1,1): (1,0) and (0,1) at distance 1 (index order), (0,0) at sqrt 2
                     [0, 1, 2]])     # four ties at sqrt(1/2): the three lowest indices
    np.testing.assert_array_equal(got, want)


def test_hand_worked_duplicates_and_collinear():
    # points on a line at x = 0, 3, 1, 3, 2 (a duplicate at 3)
    locs = np.array([(0, 0), (3, 0), (1, 0), (3, 0), (2, 0)], dtype=float)
    got = oracle.knn_rows(locs, 2, rows=[3, 4])
    # row 3 (x=3): the earlier x=3 (distance 0), then x=1 (2) ties nothing; x=0 is 3 away
    # row 4 (x=2): x=3 (index 1) and x=1 (index 2) both at 1, x=3 (index 3) also at 1 -> lowest two indices
    np.testing.assert_array_equal(got, [[1, 2], [1, 2]])


def test_matches_kdtree_on_random_points():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(11)
    n, m = 300, 12
    locs = rng.uniform(size=(n, 2))
    got = oracle.knn_rows(locs, m)
    for i in range(1, n):
        k = min(i, m)
        d, idx = cKDTree(locs[:i]).query(locs[i], k=k)
        idx = np.atleast_1d(idx)
        np.testing.assert_array_equal(got[i, :k], idx, err_msg=f"row {i}")
        assert (got[i, k:] == -1).all()
        dd = np.sqrt(((locs[got[i, :k]] - locs[i]) ** 2).sum(1))
        np.testing.assert_allclose(dd, np.atleast_1d(d), rtol=1e-14)


def test_matches_grid_search_of_the_workload_generator():
    rng = np.random.default_rng(12)
    locs = wl.jittered_grid_locations(rng, 4096)[rng.permutation(4096)]
    for m in (1, 7, 40):
        np.testing.assert_array_equal(oracle.knn_rows(locs, m), wl.nearest_previous_neighbours(locs, m))


def test_row_selection_and_errors():
    rng = np.random.default_rng(13)
    locs = rng.uniform(size=(50, 2))
    full = oracle.knn_rows(locs, 5)
    np.testing.assert_array_equal(oracle.knn_rows(locs, 5, rows=[49, 0, 17]), full[[49, 0, 17]])
    assert oracle.knn_rows(locs, 0).shape == (50, 0)
    with pytest.raises(oracle.OracleError):
        oracle.knn_rows(locs, 5, rows=[50])


def _quadrant_blocks(codes_order, locs, lo, hi, depth):
    """Points of a square visited in Z order: lower-left, lower-right, upper-left, upper-right."""
    if depth == 0 or len(codes_order) < 2:
        return
    mid = (lo + hi) / 2
    q = (locs[codes_order, 0] >= mid[0]).astype(int) + 2 * (locs[codes_order, 1] >= mid[1]).astype(int)
    assert (np.diff(q) >= 0).all(), "quadrants out of Z order"
    for quad in range(4):
        sel = codes_order[q == quad]
        nlo = lo + np.array([quad % 2, quad // 2]) * (mid - lo)
        _quadrant_blocks(sel, locs, nlo, nlo + (mid - lo), depth - 1)


def test_morton_follows_the_z_curve():
    rng = np.random.default_rng(14)
    # points strictly inside cells of a 16 x 16 grid over [0, 1]^2 with both corners present
    locs = (rng.integers(0, 16, size=(3000, 2)) + rng.uniform(0.1, 0.9, size=(3000, 2))) / 16
    locs = np.vstack([[0.0, 0.0], locs, [1.0, 1.0]])
    perm = oracle.morton_order(locs)
    assert sorted(perm) == list(range(len(locs)))
    _quadrant_blocks(perm, locs, np.array([0.0, 0.0]), np.array([1.0, 1.0]), 4)


def test_morton_corners_and_ties():
    locs = np.array([(1, 1), (0, 0), (1, 0), (0, 1), (0, 0)], dtype=float)
    # codes: (0,0) -> 0 twice (indices 1 and 4), (1,0) -> x bits, (0,1) -> y bits, (1,1) -> all bits
    np.testing.assert_array_equal(oracle.morton_order(locs), [1, 4, 2, 3, 0])
    # a zero extent maps every coordinate to cell 0
    flat = np.array([(0.3, 5.0), (0.1, 5.0), (0.2, 5.0)])
    np.testing.assert_array_equal(oracle.morton_order(flat), [1, 2, 0])


# ---- exact likelihood and the KL divergence of Eq. (9) ----------------------

def test_exact_loglik_matches_lapack_on_a_bessel_covariance():
    """Independent covariance (scipy's Bessel K form of Eq. (2)) and LAPACK's factorisation."""
    rng = np.random.default_rng(15)
    n = 300
    locs = rng.uniform(size=(n, 2))
    for nu, theta in ((0.5, (1.3, 0.1, 0.01)), (1.5, (0.7, 0.05, 1e-3)), (2.5, (2.0, 0.08, 0.05))):
        d = np.sqrt(((locs[:, None, :] - locs[None, :, :]) ** 2).sum(-1))
        cov = wl.matern_bessel(d, nu, theta[0], theta[1]) + theta[2] * np.eye(n)
        sign, logdet = np.linalg.slogdet(cov)
        z = rng.standard_normal(n)
        want = -0.5 * (n * np.log(2 * np.pi) + logdet + z @ np.linalg.solve(cov, z))
        want0 = -0.5 * (n * np.log(2 * np.pi) + logdet)
        assert abs(oracle.exact_loglik(locs, z, nu, theta) - want) <= 1e-10 * abs(want)
        assert abs(oracle.exact_loglik(locs, None, nu, theta) - want0) <= 1e-10 * abs(want0)


def test_kl_is_zero_for_full_sets_and_decreases_with_m():
    rng = np.random.default_rng(16)
    n = 400
    locs = rng.uniform(size=(n, 2))
    theta = (1.0, 0.1, 1e-3)
    kls = []
    for m in (1, 5, 15, 40):
        kls.append(oracle.kl_divergence(locs, wl.nearest_previous_neighbours(locs, m), m, 1.5, theta))
    assert all(k > 0 for k in kls)
    assert all(a >= b for a, b in zip(kls, kls[1:]))  # nested nearest-neighbour sets (Eq. (9) >= 0, monotone)
    full = oracle.kl_divergence(locs, wl.nearest_previous_neighbours(locs, n - 1), n - 1, 1.5, theta)
    assert abs(full) <= 1e-9 * n


# ---- approximate maxmin ordering -------------------------------------------------------------
def test_maxmin_hand_worked():
    # box [0, 1]^2: round 0 elects the point nearest (0.5, 0.5); round 1 one point per quadrant (the
    # lower-left quadrant's is the one nearest (0.25, 0.25)); round 2 the rest
    pts = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [0.5, 0.5], [0.26, 0.24]], dtype=float)
    for seed in (0, 7, 2 ** 63 + 5):
        p = oracle.maxmin_order(pts, seed)
        assert p[0] == 4 and set(p[1:5]) == {1, 2, 3, 5} and p[5] == 0


def test_maxmin_rounds_are_seed_independent_and_spread():
    rng = np.random.default_rng(1600)
    x = rng.uniform(size=(2000, 2))
    a, b = oracle.maxmin_order(x, 1), oracle.maxmin_order(x, 2)
    assert sorted(a) == list(range(2000)) and sorted(b) == list(range(2000))
    w = (x.max(0) - x.min(0)).max()      # side of the square box on the lower-left corner
    centre = np.argmin(((x - (x.min(0) + 0.5 * w)) ** 2).sum(1))
    assert a[0] == b[0] == centre
    for level, end in ((1, 5), (2, 21), (3, 85)):
        assert set(a[:end]) == set(b[:end])
        g = 2 ** level
        start = end - g * g
        cells = np.minimum(np.floor((x[a[start:end]] - x.min(0)) / w * g), g - 1)
        assert len({(int(cx), int(cy)) for cx, cy in cells}) == g * g
    # maxmin character: the first points are far more spread than a random subset of the same size
    def min_gap(p):
        d = np.sqrt(((p[:, None, :] - p[None, :, :]) ** 2).sum(-1))
        return d[np.triu_indices(len(p), 1)].min()
    assert min_gap(x[a[:85]]) > 4 * min_gap(x[rng.permutation(2000)[:85]])


def test_maxmin_coincident_points():
    pts = np.full((100, 2), 0.3)
    p = oracle.maxmin_order(pts, 11)
    # lmax = 5 for n = 100: 38 rounds elect one point each (lowest index first), the rest follow by key
    np.testing.assert_array_equal(p[:38], np.arange(38))
    assert sorted(p) == list(range(100))

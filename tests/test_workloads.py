"""The seeded input generators: conditioning sets against brute force, shapes and determinism."""
import numpy as np
import pytest

import workloads as wl


def brute_previous_neighbours(locs, m):
    n = len(locs)
    out = np.full((n, m), -1, dtype=np.int32)
    for i in range(n):
        d = ((locs[:i] - locs[i]) ** 2).sum(1)
        order = np.lexsort((np.arange(i), d))[:m]
        out[i, :len(order)] = order
    return out


@pytest.mark.parametrize("n,m,grid", [(1, 3, False), (7, 10, False), (400, 1, False), (900, 30, True),
                                      (3000, 60, False), (2500, 150, True)])
def test_knn_matches_brute_force(n, m, grid):
    rng = np.random.default_rng(n + m)
    locs = wl.jittered_grid_locations(rng, n) if grid else wl.uniform_locations(rng, n)
    locs = locs[rng.permutation(n)]
    got = wl.nearest_previous_neighbours(locs, m)
    np.testing.assert_array_equal(got, brute_previous_neighbours(locs, m))


def test_knn_sampled_large():
    rng = np.random.default_rng(9)
    n, m = 60000, 120
    locs = wl.uniform_locations(rng, n)
    got = wl.nearest_previous_neighbours(locs, m)
    for i in rng.choice(n, 200, replace=False):
        d = ((locs[:i] - locs[i]) ** 2).sum(1)
        order = np.lexsort((np.arange(i), d))[:m]
        ref = np.full(m, -1, np.int32)
        ref[:len(order)] = order
        np.testing.assert_array_equal(got[i], ref)


def test_knn_thread_count_independent():
    rng = np.random.default_rng(10)
    locs = wl.uniform_locations(rng, 20000)
    a = wl.nearest_previous_neighbours(locs, 40, threads=1)
    b = wl.nearest_previous_neighbours(locs, 40, threads=8)
    np.testing.assert_array_equal(a, b)


def test_small_workload_recipe():
    w = wl.config_small()
    f = w.fields[0]
    assert f.n == 2000 and f.m == 30 and f.nu == 0.5
    assert f.locs.min() >= 0 and f.locs.max() <= 1
    np.testing.assert_array_equal(f.thetas, [[1.0, 0.1, 0.0]])
    assert (f.nbr[0] == -1).all() and (f.nbr[5, :5] >= 0).all() and (f.nbr[5, 5:] == -1).all()
    w2 = wl.config_small()
    np.testing.assert_array_equal(w.fields[0].z, w2.fields[0].z)


def test_jittered_grid():
    rng = np.random.default_rng(1)
    g = wl.jittered_grid_locations(rng, 400)
    cells = np.floor(g * 20).astype(int)
    # every point stays in its own cell (jitter 0.4 of a cell)
    assert len({tuple(c) for c in cells}) == 400


def test_multifield_recipe_sizes():
    rng = np.random.default_rng(wl.SEEDS[5])
    ns = np.rint(np.exp(rng.uniform(np.log(1e4), np.log(5e5), 32)))
    ms = rng.integers(10, 151, 32)
    assert ns.min() >= 1e4 and ns.max() <= 5e5
    assert ms.min() >= 10 and ms.max() <= 150

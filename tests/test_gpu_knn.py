"""GPU conditioning sets and Morton ordering against the oracle (exact, integer results).

Sizes span both search paths of the kernel (the first 8192 rows scan all
earlier points, later rows search grid rings), exact distance ties (integer
lattices, duplicated points), anisotropic extents and the full benchmark
field, where sampled rows are recomputed by brute force.
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


def gpu_knn(v, locs, m):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(locs, dtype=np.float64)).cuda()
    out = v.vecchia_knn(t, m)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,m", [(3000, 1), (3000, 30), (3000, 160), (20000, 30), (20000, 160), (9000, 60)])
def test_uniform_all_rows(v, n, m):
    rng = np.random.default_rng(100 + m + n)
    locs = rng.uniform(size=(n, 2))
    print(f"uniform n={n} m={m}", flush=True)
    np.testing.assert_array_equal(gpu_knn(v, locs, m), oracle.knn_rows(locs, m))


def test_lattice_ties_and_duplicates(v):
    rng = np.random.default_rng(201)
    g = 150
    pts = np.stack(np.meshgrid(np.arange(g), np.arange(g)), -1).reshape(-1, 2).astype(np.float64)
    pts = np.vstack([pts, pts[rng.choice(len(pts), 2000, replace=False)]])  # exact duplicates
    locs = pts[rng.permutation(len(pts))]
    print(f"lattice n={len(locs)}", flush=True)
    for m in (8, 60):
        np.testing.assert_array_equal(gpu_knn(v, locs, m), oracle.knn_rows(locs, m))


def test_thin_strip_and_clusters(v):
    rng = np.random.default_rng(202)
    strip = np.column_stack([rng.uniform(0, 1000, 15000), rng.uniform(0, 1, 15000)])
    centres = rng.uniform(0, 1, size=(20, 2))
    clusters = centres[rng.integers(0, 20, 15000)] + rng.normal(0, 1e-3, size=(15000, 2))
    for name, locs in (("strip", strip), ("clusters", clusters)):
        print(name, flush=True)
        np.testing.assert_array_equal(gpu_knn(v, locs, 40), oracle.knn_rows(locs, 40))


def test_benchmark_field_sampled_rows(v):
    w = wl.config_large(knn_threads=16)
    f = w.fields[0]
    got = gpu_knn(v, f.locs, f.m)
    # the workload generator's sets (CPU grid search) agree everywhere
    np.testing.assert_array_equal(got, f.nbr)
    rng = np.random.default_rng(203)
    rows = np.unique(np.concatenate([np.arange(0, 200), np.arange(8150, 8250), rng.choice(f.n, 600, replace=False)]))
    np.testing.assert_array_equal(got[rows], oracle.knn_rows(f.locs, f.m, rows=rows, threads=16))


def test_edge_cases_and_errors(v):
    import torch
    dev = torch.device("cuda:0")
    one = torch.tensor([[0.5, 0.5]], dtype=torch.float64, device=dev)
    assert (v.vecchia_knn(one, 5).cpu().numpy() == -1).all()
    empty = torch.empty((0, 2), dtype=torch.float64, device=dev)
    assert v.vecchia_knn(empty, 5).shape == (0, 5)
    locs = torch.rand((100, 2), dtype=torch.float64, device=dev)
    assert v.vecchia_knn(locs, 0).shape == (100, 0)
    with pytest.raises(v.VecchiaError):
        v.vecchia_knn(locs, 161)
    # the C ABI rejects a workspace below vecchia_knn_workspace_size (the binding would allocate one)
    import ctypes
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    out = torch.empty((100, 5), dtype=torch.int32, device=dev)
    rc = v.library().vecchia_knn(ctypes.c_void_p(locs.data_ptr()), 100, 5, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(small.data_ptr()), 16, None)
    assert rc == 4  # VECCHIA_EWORKSPACE
    # all points coincide: every earlier point ties at distance 0, lowest indices win
    same = torch.full((50, 2), 0.25, dtype=torch.float64, device=dev)
    got = v.vecchia_knn(same, 4).cpu().numpy()
    want = np.array([[j if j < min(i, 4) else -1 for j in range(4)] for i in range(50)])
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n", [1, 7, 50000])
def test_morton_order(v, n):
    import torch
    rng = np.random.default_rng(300 + n)
    locs = rng.uniform(size=(n, 2))
    if n > 10:
        locs[rng.choice(n, n // 10, replace=False)] = locs[rng.choice(n, n // 10, replace=False)]  # duplicates
    perm = v.vecchia_morton_order(torch.from_numpy(locs).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(perm.cpu().numpy(), oracle.morton_order(locs))


@pytest.mark.parametrize("case", ["uniform3000", "uniform50000", "lattice", "duplicates", "clusters", "one", "seven"])
def test_maxmin_order(v, case):
    import torch
    rng = np.random.default_rng(1700)
    if case.startswith("uniform"):
        locs = rng.uniform(size=(int(case[7:]), 2))
    elif case == "lattice":       # exact distance ties to the cell centres
        g = 64
        locs = np.stack(np.meshgrid(np.arange(g), np.arange(g)), -1).reshape(-1, 2).astype(np.float64)
        locs = locs[rng.permutation(len(locs))]
    elif case == "duplicates":
        locs = np.repeat(rng.uniform(size=(40, 2)), 25, axis=0)[rng.permutation(1000)]
    elif case == "clusters":
        c = rng.uniform(size=(5, 2))
        locs = c[rng.integers(0, 5, 20000)] + rng.normal(0, 1e-4, size=(20000, 2))
    else:
        locs = rng.uniform(size=(1 if case == "one" else 7, 2))
    print(case, len(locs), flush=True)
    for seed in (0, 12345):
        got = v.vecchia_maxmin_order(torch.from_numpy(locs).cuda(), seed=seed)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.maxmin_order(locs, seed))


def test_query_and_maxmin_edge_cases(v):
    import torch
    dev = torch.device("cuda:0")
    q = torch.rand((5, 2), dtype=torch.float64, device=dev)
    empty = torch.empty((0, 2), dtype=torch.float64, device=dev)
    for metric in (0, 1):
        out = v.vecchia_knn_query(empty, q, 7, metric=metric)
        torch.cuda.synchronize()
        assert out.shape == (5, 7) and (out.cpu().numpy() == -1).all()
    assert v.vecchia_knn_query(q, empty, 7).shape == (0, 7)
    # non-finite coordinates still give a permutation (they fall into cell 0)
    rng = np.random.default_rng(1710)
    locs = rng.uniform(size=(500, 2))
    locs[[3, 77, 400]] = np.nan
    got = v.vecchia_maxmin_order(torch.from_numpy(locs).cuda(), seed=5).cpu().numpy()
    assert sorted(got) == list(range(500))
    assert v.vecchia_maxmin_order(empty).shape == (0,)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 5), (1023, 1), (1024, 1), (1025, 2), (300_001, 3), (2_000_000, 99)])
def test_random_order_equals_the_oracle(v, n, seed):
    """vecchia_random_order (device radix sort of 64-bit keys, 8 passes) against the oracle's sort."""
    got = v.vecchia_random_order(n, seed=seed)
    import torch
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.random_order(n, seed))


def test_conditioning_sets_replay_from_a_graph(v):
    """The neighbour search is kernel launches only (device sort and scan): captured once, every replay
    gives the eager sets, with eager work between the replays."""
    import torch
    rng = np.random.default_rng(321)
    n, m = 30_000, 40
    locs = torch.from_numpy(rng.uniform(size=(n, 2))).cuda()
    ws = torch.empty(v.vecchia_knn_workspace_size(n), dtype=torch.uint8, device="cuda")
    out = torch.empty((n, m), dtype=torch.int32, device="cuda")
    want = torch.from_numpy(oracle.knn_rows(locs.cpu().numpy(), m)).cuda()
    v.vecchia_knn(locs, m, out=out, ws=ws)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        v.vecchia_knn(locs, m, out=out, ws=ws)
    for rep in range(3):
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), rep
        junk = torch.randn(5000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk

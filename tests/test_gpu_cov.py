"""Power-exponential and great-circle covariance models, kriging and query
neighbour sets on the GPU, against the oracle (Sec. V-C).

Points for the great-circle cases are (longitude, latitude) degrees over a
10 x 10 degree box (the extent of a regional data set such as the paper's
soil-moisture field); ranges are in km.  Sizes span several 16-row tiles with
ragged last tiles, the unblocked and every tiled kernel variant, prediction
points with fewer observed points than m, and the grid path of the query
search (more than 8192 observed points).
"""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

REL_VALUE = 1e-10
REL_GRAD = 1e-9


@pytest.fixture(scope="module")
def v():
    import paper_2403_07412_amd as v
    v.library()
    return v


def lonlat(rng, n):
    return np.column_stack([rng.uniform(-95.0, -85.0, n), rng.uniform(30.0, 40.0, n)])


# (family, metric, smoothness), theta
CASES = [
    ((1, 0, 0.7), (1.2, 0.08, 1e-3)),
    ((1, 0, 1.0), (0.9, 0.05, 1e-4)),
    ((1, 0, 1.6), (1.5, 0.02, 1e-2)),
    ((1, 0, 2.0), (1.0, 0.004, 1e-2)),
    ((1, 1, 0.8), (1.1, 40.0, 1e-3)),
    ((1, 1, 1.3), (0.8, 600.0, 1e-2)),
    ((0, 1, 0.5), (1.3, 60.0, 1e-4)),
    ((0, 1, 1.5), (1.0, 30.0, 1e-3)),
    ((0, 1, 2.5), (0.7, 25.0, 1e-2)),
]


def field(rng, n, metric):
    locs = lonlat(rng, n) if metric == 1 else rng.uniform(size=(n, 2))
    return locs, rng.standard_normal(n)


@pytest.mark.parametrize("cov,theta", CASES)
@pytest.mark.parametrize("m", [7, 30, 61])
def test_loglik_cov_matches_oracle(v, cov, theta, m):
    import torch
    rng = np.random.default_rng(1000 + 7 * m + int(10 * cov[2]) + 100 * cov[1])
    n = 1500
    locs, z = field(rng, n, cov[1])
    nbr = oracle.knn_rows(locs, m, metric=cov[1], threads=16)
    want, gwant = oracle.loglik_cov(locs, z, nbr, m, cov, theta, with_grad=True, threads=16)
    dev = torch.device("cuda:0")
    L, Z, N = (torch.from_numpy(a).to(dev) for a in (locs, z, nbr))
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    out, grad, st = v.vecchia_loglik_cov(L, Z, N, m, cov, th, with_grad=True)
    val, _, st2 = v.vecchia_loglik_cov(L, Z, N, m, cov, th)
    torch.cuda.synchronize()
    print(cov, m, out.item(), want, grad.cpu().numpy(), gwant, flush=True)
    assert int(st.item()) == 0 and int(st2.item()) == 0
    assert abs(out.item() - want) <= REL_VALUE * abs(want)
    assert abs(val.item() - want) <= REL_VALUE * abs(want)
    np.testing.assert_allclose(grad.cpu().numpy(), gwant, rtol=REL_GRAD, atol=REL_GRAD * np.abs(gwant).max())


@pytest.mark.parametrize("cov,theta", [CASES[0], CASES[5], CASES[8]])
@pytest.mark.parametrize("variant", ["unblocked", "tile_w1", "tile_w2", "tile_w4", "tile_w8"])
def test_terms_every_variant(v, cov, theta, variant):
    import torch
    m = 45
    if not v.vecchia_variant_feasible(m, variant):
        pytest.skip(f"{variant} cannot hold m={m}")
    rng = np.random.default_rng(1100)
    n = 700
    locs, z = field(rng, n, cov[1])
    nbr = oracle.knn_rows(locs, m, metric=cov[1], threads=16)
    want, gwant = oracle.terms_cov(locs, z, nbr, m, cov, theta, with_grad=True, threads=16)
    dev = torch.device("cuda:0")
    L, Z, N = (torch.from_numpy(a).to(dev) for a in (locs, z, nbr))
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    try:
        for g in (False, True):
            v.vecchia_set_variant(m, g, variant)
        t, gt, st = v.vecchia_loglik_terms_cov(L, Z, N, m, cov, th, with_grad=True)
        t0, _, st0 = v.vecchia_loglik_terms_cov(L, Z, N, m, cov, th)
        torch.cuda.synchronize()
    finally:
        for g in (False, True):
            v.vecchia_set_variant(m, g, "auto")
    assert int(st.item()) == 0 and int(st0.item()) == 0
    np.testing.assert_allclose(t.cpu().numpy(), want, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(t0.cpu().numpy(), want, rtol=1e-9, atol=1e-11)
    scale = np.abs(gwant).max(axis=0)
    np.testing.assert_allclose(gt.cpu().numpy(), gwant, rtol=1e-8, atol=1e-9 * scale.max())


def test_matern_euclidean_model_is_the_nu_call(v):
    import torch
    rng = np.random.default_rng(1200)
    f = wl.small_field(rng, 900, 20, 1.5, (1.0, 0.07, 1e-3))
    dev = torch.device("cuda:0")
    L, Z, N = (torch.from_numpy(a).to(dev) for a in (f.locs, f.z, f.nbr))
    th = torch.tensor((1.0, 0.07, 1e-3), dtype=torch.float64, device=dev)
    a, ga, _ = v.vecchia_loglik_grad(L, Z, N, 20, 1.5, th)
    b, gb, _ = v.vecchia_loglik_cov(L, Z, N, 20, (0, 0, 1.5), th, with_grad=True)
    torch.cuda.synchronize()
    assert a.item() == b.item() and torch.equal(ga, gb)


def test_invalid_models_are_rejected(v):
    import torch
    dev = torch.device("cuda:0")
    L = torch.rand((10, 2), dtype=torch.float64, device=dev)
    Z = torch.zeros(10, dtype=torch.float64, device=dev)
    N = torch.full((10, 3), -1, dtype=torch.int32, device=dev)
    th = torch.tensor((1.0, 0.1, 0.0), dtype=torch.float64, device=dev)
    for cov in ((1, 0, 2.5), (1, 0, 0.0), (0, 0, 1.0), (2, 0, 1.0), (0, 2, 0.5)):
        with pytest.raises(v.VecchiaError):
            v.vecchia_loglik_cov(L, Z, N, 3, cov, th)
        with pytest.raises(v.VecchiaError):
            v.vecchia_predict(L, Z, L[:2].contiguous(), N[:2].contiguous(), 3, cov, th)


@pytest.mark.parametrize("cov,theta", [CASES[1], CASES[2], CASES[4], CASES[7]])
@pytest.mark.parametrize("nref,m", [(5, 12), (3000, 12), (3000, 60), (20000, 100)])
def test_kriging_matches_oracle(v, cov, theta, nref, m):
    import torch
    rng = np.random.default_rng(1300 + nref + m)
    ref, z = field(rng, nref, cov[1])
    nq = 777
    q = lonlat(rng, nq) if cov[1] == 1 else rng.uniform(-0.05, 1.05, size=(nq, 2))
    dev = torch.device("cuda:0")
    R, Z, Q = (torch.from_numpy(a).to(dev) for a in (ref, z, q))
    nbr = v.vecchia_knn_query(R, Q, m, metric=cov[1])
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    mean, var, st = v.vecchia_predict(R, Z, Q, nbr, m, cov, th)
    torch.cuda.synchronize()
    nbr_h = nbr.cpu().numpy()
    np.testing.assert_array_equal(nbr_h, oracle.knn_query(ref, q, m, metric=cov[1], threads=16))
    k = min(nref, m)
    assert (nbr_h[:, k:] == -1).all()
    wmean, wvar = oracle.predict(ref, z, q, nbr_h, m, cov, theta, threads=16)
    assert int(st.item()) == 0
    mh, vh = mean.cpu().numpy(), var.cpu().numpy()
    print(cov, nref, m, np.abs(mh - wmean).max(), np.abs(vh / wvar - 1).max(), flush=True)
    np.testing.assert_allclose(mh, wmean, rtol=1e-9, atol=1e-10 * np.abs(z).max())
    np.testing.assert_allclose(vh, wvar, rtol=1e-9)


def test_kriging_edge_cases(v):
    import torch
    dev = torch.device("cuda:0")
    ref = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    zref = np.array([1.0, 2.0, 3.0])
    q = np.array([[0.5, 0.5], [0.3, 0.2], [0.9, 0.9]])
    nbr = np.array([[0, 1, 2], [0, 0, 1], [2, 1, 0]], dtype=np.int32)
    cov, theta = (1, 0, 1.0), (1.0, 0.5, 0.0)
    R, Z, Q, N = (torch.from_numpy(a).to(dev) for a in (ref, zref, q, nbr))
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    mean, var, st = v.vecchia_predict(R, Z, Q, N, 3, cov, th)
    torch.cuda.synchronize()
    # a repeated neighbour without nugget: singular block, reported at position 2
    assert int(st.item()) == 2
    mh, vh = mean.cpu().numpy(), var.cpu().numpy()
    assert np.isnan(mh[1]) and np.isnan(vh[1])
    wm, wv = oracle.predict(ref, zref, q[[0, 2]], nbr[[0, 2]], 3, cov, theta)
    np.testing.assert_allclose(mh[[0, 2]], wm, rtol=1e-12)
    np.testing.assert_allclose(vh[[0, 2]], wv, rtol=1e-12)
    # no observed points: the prior
    empty = torch.empty((0, 2), dtype=torch.float64, device=dev)
    mean, var, st = v.vecchia_predict(empty, torch.empty(0, dtype=torch.float64, device=dev), Q,
                                      torch.full((3, 4), -1, dtype=torch.int32, device=dev), 4, cov, th)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and (mean.cpu().numpy() == 0).all() and (var.cpu().numpy() == 1.0).all()
    # an out-of-range neighbour index is reported, not read
    bad = torch.tensor([[0, 1, 3]], dtype=torch.int32, device=dev)
    mean, var, st = v.vecchia_predict(R, Z, Q[:1].contiguous(), bad, 3, cov, th)
    torch.cuda.synchronize()
    assert int(st.item()) == 1 and np.isnan(mean.item())


@pytest.mark.parametrize("n,m", [(3000, 30), (9000, 60)])
def test_great_circle_sets_match_oracle(v, n, m):
    import torch
    rng = np.random.default_rng(1400 + n)
    locs = lonlat(rng, n)
    got = v.vecchia_knn(torch.from_numpy(locs).cuda(), m, metric=1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.knn_rows(locs, m, metric=1, threads=16))


def test_query_sets_outside_the_box_and_errors(v):
    import torch
    rng = np.random.default_rng(1500)
    ref = rng.uniform(size=(12000, 2))           # grid path
    q = np.vstack([rng.uniform(-0.5, 1.5, size=(400, 2)), ref[:50]])
    dev = torch.device("cuda:0")
    got = v.vecchia_knn_query(torch.from_numpy(ref).to(dev), torch.from_numpy(q).to(dev), 40)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.knn_query(ref, q, 40, threads=16))
    R = torch.from_numpy(ref).to(dev)
    with pytest.raises(v.VecchiaError):
        v.vecchia_knn_query(R, R[:4].contiguous(), 161)
    with pytest.raises(v.VecchiaError):
        v.vecchia_knn_query(R, R[:4].contiguous(), 5, metric=2)
    small = torch.empty(16, dtype=torch.uint8, device=dev)
    out = torch.empty((4, 5), dtype=torch.int32, device=dev)
    rc = v.library().vecchia_knn_query(ctypes.c_void_p(R.data_ptr()), 12000, ctypes.c_void_p(R.data_ptr()), 4, 5, 0,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(small.data_ptr()), 16, None)
    assert rc == 4  # VECCHIA_EWORKSPACE


@pytest.mark.parametrize("region", ["mid", "polar", "antimeridian"])
def test_great_circle_grid_search_matches_oracle(v, region):
    """Beyond 8192 points the great-circle sets come from the grid with the haversine bound; near the
    pole the bound is weak, across the antimeridian (longitude span above 180 degrees) every cell is
    scanned.  Both kinds of sets against brute force."""
    import torch
    rng = np.random.default_rng(1450 + len(region))
    n, nq, m = 30000, 1500, 40
    if region == "mid":
        locs, q = lonlat(rng, n), lonlat(rng, nq)
    elif region == "polar":
        locs = np.column_stack([rng.uniform(-180, 180, n), rng.uniform(80.0, 89.9, n)])
        q = np.column_stack([rng.uniform(-180, 180, nq), rng.uniform(78.0, 89.9, nq)])
    else:
        lon = rng.uniform(170.0, 190.0, n)
        locs = np.column_stack([np.where(lon > 180.0, lon - 360.0, lon), rng.uniform(-5, 5, n)])
        lq = rng.uniform(170.0, 190.0, nq)
        q = np.column_stack([np.where(lq > 180.0, lq - 360.0, lq), rng.uniform(-5, 5, nq)])
    dev = torch.device("cuda:0")
    L, Q = torch.from_numpy(locs).to(dev), torch.from_numpy(q).to(dev)
    got = v.vecchia_knn(L, m, metric=1)
    gq = v.vecchia_knn_query(L, Q, m, metric=1)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([np.arange(8150, 8300), rng.choice(n, 1500, replace=False)]))
    np.testing.assert_array_equal(got.cpu().numpy()[rows], oracle.knn_rows(locs, m, rows=rows, metric=1, threads=16))
    np.testing.assert_array_equal(gq.cpu().numpy(), oracle.knn_query(locs, q, m, metric=1, threads=16))


def test_autograd_under_a_covariance_model(v):
    """loglik(..., cov=...) differentiates through the adjoint kernel for the real-data model."""
    import torch
    rng = np.random.default_rng(1550)
    n, m = 900, 25
    locs, z = field(rng, n, 1)
    nbr = oracle.knn_rows(locs, m, metric=1, threads=16)
    cov, theta = CASES[4]
    dev = torch.device("cuda:0")
    L, Z, N = (torch.from_numpy(a).to(dev) for a in (locs, z, nbr))
    th = torch.tensor(theta, dtype=torch.float64, device=dev, requires_grad=True)
    ell = v.loglik(L, Z, N, th, 0.0, m, cov=cov)
    ell.backward()
    want, gwant = oracle.loglik_cov(locs, z, nbr, m, cov, theta, with_grad=True, threads=16)
    assert abs(ell.item() - want) <= REL_VALUE * abs(want)
    np.testing.assert_allclose(th.grad.cpu().numpy(), gwant, rtol=REL_GRAD, atol=REL_GRAD * np.abs(gwant).max())


@pytest.mark.parametrize("cov", [(1, 1, 0.8), (1, 0, 2.0), (0, 1, 2.5), (0, 1, 1.5)])
def test_batched_plan_under_a_covariance_model(v, cov):
    """Fields of uneven n and m with several parameter vectors (four-vector lockstep workgroups with shared
    distances at m = 10 and 45, one vector per workgroup at m = 70), power exponential and Matern on great-circle or
    Euclidean distances, in one plan and one captured graph: every evaluation bitwise equal to its single
    call."""
    import torch
    rng = np.random.default_rng(1560)
    dev = torch.device("cuda:0")
    fields = []
    for n, m in ((3000, 10), (5000, 45), (2000, 70)):
        locs, z = field(rng, n, cov[1])
        nbr = oracle.knn_rows(locs, m, metric=cov[1], threads=16)
        fields.append(tuple(torch.from_numpy(a).to(dev) for a in (locs, z, nbr)) + (m,))
    scale = 1.0 if cov[1] == 1 else 1e-3  # ranges in km, or in the unit square
    thetas = torch.from_numpy(np.stack([np.column_stack([rng.uniform(0.5, 2, 4), scale * rng.uniform(20, 80, 4),
                                                         rng.uniform(1e-3, 1e-2, 4)]) for _ in fields])).to(dev)
    thetas = thetas.contiguous()
    plan = v.BatchedPlan(fields, 4, 0.0, True, cov=cov)
    print("classes", plan.classes(), "groups", plan.groups(), flush=True)
    assert 4 in plan.groups()
    out, grad, st = plan(thetas)
    g_out, g_grad, g_st = plan.outputs()
    graph = plan.capture(thetas, g_out, g_grad, g_st)
    graph.launch()
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all() and (g_st.cpu().numpy() == 0).all()
    assert torch.equal(out, g_out) and torch.equal(grad, g_grad)
    # single calls with the variant of each field's class (lockstep classes run the one-wavefront one)
    var_of = {T: var for T, var, _, _ in plan.classes()}
    for q, (L, Z, N, m) in enumerate(fields):
        prev = v.vecchia_get_variant(m, True)
        v.vecchia_set_variant(m, True, var_of[(m + 2 + 15) // 16])
        try:
            for p in range(4):
                o, g, s = v.vecchia_loglik_cov(L, Z, N, m, cov, thetas[q, p].contiguous(), with_grad=True)
                torch.cuda.synchronize()
                assert o.item() == out[q, p].item() and torch.equal(g, grad[q, p])
        finally:
            v.vecchia_set_variant(m, True, prev)
    graph.close()
    plan.close()

"""GPU parity: the HIP library (through its C ABI) against the oracle.

Tolerances: the total log-likelihood within relative 1e-10 and its gradient
within relative 1e-9 per component (see util.assert_grad_close for the floor
on components that cancel).  Individual conditional terms are compared to a
looser bound because each carries rounding of order kappa(Sigma_i) * eps.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from util import assert_grad_close, assert_total_close, to_device

pytestmark = pytest.mark.gpu

REL_VALUE = 1e-10
REL_GRAD = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def v():
    import paper_2403_07412_amd as v
    v.library()
    return v


def gpu_total(v, f, with_grad, theta_row=0):
    import torch
    locs, z, nbr, theta = to_device(f, theta_row)
    if with_grad:
        out, g, st = v.vecchia_loglik_grad(locs, z, nbr, f.m, f.nu, theta)
        torch.cuda.synchronize()
        return out.item(), g.cpu().numpy(), int(st.item())
    out, st = v.vecchia_loglik(locs, z, nbr, f.m, f.nu, theta)
    torch.cuda.synchronize()
    return out.item(), None, int(st.item())


def check_field(v, f, with_grad=True, rel=REL_VALUE, relg=REL_GRAD, what=""):
    say(f"case {what}: n={f.n} m={f.m} nu={f.nu} theta={f.thetas[0]} grad={with_grad}")
    th = f.thetas[0]
    got, g, st = gpu_total(v, f, with_grad)
    assert st == 0, f"status {st}"
    if with_grad:
        ell, gt = oracle.terms(f.locs, f.z, f.nbr, f.m, f.nu, th, with_grad=True)
        ref = oracle.compensated_sum(ell)
        gref = [oracle.compensated_sum(gt[:, p]) for p in range(3)]
        assert_total_close(got, ref, rel, what)
        assert_grad_close(g, gref, np.abs(gt).sum(0), relg, what)
    else:
        ref = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, th)
        assert_total_close(got, ref, rel, what)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("m", [0, 1, 10, 30, 60, 64, 65])
def test_parity_small_m(v, nu, m):
    rng = np.random.default_rng(1000 + m)
    f = wl.small_field(rng, 1237, m, nu, (1.3, 0.06, 1e-3))  # 1237 = 77 chunks of 16 + a ragged 5
    check_field(v, f, what=f"small nu={nu} m={m}")


@pytest.mark.parametrize("m", [120, 121, 150, 160])
def test_parity_large_m(v, m):
    rng = np.random.default_rng(2000 + m)
    f = wl.small_field(rng, 700, m, 0.5, (1.5, 0.03, 1e-4))
    check_field(v, f, what=f"large m={m}")


def test_parity_small_workload(v):
    w = wl.config_small()
    check_field(v, w.fields[0], with_grad=True, what="n=2000 m=30 exact draw")


def test_parity_ill_conditioned_grid(v):
    # the jittered-grid recipe (nu=1.5, beta=0.05, tau2=1e-6) at a size the oracle takes in seconds
    w = wl.config_grid(n=40_000)
    check_field(v, w.fields[0], with_grad=True, what="grid n=40000 m=60")


def test_terms_match_oracle(v):
    import torch
    rng = np.random.default_rng(7)
    f = wl.small_field(rng, 3001, 45, 2.5, (0.8, 0.1, 5e-4))
    locs, z, nbr, theta = to_device(f)
    idx = np.sort(rng.choice(f.n, 500, replace=False)).astype(np.int64)
    idx[:3] = [0, 1, 44]  # short conditioning sets
    t, gt, st = v.vecchia_loglik_terms(locs, z, nbr, f.m, f.nu, theta, idx=torch.from_numpy(idx).cuda(),
                                       with_grad=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ell, gref = oracle.terms(f.locs, f.z, f.nbr, f.m, f.nu, f.thetas[0], idx=idx, with_grad=True)
    np.testing.assert_allclose(t.cpu().numpy(), ell, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gt.cpu().numpy(), gref, rtol=1e-7, atol=1e-9 * np.abs(gref).max())


def test_terms_sum_to_total(v):
    import torch
    rng = np.random.default_rng(8)
    f = wl.small_field(rng, 2000, 30, 0.5, (1.0, 0.1, 0.0))
    locs, z, nbr, theta = to_device(f)
    t, gt, st = v.vecchia_loglik_terms(locs, z, nbr, f.m, f.nu, theta, with_grad=True)
    out, g, st2 = v.vecchia_loglik_grad(locs, z, nbr, f.m, f.nu, theta)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(st2.item()) == 0
    assert_total_close(out.item(), math.fsum(t.cpu().numpy()), 1e-13, "terms sum")


def test_deterministic(v):
    import torch
    rng = np.random.default_rng(9)
    f = wl.small_field(rng, 5000, 60, 1.5, (1.0, 0.05, 1e-6), grid=False)
    locs, z, nbr, theta = to_device(f)
    a = v.vecchia_loglik_grad(locs, z, nbr, f.m, f.nu, theta)
    b = v.vecchia_loglik_grad(locs, z, nbr, f.m, f.nu, theta)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


# ----------------------------------------------------------------- edge cases
def test_empty_and_single_point(v):
    import torch
    dev = torch.device("cuda:0")
    theta = torch.tensor([1.0, 0.1, 0.0], dtype=torch.float64, device=dev)
    locs = torch.zeros((0, 2), dtype=torch.float64, device=dev)
    z = torch.zeros(0, dtype=torch.float64, device=dev)
    nbr = torch.zeros((0, 5), dtype=torch.int32, device=dev)
    out, g, st = v.vecchia_loglik_grad(locs, z, nbr, 5, 0.5, theta)
    torch.cuda.synchronize()
    assert out.item() == 0.0 and int(st.item()) == 0 and g.abs().sum().item() == 0.0
    locs = torch.tensor([[0.3, 0.4]], dtype=torch.float64, device=dev)
    z = torch.tensor([0.7], dtype=torch.float64, device=dev)
    nbr = torch.full((1, 5), -1, dtype=torch.int32, device=dev)
    out, st = v.vecchia_loglik(locs, z, nbr, 5, 0.5, theta)
    ref = -0.5 * (math.log(2 * math.pi) + 0.49)
    torch.cuda.synchronize()
    assert out.item() == pytest.approx(ref, rel=1e-15)


def test_m_larger_than_n(v):
    rng = np.random.default_rng(10)
    f = wl.small_field(rng, 50, 100, 1.5, (1.0, 0.2, 1e-3))
    check_field(v, f, what="m > n")


def test_bad_neighbour_index_reports_status(v):
    import torch
    rng = np.random.default_rng(11)
    f = wl.small_field(rng, 300, 10, 0.5, (1.0, 0.1, 0.0))
    f.nbr[200, 3] = 250   # not a previous point
    f.nbr[100, 0] = -7    # negative
    locs, z, nbr, theta = to_device(f)
    out, st = v.vecchia_loglik(locs, z, nbr, f.m, f.nu, theta)
    torch.cuda.synchronize()
    assert int(st.item()) == 101 and math.isnan(out.item())


def test_not_positive_definite_reports_first_point(v):
    import torch
    rng = np.random.default_rng(12)
    f = wl.small_field(rng, 400, 10, 0.5, (1.0, 0.1, 0.0))
    # points 0 and 1 coincide: with sigma2 = 1 and tau2 = 0 the conditional variance of point 1 is
    # 1 - 1*1 = 0 exactly, in any rounding order, so point 1 is the first failure
    f.locs[1] = f.locs[0]
    f.nbr = wl.nearest_previous_neighbours(f.locs, 10)
    locs, z, nbr, theta = to_device(f)
    out, g, st = v.vecchia_loglik_grad(locs, z, nbr, f.m, f.nu, theta)
    torch.cuda.synchronize()
    with pytest.raises(oracle.OracleError) as e:
        oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, f.thetas[0])
    assert e.value.code == 2
    assert int(st.item()) == 2
    assert math.isnan(out.item()) and torch.isnan(g).all()


def test_bad_theta_reports_status(v):
    import torch
    rng = np.random.default_rng(13)
    f = wl.small_field(rng, 100, 5, 0.5, (1.0, 0.1, 0.0))
    locs, z, nbr, _ = to_device(f)
    for bad in [(0.0, 0.1, 0.0), (1.0, -1.0, 0.0), (1.0, 0.1, -1e-9), (float("nan"), 0.1, 0.0)]:
        theta = torch.tensor(bad, dtype=torch.float64, device="cuda:0")
        out, st = v.vecchia_loglik(locs, z, nbr, f.m, f.nu, theta)
        torch.cuda.synchronize()
        assert int(st.item()) == -1 and math.isnan(out.item())


def test_nonfinite_observation_reports_status(v):
    import torch
    rng = np.random.default_rng(14)
    f = wl.small_field(rng, 200, 8, 1.5, (1.0, 0.1, 1e-3))
    f.z[77] = np.nan
    locs, z, nbr, theta = to_device(f)
    out, st = v.vecchia_loglik(locs, z, nbr, f.m, f.nu, theta)
    torch.cuda.synchronize()
    assert int(st.item()) == 78 and math.isnan(out.item())


# ----------------------------------------------------------------- autograd
def test_autograd_matches_adjoint_and_finite_differences(v):
    import torch
    rng = np.random.default_rng(15)
    f = wl.small_field(rng, 3000, 30, 1.5, (1.2, 0.07, 2e-3))
    locs, z, nbr, theta = to_device(f)
    th = theta.clone().requires_grad_(True)
    ell = v.loglik(locs, z, nbr, th, f.nu, f.m)
    ell.backward()
    g_auto = th.grad.cpu().numpy()
    _, gref = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, f.thetas[0], with_grad=True)
    np.testing.assert_allclose(g_auto, gref, rtol=1e-9)
    base = f.thetas[0]
    for p in range(3):
        h = 1e-5 * base[p]
        tp, tm = base.copy(), base.copy()
        tp[p] += h
        tm[p] -= h
        lp = v.loglik(locs, z, nbr, torch.from_numpy(tp).cuda(), f.nu, f.m).item()
        lm = v.loglik(locs, z, nbr, torch.from_numpy(tm).cuda(), f.nu, f.m).item()
        assert g_auto[p] == pytest.approx((lp - lm) / (2 * h), rel=1e-5)

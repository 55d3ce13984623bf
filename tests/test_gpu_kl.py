"""Exact log-likelihood on the GPU and the KL divergence of Eq. (9) against the oracle."""
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


@pytest.mark.parametrize("n,nu,theta", [(1, 0.5, (1.0, 0.1, 0.0)), (50, 1.5, (0.8, 0.2, 1e-4)),
                                        (777, 0.5, (1.5, 0.05, 1e-3)), (1500, 2.5, (1.0, 0.08, 1e-2))])
def test_exact_loglik_matches_oracle(v, n, nu, theta):
    import torch
    rng = np.random.default_rng(700 + n)
    locs = rng.uniform(size=(n, 2))
    z = rng.standard_normal(n)
    dev = torch.device("cuda:0")
    L, Z = torch.from_numpy(locs).to(dev), torch.from_numpy(z).to(dev)
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    for zz, zn in ((Z, z), (None, None)):
        out, st = v.vecchia_exact_loglik(L, zz, nu, th)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        want = oracle.exact_loglik(locs, zn, nu, theta)
        print(n, nu, out.item(), want, flush=True)
        assert abs(out.item() - want) <= 1e-10 * max(1.0, abs(want))


def test_exact_loglik_reports_failure(v):
    import torch
    dev = torch.device("cuda:0")
    locs = torch.tensor([[0.0, 0.0], [0.0, 0.0], [1.0, 1.0]], dtype=torch.float64, device=dev)
    th = torch.tensor([1.0, 0.1, 0.0], dtype=torch.float64, device=dev)   # coincident points, no nugget
    out, st = v.vecchia_exact_loglik(locs, None, 0.5, th)
    torch.cuda.synchronize()
    assert int(st.item()) == 2 and np.isnan(out.item())
    bad = torch.tensor([-1.0, 0.1, 0.0], dtype=torch.float64, device=dev)
    out, st = v.vecchia_exact_loglik(locs, None, 0.5, bad)
    torch.cuda.synchronize()
    assert int(st.item()) == -1


def test_kl_matches_oracle_and_decreases(v):
    import torch
    rng = np.random.default_rng(710)
    n = 2000
    locs = rng.uniform(size=(n, 2))
    theta = (1.0, 0.052537, 1e-4)   # Table II: effective range 0.3 at nu = 1.5
    dev = torch.device("cuda:0")
    L = torch.from_numpy(locs).to(dev)
    th = torch.tensor(theta, dtype=torch.float64, device=dev)
    kls = []
    exact0 = oracle.exact_loglik(locs, None, 1.5, theta)
    for m in (5, 15, 30, 60):
        nbr = wl.nearest_previous_neighbours(locs, m)
        got = v.kl_divergence(L, torch.from_numpy(nbr).to(dev), m, 1.5, th)
        want = exact0 - oracle.loglik(locs, np.zeros(n), nbr, m, 1.5, theta, threads=16)
        print("KL", m, got, want, flush=True)
        # a difference of two totals of size ~n: absolute agreement scaled by the totals
        assert abs(got - want) <= 1e-9 * n
        kls.append(got)
    assert all(k > 0 for k in kls) and all(a > b for a, b in zip(kls, kls[1:]))

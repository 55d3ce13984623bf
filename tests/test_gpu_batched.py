"""Batched evaluation (many fields, many parameter vectors), its graph capture and the autotuner.

The batched form must equal single calls with the same kernel variant bit for
bit (same per-point kernels, same fixed summation order), match the oracle to
the parity tolerances, and give the eager results on every graph replay.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from util import assert_grad_close, assert_total_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v():
    import paper_2403_07412_amd as v
    v.library()
    return v


def make_fields(rng, specs, nu):
    import torch
    out = []
    for n, m in specs:
        f = wl.small_field(rng, n, m, nu, (1.0, 0.1, 0.0))
        dev = torch.device("cuda:0")
        nbr = torch.from_numpy(f.nbr).to(dev) if m > 0 else torch.empty((n, 0), dtype=torch.int32, device=dev)
        out.append((f, (torch.from_numpy(f.locs).to(dev), torch.from_numpy(f.z).to(dev), nbr, m)))
    return out


def random_thetas(rng, nf, ntheta):
    th = np.stack([rng.uniform(0.5, 2.0, (nf, ntheta)), rng.uniform(0.03, 0.2, (nf, ntheta)),
                   rng.uniform(1e-5, 1e-3, (nf, ntheta))], axis=-1)
    return th


SPECS = [(700, 10), (1500, 30), (0, 20), (900, 62), (1, 5), (400, 120), (333, 150), (2000, 47)]


@pytest.mark.parametrize("with_grad", [True, False])
def test_batched_equals_single_calls_bitwise_and_oracle(v, with_grad):
    import torch
    rng = np.random.default_rng(77)
    nu = 1.5
    fields = make_fields(rng, SPECS, nu)
    ntheta = 3
    th = random_thetas(rng, len(SPECS), ntheta)
    thetas = torch.from_numpy(th).cuda()
    plan = v.BatchedPlan([f[1] for f in fields], ntheta, nu, with_grad)
    print("classes", plan.classes(), flush=True)
    out, grad, status = plan(thetas)
    torch.cuda.synchronize()
    assert (status == 0).all()
    class_variant = {T: var for T, var, _, _ in plan.classes()}
    for fi, (f, (locs, z, nbr, m)) in enumerate(fields):
        for q in range(ntheta):
            if f.n == 0:
                assert out[fi, q].item() == 0.0
                continue
            variant = class_variant[(m + 2 + 15) // 16]
            o1, g1, s1 = v.vecchia_loglik_variant(locs, z, nbr if m > 0 else None, m, nu, thetas[fi, q].contiguous(),
                                                  variant, with_grad=with_grad)
            torch.cuda.synchronize()
            assert int(s1.item()) == 0
            assert torch.equal(o1[0], out[fi, q]), (fi, q)
            if with_grad:
                assert torch.equal(g1, grad[fi, q])
            ell, gt = oracle.terms(f.locs, f.z, f.nbr, m, nu, th[fi, q], with_grad=True)
            assert_total_close(out[fi, q].item(), oracle.compensated_sum(ell), 1e-10, f"field {fi} theta {q}")
            if with_grad:
                assert_grad_close(grad[fi, q].cpu().numpy(), [oracle.compensated_sum(gt[:, p]) for p in range(3)],
                                  np.abs(gt).sum(0), 1e-9, f"field {fi} theta {q}")
    plan.close()


def table_as_plan(v, ms, plan, with_grad):
    """Points the variant table at the variant each m's tile class uses in `plan` (lockstep classes take the
    one-wavefront variant); returns the previous entries for restore_table."""
    var_of = {T: var for T, var, _, _ in plan.classes()}
    old = {}
    for m in ms:
        T = (m + 2 + 15) // 16
        if m not in old and T in var_of:
            old[m] = v.vecchia_get_variant(m, with_grad)
            v.vecchia_set_variant(m, with_grad, var_of[T])
    return old


def restore_table(v, old, with_grad):
    for m, var in old.items():
        v.vecchia_set_variant(m, with_grad, var)


LOCKSTEP_SPECS = [(700, 10), (1500, 30), (900, 62), (1, 5), (0, 20), (610, 94), (400, 120), (64, 3), (17, 40),
                  (350, 75)]


@pytest.mark.parametrize("ntheta,nu", [(4, 2.5), (8, 1.5), (12, 0.5)])
@pytest.mark.parametrize("with_grad", [True, False])
def test_lockstep_groups_equal_one_vector_workgroups_bitwise(v, with_grad, ntheta, nu):
    """Several parameter vectors per workgroup (shared gather and pair distances) give the bits of one vector
    per workgroup, for every class shape, with an invalid vector inside a group."""
    import torch
    rng = np.random.default_rng(81 + ntheta)
    fields = make_fields(rng, LOCKSTEP_SPECS, nu)
    th = random_thetas(rng, len(LOCKSTEP_SPECS), ntheta)
    th[2, 1] = [-1.0, 0.1, 0.0]
    thetas = torch.from_numpy(th).cuda()
    prev = v.set_lockstep(True)
    old = {}
    try:
        plan = v.BatchedPlan([f[1] for f in fields], ntheta, nu, with_grad)
        v.set_lockstep(False)
        # one vector per workgroup with the variants the lockstep plan uses
        old = table_as_plan(v, [m for _, m in LOCKSTEP_SPECS], plan, with_grad)
        plan1 = v.BatchedPlan([f[1] for f in fields], ntheta, nu, with_grad)
    finally:
        v.set_lockstep(prev)
        restore_table(v, old, with_grad)
    groups = plan.groups()
    print("classes", plan.classes(), "groups", groups, flush=True)
    assert max(groups) > 1 and all(g == 1 for g in plan1.groups())
    assert [c[1] for c in plan.classes()] == [c[1] for c in plan1.classes()]
    out, grad, status = plan(thetas)
    out1, grad1, status1 = plan1(thetas)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[2, 1] == -1
    st[2, 1] = 0
    assert (st == 0).all()
    assert torch.equal(status, status1)
    assert torch.equal(out.view(torch.int64), out1.view(torch.int64))
    if with_grad:
        assert torch.equal(grad.view(torch.int64), grad1.view(torch.int64))
    # and the oracle, on one vector of a lockstep class
    fi, q = 2, 0
    f = fields[fi][0]
    ell, gt = oracle.terms(f.locs, f.z, f.nbr, f.m, nu, th[fi, q], with_grad=True)
    assert_total_close(out[fi, q].item(), oracle.compensated_sum(ell), 1e-10, "lockstep field 2")
    plan.close()
    plan1.close()


def test_graph_replays_match_eager(v):
    import torch
    rng = np.random.default_rng(78)
    nu = 0.5
    fields = make_fields(rng, [(1200, 30), (800, 90), (500, 14)], nu)
    ntheta = 4
    plan = v.BatchedPlan([f[1] for f in fields], ntheta, nu, True)
    thetas = torch.from_numpy(random_thetas(rng, 3, ntheta)).cuda()
    out, grad, status = plan.outputs()
    graph = plan.capture(thetas, out, grad, status)
    for rep in range(4):
        new = torch.from_numpy(random_thetas(rng, 3, ntheta)).cuda()
        thetas.copy_(new)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        got = (out.clone(), grad.clone(), status.clone())
        # eager work in between replays
        e_out, e_grad, e_status = plan(thetas)
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.equal(got[0], e_out) and torch.equal(got[1], e_grad) and torch.equal(got[2], e_status), rep
        assert (e_status == 0).all()
        del junk
    graph.close()
    plan.close()


def test_batched_reports_failure_per_evaluation(v):
    import torch
    rng = np.random.default_rng(79)
    nu = 0.5
    fields = make_fields(rng, [(300, 10), (300, 10)], nu)
    # second field: points 0 and 1 coincide -> with sigma2 = 1, tau2 = 0 point 1 fails exactly
    f, (locs, z, nbr, m) = fields[1]
    f.locs[1] = f.locs[0]
    f.nbr = wl.nearest_previous_neighbours(f.locs, 10)
    locs.copy_(torch.from_numpy(f.locs))
    nbr.copy_(torch.from_numpy(f.nbr))
    plan = v.BatchedPlan([fl[1] for fl in fields], 2, nu, True)
    th = np.array([[[1.0, 0.1, 0.0], [1.0, 0.1, 1e-2]], [[1.0, 0.1, 0.0], [-1.0, 0.1, 0.0]]])
    out, grad, status = plan(torch.from_numpy(th).cuda())
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[0, 0] == 0 and st[0, 1] == 0
    assert st[1, 0] == 2          # point 1 of field 1
    assert st[1, 1] == -1         # invalid theta
    assert np.isnan(out[1, 0].item()) and np.isnan(out[1, 1].item())
    assert np.isfinite(out[0].cpu().numpy()).all()
    plan.close()


def test_autotune_sets_a_feasible_variant(v):
    import torch
    rng = np.random.default_rng(80)
    f, (locs, z, nbr, m) = make_fields(rng, [(6000, 60)], 1.5)[0]
    theta = torch.tensor([1.0, 0.05, 1e-5], dtype=torch.float64, device="cuda")
    before = v.vecchia_get_variant(60, True)
    best, times = v.vecchia_autotune(locs, z, nbr, 60, 1.5, theta, True, sample=3000, reps=2)
    print("autotune m=60", best, times, flush=True)
    assert v.vecchia_variant_feasible(60, best)
    assert v.vecchia_get_variant(60, True) == best
    assert all(t > 0 for t in times.values())
    assert min(times, key=times.get) == {val: k for k, val in v.VARIANTS.items()}[best]
    v.vecchia_set_variant(60, True, before)


def test_one_call_form_equals_the_plan_bitwise(v):
    """vecchia_loglik_batched (fields in a host array, no plan object) against vecchia_plan_loglik."""
    import torch
    rng = np.random.default_rng(81)
    nu = 2.5
    fields = make_fields(rng, [(900, 60), (0, 8), (1300, 17), (450, 100)], nu)
    ntheta = 5
    thetas = torch.from_numpy(random_thetas(rng, len(fields), ntheta)).cuda()
    plan = v.BatchedPlan([f[1] for f in fields], ntheta, nu, True)
    p_out, p_grad, p_status = plan(thetas)
    assert v.vecchia_batched_workspace([f[1] for f in fields], ntheta) == plan.ws.numel()
    for rep in range(2):  # the second call reuses nothing from the first
        o, g, s = v.vecchia_loglik_batched([f[1] for f in fields], thetas, nu, True)
        torch.cuda.synchronize()
        assert torch.equal(o, p_out) and torch.equal(g, p_grad) and torch.equal(s, p_status), rep
    assert (p_status == 0).all()
    o2, g2, s2 = v.vecchia_loglik_batched([f[1] for f in fields], thetas, nu, False)
    torch.cuda.synchronize()
    assert g2 is None and torch.equal(o2, p_out) and (s2 == 0).all()
    plan.close()


def test_binding_rejects_mistyped_theta_and_outputs(v):
    """A float32 theta or an int32 status would be read or written past its end through the raw pointer."""
    import torch
    rng = np.random.default_rng(82)
    f, (locs, z, nbr, m) = make_fields(rng, [(200, 10)], 0.5)[0]
    good = torch.tensor([1.0, 0.1, 1e-3], dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        v.vecchia_loglik_grad(locs, z, nbr, m, 0.5, good.float())
    with pytest.raises(ValueError):
        v.vecchia_loglik_grad(locs, z, nbr, m, 0.5, torch.ones(2, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        v.vecchia_loglik(locs, z, nbr, m, 0.5, good, status=torch.zeros(1, dtype=torch.int32, device="cuda"))
    with pytest.raises(TypeError):
        v.vecchia_loglik_grad(locs, z, nbr, m, 0.5, good, out=torch.zeros(1, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        v.vecchia_loglik_grad(locs, z, nbr, m, 0.5, good, grad=torch.zeros(2, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        v.loglik(locs, z, nbr, good.float().requires_grad_(True), 0.5, m)
    with pytest.raises(TypeError):
        v.vecchia_predict(locs, z, locs[:5].contiguous(), nbr[:5].contiguous(), m, (v.MATERN, v.EUCLIDEAN, 0.5),
                          good.float())
    plan = v.BatchedPlan([(locs, z, nbr, m)], 2, 0.5, True)
    with pytest.raises(ValueError):
        plan(torch.ones((1, 3, 3), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        o, g, s = plan.outputs()
        plan(torch.ones((1, 2, 3), dtype=torch.float64, device="cuda"), status=s.int())
    plan.close()
    out, st = v.vecchia_loglik(locs, z, nbr, m, 0.5, good)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and np.isfinite(out.item())

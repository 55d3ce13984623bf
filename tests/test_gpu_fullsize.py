"""Parity at the full sizes of the benchmark workloads, in the launch forms the benchmark times.

- n = 10^6, m = 120, nu = 1/2, value + gradient: the per-call tile_w4 kernel and the batched plan
  replayed from a captured graph, both against the oracle's total over all 10^6 conditionals
  (rel 1e-10 value, 1e-9 gradient), bitwise equal to each other, plus sampled per-point terms.
  Sampled terms agree to 1e-9; where an ill-conditioned term does not, a 50-digit evaluation decides
  and the kernel's error must stay within 3 times the FP64 oracle's (assert_adjudicated).
- n = 250,000 jittered grid, m = 60, nu = 3/2, value: the total against the oracle.
- n = 200,000, m = 60, nu = 5/2, 64 parameter vectors with gradients in one batched launch: every
  vector bitwise equal to its own single call, four of them against the oracle's totals.
- 32 fields of uneven n and m in one captured graph: every field bitwise equal to its single call,
  the four smallest against the oracle's totals and sampled terms of every field against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

REL_VALUE = 1e-10
REL_GRAD = 1e-9
THREADS = 16


@pytest.fixture(scope="module")
def v():
    import paper_2403_07412_amd as v
    v.library()
    return v


def dev_field(f):
    import torch
    d = torch.device("cuda:0")
    return (torch.from_numpy(f.locs).to(d), torch.from_numpy(f.z).to(d), torch.from_numpy(f.nbr).to(d))


def assert_total(got, want, g=None, gwant=None):
    assert abs(got - want) <= REL_VALUE * abs(want), (got, want)
    if g is not None:
        np.testing.assert_allclose(g, gwant, rtol=REL_GRAD, atol=1e-12 * np.abs(gwant).max())


def sample_rows(rng, n, m, count):
    rows = np.concatenate([np.arange(min(n, m + 2)), rng.choice(n, min(n, count), replace=False), [n - 1]])
    return np.unique(rows).astype(np.int64)


def check_terms(v, f, theta, L, Z, N, rows, with_grad):
    import torch
    idx = torch.from_numpy(rows).cuda()
    th = torch.tensor(theta, dtype=torch.float64, device="cuda")
    t, gt, st = v.vecchia_loglik_terms(L, Z, N, f.m, f.nu, th, idx=idx, with_grad=with_grad)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    if with_grad:
        want, gwant = oracle.terms(f.locs, f.z, f.nbr, f.m, f.nu, theta, idx=rows, with_grad=True, threads=THREADS)
        np.testing.assert_allclose(gt.cpu().numpy(), gwant, rtol=1e-8, atol=1e-9 * np.abs(gwant).max())
    else:
        want = oracle.terms(f.locs, f.z, f.nbr, f.m, f.nu, theta, idx=rows, threads=THREADS)
    got = t.cpu().numpy()
    rel = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    print(f"{rows.size} sampled terms: max rel difference to the oracle {rel.max():.2e}", flush=True)
    off = np.argsort(rel)[::-1][:40]
    off = off[rel[off] > 1e-9]
    if not off.size:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    # ill-conditioned conditionals: two FP64 evaluations may differ by about kappa * u, so the 50-digit
    # value decides (assert_adjudicated)
    exact = np.array([oracle.term_mp(f.locs, f.z, f.nbr, f.m, f.nu, theta, int(rows[q])) for q in off])
    print(f"{off.size} terms beyond 1e-9 (max {rel.max():.2e})", flush=True)
    return got[off] - exact, want[off] - exact, exact


def assert_adjudicated(parts):
    """Errors against the 50-digit values, pooled over every term that two FP64 evaluations disagreed
    on.  Every triangular solve of the kernels is a substitution, as in the oracle; the two remain
    different backward-stable orderings (blocked right-looking with 4-term matrix-core partial sums
    against row-by-row dot products), whose errors on a handful of terms differ by small factors
    either way.  The pooled root-mean-square error may be 3 times the oracle's (measured: 2.3 on the
    11 adjudicated terms of the 32 fields; the dedicated ill-conditioned test, test_gpu_accuracy.py,
    holds the kernels to 1.5 on its 24 worst terms).  The tiled kernels once multiplied by explicit
    inverses of their 16 x 16 diagonal tiles and were 3-4 times less accurate than the oracle on blocks
    with kappa near 1e7 while the grid workload alone adjudicated 40 terms; with substitution its
    1500 sampled terms all agree with the oracle to 1e-9."""
    e_gpu = np.concatenate([p[0] for p in parts])
    e_orc = np.concatenate([p[1] for p in parts])
    exact = np.concatenate([p[2] for p in parts])
    if not e_gpu.size:
        return
    rg, ro = np.sqrt(np.mean(e_gpu ** 2)), np.sqrt(np.mean(e_orc ** 2))
    print(f"adjudicated {e_gpu.size} terms: rms error vs 50 digits kernel {rg:.3e}, oracle {ro:.3e}", flush=True)
    for a, b, c in zip(e_gpu, e_orc, exact):
        print(f"  term {c:.16e}: kernel error {a:.2e}, oracle error {b:.2e}", flush=True)
    assert rg <= 3.0 * ro + 1e-13 * np.sqrt(np.mean(exact ** 2))
    assert np.max(np.abs(e_gpu) / np.maximum(1.0, np.abs(exact))) <= 1e-6


def test_n1M_m120_value_and_gradient(v):
    import torch
    f = wl.config_large(knn_threads=THREADS).fields[0]
    theta = f.thetas[0]
    print("oracle over 10^6 conditionals", flush=True)
    want, gwant = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, theta, with_grad=True, threads=THREADS)
    L, Z, N = dev_field(f)
    th = torch.tensor(theta, dtype=torch.float64, device="cuda")
    out, grad, st = v.vecchia_loglik_variant(L, Z, N, f.m, f.nu, th, "tile_w4", with_grad=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    print("plain", out.item(), grad.cpu().numpy(), "oracle", want, gwant, flush=True)
    assert_total(out.item(), want, grad.cpu().numpy(), gwant)
    # the batched plan replayed from a captured graph, as the benchmark times it
    plan = v.BatchedPlan([(L, Z, N, f.m)], 1, f.nu, True)
    thetas = th.reshape(1, 1, 3).contiguous()
    b_out, b_grad, b_st = plan.outputs()
    graph = plan.capture(thetas, b_out, b_grad, b_st)
    for _ in range(3):
        b_out.fill_(0.0)
        graph.launch()
        torch.cuda.synchronize()
        assert int(b_st.reshape(-1)[0].item()) == 0
        assert b_out.reshape(-1)[0].item() == out.item()
        assert torch.equal(b_grad.reshape(3), grad)
    graph.close()
    plan.close()
    assert_adjudicated([check_terms(v, f, theta, L, Z, N, sample_rows(np.random.default_rng(1800), f.n, f.m, 1500),
                                    True)])


def test_n250k_grid_m60_value(v):
    import torch
    f = wl.config_grid(knn_threads=THREADS).fields[0]
    theta = f.thetas[0]
    want = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, theta, threads=THREADS)
    L, Z, N = dev_field(f)
    out, st = v.vecchia_loglik(L, Z, N, f.m, f.nu, torch.tensor(theta, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    print("grid", out.item(), want, flush=True)
    assert_total(out.item(), want)
    assert_adjudicated([check_terms(v, f, theta, L, Z, N, sample_rows(np.random.default_rng(1810), f.n, f.m, 1500),
                                    False)])


def test_n200k_64_thetas_batched(v):
    import torch
    f = wl.config_multitheta(knn_threads=THREADS).fields[0]
    L, Z, N = dev_field(f)
    thetas = torch.from_numpy(f.thetas).cuda().reshape(1, -1, 3).contiguous()
    plan = v.BatchedPlan([(L, Z, N, f.m)], thetas.shape[1], f.nu, True)
    out, grad, st = plan(thetas)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for p in range(thetas.shape[1]):
        o, g, s = v.vecchia_loglik_grad(L, Z, N, f.m, f.nu, thetas[0, p].contiguous())
        torch.cuda.synchronize()
        assert o.item() == out[0, p].item() and torch.equal(g, grad[0, p])
    for p in (0, 21, 42, 63):
        want, gwant = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, f.thetas[p], with_grad=True, threads=THREADS)
        print("theta", p, out[0, p].item(), want, flush=True)
        assert_total(out[0, p].item(), want, grad[0, p].cpu().numpy(), gwant)
    plan.close()


def test_32_fields_captured_graph(v):
    import torch
    w = wl.config_multifield(knn_threads=THREADS)
    dfs = [dev_field(f) for f in w.fields]
    plan = v.BatchedPlan([(L, Z, N, f.m) for (L, Z, N), f in zip(dfs, w.fields)], 1, 1.5, True)
    thetas = torch.from_numpy(np.stack([f.thetas[0] for f in w.fields])).cuda().reshape(-1, 1, 3).contiguous()
    out, grad, st = plan.outputs()
    graph = plan.capture(thetas, out, grad, st)
    graph.launch()
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    rng = np.random.default_rng(1820)
    parts = []
    for q, ((L, Z, N), f) in enumerate(zip(dfs, w.fields)):
        o, g, s = v.vecchia_loglik_grad(L, Z, N, f.m, f.nu, thetas[q, 0].contiguous())
        torch.cuda.synchronize()
        assert o.item() == out[q, 0].item() and torch.equal(g, grad[q, 0]), q
        parts.append(check_terms(v, f, f.thetas[0], L, Z, N, sample_rows(rng, f.n, f.m, 300), True))
    assert_adjudicated(parts)
    for q in np.argsort([f.n for f in w.fields])[:4]:
        f = w.fields[q]
        want, gwant = oracle.loglik(f.locs, f.z, f.nbr, f.m, f.nu, f.thetas[0], with_grad=True, threads=THREADS)
        print("field", q, f.n, f.m, out[q, 0].item(), want, flush=True)
        assert_total(out[q, 0].item(), want, grad[q, 0].cpu().numpy(), gwant)
    graph.close()
    plan.close()

"""vecchia_loglik_grad_noalloc, the workspace-free form of vecchia_loglik_grad for callers that cannot
allocate: through the C ABI it must give the results of vecchia_loglik_grad (same kernels, same summation
order: bitwise equal) on two calls in a row, the second on a smaller input, and refuse sizes beyond its
static scratch on the host."""
import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def v():
    import paper_2403_07412_amd as v
    v.library()
    return v


def _call_noalloc(v, locs, z, nbr, m, nu, theta):
    import torch
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(3, dtype=torch.float64, device="cuda")
    status = torch.empty(1, dtype=torch.int64, device="cuda")
    rc = v.library().vecchia_loglik_grad_noalloc(
        ctypes.c_void_p(locs.data_ptr()), ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(nbr.data_ptr()),
        ctypes.c_int64(z.shape[0]), ctypes.c_int32(m), ctypes.c_double(nu), ctypes.c_void_p(theta.data_ptr()),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(status.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    return out, grad, status


def test_noalloc_equals_the_workspace_entry_point(v):
    import torch
    rng = np.random.default_rng(4242)
    # first call: several slices of the static scratch and a ragged last one; second call: one small slice
    for n, m, nu in [(600_000, 30, 1.5), (5_000, 61, 0.5)]:
        print(f"noalloc n={n} m={m} nu={nu}", flush=True)
        locs = rng.uniform(size=(n, 2))
        nbr = wl.nearest_previous_neighbours(locs, m)
        z = rng.standard_normal(n)
        dev = torch.device("cuda:0")
        L = torch.from_numpy(locs).to(dev)
        Z = torch.from_numpy(z).to(dev)
        N = torch.from_numpy(nbr).to(dev)
        th = torch.tensor([1.3, 0.07, 1e-3], dtype=torch.float64, device=dev)
        o1, g1, s1 = _call_noalloc(v, L, Z, N, m, nu, th)
        o2, g2, s2 = v.vecchia_loglik_grad(L, Z, N, m, nu, th)
        torch.cuda.synchronize()
        assert int(s1.item()) == 0 and int(s2.item()) == 0
        assert torch.equal(o1, o2), (o1.item(), o2.item())
        assert torch.equal(g1, g2), (g1.cpu().numpy(), g2.cpu().numpy())


def test_noalloc_rejects_sizes_beyond_its_scratch(v):
    lib = v.library()
    d = ctypes.c_void_p(0x1000)  # never dereferenced: the size check comes first
    too_big = (1 << 26) + 1
    assert lib.vecchia_loglik_grad_noalloc(d, d, d, ctypes.c_int64(too_big), ctypes.c_int32(10),
                                           ctypes.c_double(0.5), d, d, d, d, None) == 2

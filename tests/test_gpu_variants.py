"""Every kernel variant against the oracle, across tile-row boundaries of m.

m + 2 rows are factored (neighbours, the point, the observation row), in
16-row tiles: m = 14 fills one tile exactly, m = 30 two, m = 126 eight; the
next m starts a new tile.  Each feasible variant must give the oracle's total
(rel 1e-10) and gradient (rel 1e-9) and the oracle's per-point terms.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from util import assert_grad_close, assert_total_close, to_device

pytestmark = pytest.mark.gpu

VARIANTS = ["unblocked", "tile_w1", "tile_w2", "tile_w4", "tile_w8"]
MS = [1, 14, 15, 30, 47, 62, 64, 94, 120, 126, 127, 150, 160]
NUS = [0.5, 1.5, 2.5]


def cases():
    out = []
    for im, m in enumerate(MS):
        for v in VARIANTS:
            out.append(pytest.param(m, NUS[im % 3], v, id=f"m{m}-nu{NUS[im % 3]}-{v}"))
    return out


@pytest.fixture(scope="module")
def lib():
    import paper_2403_07412_amd as v
    v.library()
    return v


@pytest.mark.parametrize("m,nu,variant", cases())
def test_variant_matches_oracle(lib, m, nu, variant):
    import torch
    if not lib.vecchia_variant_feasible(m, variant):
        pytest.skip(f"{variant} cannot hold m={m}")
    print(f"case m={m} nu={nu} variant={variant}", flush=True)
    rng = np.random.default_rng(3000 + m)
    n = 3 * m + 57 if m < 100 else 2 * m + 41
    f = wl.small_field(rng, n, m, nu, (1.1, 0.07, 5e-4))
    locs, z, nbr, theta = to_device(f)
    out, g, st = lib.vecchia_loglik_variant(locs, z, nbr, m, nu, theta, variant, with_grad=True)
    out0, _, st0 = lib.vecchia_loglik_variant(locs, z, nbr, m, nu, theta, variant, with_grad=False)
    t, gt, st1 = lib.vecchia_loglik_terms_variant(locs, z, nbr, m, nu, theta, variant, with_grad=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(st0.item()) == 0 and int(st1.item()) == 0
    ell, gref = oracle.terms(f.locs, f.z, f.nbr, m, nu, f.thetas[0], with_grad=True)
    ref = oracle.compensated_sum(ell)
    assert_total_close(out.item(), ref, 1e-10, "value with gradient")
    assert_total_close(out0.item(), ref, 1e-10, "value only")
    assert_grad_close(g.cpu().numpy(), [oracle.compensated_sum(gref[:, p]) for p in range(3)],
                      np.abs(gref).sum(0), 1e-9, "gradient")
    np.testing.assert_allclose(t.cpu().numpy(), ell, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(gt.cpu().numpy(), gref, rtol=2e-7, atol=1e-9 * np.abs(gref).max())


def test_variant_table_roundtrip(lib):
    for m in [10, 60, 120]:
        before = lib.vecchia_get_variant(m, True)
        lib.vecchia_set_variant(m, True, "unblocked")
        assert lib.vecchia_get_variant(m, True) == 1
        lib.vecchia_set_variant(m, True, "auto")
        assert lib.vecchia_get_variant(m, True) == before
    with pytest.raises(lib.VecchiaError):
        lib.vecchia_set_variant(150, True, "tile_w1")  # 66 tiles do not fit one wavefront

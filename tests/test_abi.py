"""The C ABI library: it loads, exports every symbol the header declares, and
rejects bad arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vecchia.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vecchia_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2403_07412_amd as v
    if not os.path.exists(v.LIB_PATH):
        pytest.fail("libvecchia.so is not built (run __graft_entry__.build())")
    return v.library()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ["vecchia_loglik", "vecchia_loglik_grad", "vecchia_loglik_terms", "vecchia_workspace_size",
                 "vecchia_strerror", "vecchia_version"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_queries(lib):
    import paper_2403_07412_amd as v
    assert "gfx950" in v.version()
    assert v.vecchia_workspace_size(0, 30) > 0
    a = v.vecchia_workspace_size(1_000_000, 120)
    assert a >= (1_000_000 // 16) * 40
    assert lib.vecchia_strerror(4) == b"workspace missing or too small"


def test_argument_errors_are_synchronous(lib):
    P = ctypes.c_void_p
    dummy = P(0x1000)  # never dereferenced: validation fails first
    ws = P(0x2000)
    # unsupported m
    assert lib.vecchia_loglik(dummy, dummy, dummy, 100, 161, 0.5, dummy, dummy, dummy, ws, 1 << 30, None) == 2
    # bad nu
    assert lib.vecchia_loglik(dummy, dummy, dummy, 100, 10, 1.0, dummy, dummy, dummy, ws, 1 << 30, None) == 1
    # negative n, missing theta, missing output
    assert lib.vecchia_loglik(dummy, dummy, dummy, -1, 10, 0.5, dummy, dummy, dummy, ws, 1 << 30, None) == 1
    assert lib.vecchia_loglik(dummy, dummy, dummy, 100, 10, 0.5, None, dummy, dummy, ws, 1 << 30, None) == 1
    assert lib.vecchia_loglik_grad(dummy, dummy, dummy, 100, 10, 0.5, dummy, dummy, None, dummy, ws, 1 << 30,
                                   None) == 1
    # workspace too small
    assert lib.vecchia_loglik(dummy, dummy, dummy, 100, 10, 0.5, dummy, dummy, dummy, ws, 16, None) == 4
    # terms: idx NULL needs nidx == n
    assert lib.vecchia_loglik_terms(dummy, dummy, dummy, 100, 10, 0.5, dummy, None, 5, dummy, None, dummy,
                                    None) == 1


def test_variant_table_roundtrip_on_host(tmp_path, lib):
    import paper_2403_07412_amd as v
    before = v.variant_table()
    assert len(before["grad"]) == v.VECCHIA_MAX_M + 1
    for m in range(v.VECCHIA_MAX_M + 1):
        assert v.vecchia_variant_feasible(m, before["grad"][m])
    v.vecchia_set_variant(60, True, "unblocked")
    path = tmp_path / "table.json"
    v.save_variant_table(str(path))
    v.vecchia_set_variant(60, True, "auto")
    assert v.vecchia_get_variant(60, True) == before["grad"][60]
    v.load_variant_table(str(path))
    assert v.vecchia_get_variant(60, True) == 1
    v.vecchia_set_variant(60, True, "auto")
    with pytest.raises(v.VecchiaError):
        v.vecchia_set_variant(150, True, "tile_w1")


def _fake_fields(v, specs):
    """Field descriptors with dummy device addresses: planning never dereferences them."""
    arr = (v._Field * len(specs))()
    for f, (n, m) in enumerate(specs):
        arr[f] = v._Field(0x10000, 0x20000, 0x30000, n, m)
    return arr


def test_batched_workspace_query_and_plan_are_host_only(lib):
    import paper_2403_07412_amd as v
    specs = [(10_000, 10), (200_000, 60), (1, 30), (0, 5), (50_000, 150)]
    arr = _fake_fields(v, specs)
    need = lib.vecchia_batched_workspace(arr, len(specs), 4)
    # at least the per-row values and flags, 36 bytes per (field, theta, point)
    assert need >= 36 * 4 * sum(n for n, _ in specs)
    handle = ctypes.c_void_p()
    cov = v.Cov(v.MATERN, v.EUCLIDEAN, 1.5)
    assert lib.vecchia_plan_create_cov(arr, len(specs), 4, ctypes.byref(cov), 1, ctypes.byref(handle)) == 0
    try:
        assert lib.vecchia_plan_workspace_size(handle) == need
        classes = lib.vecchia_plan_num_classes(handle)
        assert classes == len({(m + 2 + 15) // 16 for n, m in specs if n > 0})
        items = ctypes.c_int64()
        total = 0
        for c in range(classes):
            assert lib.vecchia_plan_class_info(handle, c, None, None, None, ctypes.byref(items)) == 0
            total += items.value
        assert total == 4 * sum(n for n, _ in specs)
    finally:
        assert lib.vecchia_plan_destroy(handle) == 0


def _expected_group(T, ntheta):
    """Lockstep group size of a class: four vectors, one wavefront each, up to five tile rows (the one-wavefront
    variant holds at most 20 tiles) when the vectors divide into fours."""
    return 4 if T <= 5 and ntheta % 4 == 0 else 1


@pytest.mark.parametrize("ntheta", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("with_grad", [0, 1])
def test_plan_picks_lockstep_groups_on_the_host(lib, ntheta, with_grad):
    import paper_2403_07412_amd as v
    specs = [(1000, 10), (1000, 30), (1000, 45), (1000, 60), (1000, 75), (1000, 94), (1000, 95), (1000, 120)]
    m_of = {(m + 2 + 15) // 16: m for _, m in specs}  # one field per tile class
    arr = _fake_fields(v, specs)
    T, var = ctypes.c_int32(), ctypes.c_int32()
    for enable in (1, 0):
        prev = lib.vecchia_set_lockstep(enable)
        handle = ctypes.c_void_p()
        try:
            assert lib.vecchia_plan_create(arr, len(specs), ntheta, ctypes.c_double(1.5), with_grad,
                                           ctypes.byref(handle)) == 0
        finally:
            lib.vecchia_set_lockstep(prev)
        try:
            groups = []
            for c in range(lib.vecchia_plan_num_classes(handle)):
                assert lib.vecchia_plan_class_info(handle, c, ctypes.byref(T), ctypes.byref(var), None, None) == 0
                g = lib.vecchia_plan_class_group(handle, c)
                assert g == (_expected_group(T.value, ntheta) if enable else 1), (T.value, var.value)
                # lockstep classes run the one-wavefront variant, the others the table's
                table = lib.vecchia_get_variant(m_of[T.value], with_grad)
                assert var.value == (2 if g == 4 else table), (T.value, var.value, table)
                groups.append(g)
            if enable and ntheta % 4 == 0:
                assert max(groups) == 4
            assert lib.vecchia_plan_class_group(handle, len(groups)) < 0
        finally:
            assert lib.vecchia_plan_destroy(handle) == 0


def test_batched_rejects_oversized_batches_on_the_host(lib):
    import paper_2403_07412_amd as v
    arr = _fake_fields(v, [(10, 5), (10, 5)])
    handle = ctypes.c_void_p()
    # nf * ntheta evaluations must fit in 2^31 - 1
    assert lib.vecchia_plan_create(arr, 2, 2 ** 31 - 1, ctypes.c_double(0.5), 0, ctypes.byref(handle)) == 2
    assert lib.vecchia_batched_workspace(arr, 2, 2 ** 31 - 1) == 0
    # m beyond the maximum, bad nu, no fields
    big = _fake_fields(v, [(10, 161)])
    assert lib.vecchia_plan_create(big, 1, 1, ctypes.c_double(0.5), 0, ctypes.byref(handle)) == 2
    assert lib.vecchia_plan_create(arr, 2, 1, ctypes.c_double(0.7), 0, ctypes.byref(handle)) == 1
    assert lib.vecchia_plan_create(arr, 0, 1, ctypes.c_double(0.5), 0, ctypes.byref(handle)) == 1
    # the one-call form checks its arguments before any device work
    P = ctypes.c_void_p
    d = P(0x1000)
    assert lib.vecchia_loglik_batched(arr, 2, d, 1, 0.5, 1, d, None, d, d, 1 << 30, None) == 1  # grad missing
    assert lib.vecchia_loglik_batched(arr, 2, d, 1, 0.5, 0, d, None, d, d, 16, None) == 4      # workspace


# Files of the likelihood path (single and batched evaluations, kernels, sums).
LIKELIHOOD_SOURCES = ["vecchia.hip", "batched.hip", "launch.h", "kernel_tile.h", "kernel_lds.h", "reduce.h",
                      "device_common.h"]


def test_likelihood_path_never_allocates_or_creates_streams():
    csrc = os.path.join(ROOT, "paper_2403_07412_amd", "csrc")
    banned = re.compile(r"\b(hipMalloc\w*|hipExtMalloc\w*|hipHostMalloc|hipFree\w*|hipStreamCreate\w*|"
                        r"hipMemcpy\w*|hipMemset\w*|hipDeviceSynchronize|hipStreamSynchronize)\b")
    for name in LIKELIHOOD_SOURCES:
        text = open(os.path.join(csrc, name)).read()
        text = re.sub(r"//[^\n]*", "", text)
        hits = banned.findall(text)
        assert not hits, (name, hits)

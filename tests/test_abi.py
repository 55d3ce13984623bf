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

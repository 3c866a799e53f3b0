"""The C ABI library loads, exports every symbol include/qfs.h declares, and
rejects bad arguments on the host (no GPU needed: nothing is enqueued)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2502_12428_amd as qfs
from oracle import fast

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qfs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qfs_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    names = declared_functions()
    assert len(names) >= 14
    assert sorted(qfs.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    L = qfs.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_sizes():
    assert [qfs.len_g(p) for p in (3, 5, 7, 11)] == [165, 969, 2925, 12341]
    assert [qfs.len_delta(p) for p in (3, 5, 7, 11)] == [2925, 91881, 818805, 14391741]
    assert qfs.len_g(13) == -1
    assert qfs.num_monomials(-1) == 0


@pytest.mark.parametrize("deg", [0, 1, 4, 8, 16, 24, 40])
def test_rank_matches_oracle_basis_order(deg):
    # the oracle enumerates B_d in descending lex order; the library's closed form must agree
    B = fast.basis(deg)
    for i, e in enumerate(B):
        assert qfs.monomial_rank(e) == i
    for i in range(0, len(B), max(1, len(B) // 97)):
        assert qfs.monomial_unrank(deg, i) == tuple(int(x) for x in B[i])


@pytest.mark.parametrize("deg", [80, 168, 440])
def test_unrank_inverts_rank_on_large_degrees(deg):
    n = qfs.num_monomials(deg)
    for i in list(range(0, 2000)) + list(range(n - 2000, n)) + list(range(0, n, max(1, n // 5000))):
        e = qfs.monomial_unrank(deg, i)
        assert sum(e) == deg and min(e) >= 0
        assert qfs.monomial_rank(e) == i


def test_unrank_rejects_out_of_range():
    with pytest.raises(qfs.QfsError):
        qfs.monomial_unrank(4, 35)
    assert qfs.monomial_rank((-1, 0, 0, 5)) == -1


def _call(fn, *args):
    L = qfs.lib()
    return getattr(L, fn)(*args)


def test_host_side_argument_errors():
    L = qfs.lib()
    nul = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(4096)
    assert L.qfs_delta1(13, 1, dummy, nul, dummy, nul, dummy, 1 << 20, nul) == qfs.QFS_EUNSUPPORTED
    assert L.qfs_delta1(7, -1, dummy, nul, dummy, nul, dummy, 1 << 20, nul) == qfs.QFS_EINVAL
    assert L.qfs_delta1(7, 0, nul, nul, nul, nul, nul, 0, nul) == qfs.QFS_OK
    assert L.qfs_delta1(7, 1, nul, nul, dummy, nul, dummy, 1 << 20, nul) == qfs.QFS_EINVAL
    assert b"null" in L.qfs_last_error()
    assert L.qfs_theta(5, 1, dummy, dummy, dummy, 65, dummy, 1 << 20, nul) == qfs.QFS_EINVAL
    assert L.qfs_theta(5, 1, dummy, dummy, dummy, 1, nul, 1 << 20, nul) == qfs.QFS_EINVAL
    assert L.qfs_height(1, dummy, dummy, 11, 7, dummy, dummy, 1 << 20, nul) == qfs.QFS_EINVAL
    assert L.qfs_height(1, dummy, dummy, 10, 13, dummy, dummy, 1 << 20, nul) == qfs.QFS_EUNSUPPORTED
    assert L.qfs_height(0, nul, nul, 10, 7, nul, nul, 0, nul) == qfs.QFS_OK
    assert L.qfs_height_plain(9, 1, dummy, 10, dummy, dummy, 1 << 20, nul) == qfs.QFS_EUNSUPPORTED
    assert L.qfs_height_plain(7, 1, dummy, 0, dummy, dummy, 1 << 20, nul) == qfs.QFS_EINVAL
    misaligned = ctypes.c_void_p(4096 + 8)
    assert L.qfs_height_plain(7, 1, dummy, 10, dummy, misaligned, 1 << 20, nul) == qfs.QFS_EINVAL


def test_mfma_counts_of_both_passes():
    for p in (3, 5, 7, 11):
        full, band = qfs.mfma_per_surface(p), qfs.mfma_per_surface(p, band=True)
        assert full > 0 and band > 0 and band < full
    assert qfs.lib().qfs_mfma_per_surface(7, 2) == -1
    assert qfs.lib().qfs_mfma_per_surface(13, 0) == -1


def test_options():
    assert qfs.get_option("height_band") == 1
    qfs.set_option("height_band", 0)
    try:
        assert qfs.get_option("height_band") == 0
    finally:
        qfs.set_option("height_band", 1)
    assert qfs.get_option("height_band") == 1
    with pytest.raises(qfs.QfsError):
        qfs.set_option("height_band", 2)
    with pytest.raises(qfs.QfsError):
        qfs.set_option("no_such_option", 1)
    with pytest.raises(qfs.QfsError):
        qfs.get_option("no_such_option")
    assert qfs.get_option("height_graph") == 1
    qfs.set_option("height_graph", 0)
    try:
        assert qfs.get_option("height_graph") == 0
    finally:
        qfs.set_option("height_graph", 1)
    assert qfs.get_option("height_graphs_cached") == 0
    # the deep chain's multiplier power per prime: J divides p(p-1), 1 <= J <= p-1
    for p in (3, 5, 7, 11):
        J = qfs.get_option("chain_power_p%d" % p)
        assert 1 <= J <= p - 1 and (p * (p - 1)) % J == 0
    with pytest.raises(qfs.QfsError):
        qfs.set_option("chain_power_p7", 1)


def test_autotune_and_tuning_cache_argument_errors(tmp_path):
    L = qfs.lib()
    assert L.qfs_autotune(0, None, None, 10, 7, None, None, 0, None, None, 2) == qfs.QFS_EINVAL
    assert L.qfs_autotune(4, None, None, 10, 7, None, None, 0, None, None, 0) == qfs.QFS_EINVAL
    assert L.qfs_load_tuning(None, 7) == qfs.QFS_EINVAL
    assert L.qfs_load_tuning(str(tmp_path / "missing.jsonl").encode(), 7) == qfs.QFS_EINVAL
    with pytest.raises(qfs.QfsError):
        qfs.set_option("gpow_per_cu", 0)
    assert qfs.get_option("gpow_per_cu") == 8


def test_epilogue_division_is_exact():
    # The deep kernels' epilogue takes floor(x / p^2) as trunc(fma(x, 1/p^2, 0.5/p^2)) in
    # fp32 for every accumulator value x <= C(4J+3,3) (p^2-1)^2; check that range exhaustively
    # (one rounding of the exact x*c1 + c2, which float64 holds exactly here).
    from math import comb
    for p in (3, 5, 7, 11):
        for J in (qfs.get_option("chain_power_p%d" % p),):
            p2 = p * p
            bound = comb(4 * J + 3, 3) * (p2 - 1) ** 2
            if bound >= 1 << 24:
                continue  # the kernels take the integer remainder there
            c1 = np.float32(1.0) / np.float32(p2)
            c2 = np.float32(0.5) / np.float32(p2)
            x = np.arange(bound + 1, dtype=np.int64)
            y = (x.astype(np.float64) * np.float64(c1) + np.float64(c2)).astype(np.float32)
            assert np.array_equal(np.trunc(y).astype(np.int64), x // p2), (p, J)


def test_height_reduced_argument_errors():
    L = qfs.lib()
    assert L.qfs_height_reduced_workspace_bytes(-1, 7) == 0
    assert L.qfs_height_reduced_workspace_bytes(16, 13) == 0
    assert L.qfs_height_reduced_workspace_bytes(16, 7) >= 256 + 3 * 256
    assert L.qfs_height_reduced(-1, None, None, 10, 7, None, None, 0, None) == qfs.QFS_EINVAL
    assert L.qfs_height_reduced(4, None, None, 11, 7, None, None, 0, None) == qfs.QFS_EINVAL
    assert L.qfs_height_reduced(4, None, None, 10, 13, None, None, 0, None) == qfs.QFS_EUNSUPPORTED
    assert L.qfs_height_reduced(4, None, None, 10, 7, None, None, 0, None) == qfs.QFS_EINVAL
    assert L.qfs_height_reduced(0, None, None, 10, 7, None, None, 0, None) == qfs.QFS_OK


def test_mfma_peak_argument_errors():
    L = qfs.lib()
    import ctypes
    t = ctypes.c_double(0.0)
    assert L.qfs_mfma_peak(0, None, ctypes.byref(t), None) == qfs.QFS_EINVAL
    assert L.qfs_mfma_peak(100, None, ctypes.byref(t), None) == qfs.QFS_EINVAL

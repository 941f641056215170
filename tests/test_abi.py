"""The C-ABI library loads and exports every entry point include/hdm.h declares (no GPU needed)."""
import ctypes as C
import os

import pytest

from paper_2311_06115_amd import hdm


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hdm.LIB_PATH):
        from paper_2311_06115_amd import build
        build.build()
    return hdm.lib()


def test_header_declares_the_boundary():
    names = hdm.declared_symbols()
    for want in ["hdm_compress", "hdm_matvec", "hdm_eigs", "hdm_submit", "hdm_poll", "hdm_op_perm", "hdm_op_knn"]:
        assert want in names


def test_every_declared_symbol_is_exported(L):
    missing = [s for s in hdm.declared_symbols() if not hasattr(L, s)]
    assert missing == []


def test_host_only_calls(L):
    p = hdm.default_params()
    assert p.alpha == 1.0 and p.knn_iters == 10 and p.budget == 0.05
    assert L.hdm_version().decode().startswith("hdm")
    assert isinstance(L.hdm_last_error(), bytes)


def test_null_arguments_are_rejected_without_touching_the_device(L):
    assert L.hdm_op_stats(None, None) == 1
    assert L.hdm_matvec(None, 0, None, None, 1, None) == 1
    assert b"NULL" in L.hdm_last_error()
    assert L.hdm_ctx_create(0, 0, None) == 1


def _params(n, m, s, dtype, k=16, dim=784):
    p = hdm.default_params()
    p.n, p.dim, p.x_dtype, p.eps = n, dim, dtype, 50.0
    p.leaf_m, p.max_rank_s, p.knn_k = m, s, k
    return p


def test_parameter_rules_without_a_device(L):
    ok = _params(65536, 256, 256, hdm.U8)            # leaves of 256 points, s = 256
    assert L.hdm_params_validate(C.byref(ok)) == 0
    # u8 points with max_rank_s above the smallest leaf are refused (171-point leaves)
    bad = _params(21850, 256, 256, hdm.U8)
    assert L.hdm_params_validate(C.byref(bad)) == 1
    assert b"smallest leaf" in L.hdm_last_error()
    assert L.hdm_params_validate(C.byref(_params(21850, 256, 128, hdm.U8))) == 0
    assert L.hdm_params_validate(C.byref(_params(4278, 256, 256, hdm.U8))) == 1
    # the rule is about u8 codes only
    assert L.hdm_params_validate(C.byref(_params(21850, 256, 256, hdm.F64, dim=3))) == 0
    # ranks above 512 (up to 1024) only with leaves of at most 512 points: the
    # 6-D shape of the scaling study (m = s = 768) at N = 100000 has 391-point leaves
    assert L.hdm_params_validate(C.byref(_params(100000, 768, 768, hdm.F64, k=64, dim=6))) == 0
    assert L.hdm_params_validate(C.byref(_params(6000, 768, 768, hdm.F64, k=64, dim=6))) == 1   # 750-point leaves
    assert b"512 points" in L.hdm_last_error()
    assert L.hdm_params_validate(C.byref(_params(100000, 768, 1025, hdm.F64, k=64, dim=6))) == 1
    for field, val in [("eps", 0.0), ("alpha", 0.5), ("max_rank_s", 0), ("knn_k", 65), ("leaf_m", 1),
                       ("budget", 1.5), ("near_prec", 7)]:
        p = _params(4096, 256, 64, hdm.F64, dim=3)
        setattr(p, field, val)
        assert L.hdm_params_validate(C.byref(p)) == 1, field
    assert L.hdm_params_validate(None) == 1

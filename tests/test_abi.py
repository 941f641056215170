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

"""Host-side checks of the C ABI (no GPU): the library loads and exports every function that
include/hespmv.h declares, and the Python binding covers the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hespmv.h")
LIB = os.path.join(ROOT, "paper_2603_04742_amd", "libhespmv.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_04742_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_protocol_calls():
    names = declared()
    for n in ("hs_keygen", "hs_encrypt", "hs_cssc_pack", "hs_he_spmv", "hs_decrypt"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_matches_header(lib):
    from paper_2603_04742_amd import hespmv
    assert sorted(hespmv.SIGNATURES) == declared()


def test_error_path_without_device(lib):
    """A null argument is rejected on the host with HS_EINVAL and a message."""
    from paper_2603_04742_amd import hespmv
    assert hespmv.lib.hs_ctx_create(None, None) == hespmv.HS_EINVAL
    assert b"null" in hespmv.lib.hs_last_error()


def test_cdt_table_matches_oracle(lib):
    """The library computes its own Gaussian CDT (128-bit fixed point); it must equal the oracle's
    table (computed from the definition at 80 decimal digits)."""
    import numpy as np
    import oracle
    from paper_2603_04742_amd import hespmv
    assert np.array_equal(hespmv.cdt_table(), oracle.cdt())

"""The C ABI: libsmx.so loads (no GPU needed) and exports every declared symbol."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smx_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["smx_create", "smx_destroy", "smx_load_k", "smx_set_groups", "smx_set_mu",
                 "smx_set_temperature", "smx_evaluate", "smx_get_d", "smx_trace", "smx_energy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2004_10811_amd as smx
    if not os.path.exists(smx.LIB_PATH):
        pytest.skip("libsmx.so not built")
    lib = ctypes.CDLL(smx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the Python binding declares a signature for every symbol, with the same names
    assert sorted(smx.SIGNATURES) == declared_functions()
    smx.load_library()


def test_last_error_without_context_is_a_string():
    import paper_2004_10811_amd as smx
    if not os.path.exists(smx.LIB_PATH):
        pytest.skip("libsmx.so not built")
    lib = smx.load_library()
    assert isinstance(lib.smx_last_error(None), bytes)


def test_constants_match_header():
    import paper_2004_10811_amd as smx
    text = open(HEADER).read()
    for name in ["SMX_OK", "SMX_E_INVALID", "SMX_E_STATE", "SMX_E_NOT_SYMMETRIC", "SMX_E_NONFINITE",
                 "SMX_E_UNSUPPORTED", "SMX_E_NOMEM", "SMX_E_HIP", "SMX_E_NOT_CONVERGED", "SMX_FP64",
                 "SMX_BF16_3W", "SMX_BF16_1W", "SMX_FP32"]:
        m = re.search(rf"#define {name}\s+(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(smx, name), name

"""The C-ABI library loads and exports every call include/sfem.h declares (CPU only:
no HIP device call is made here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfem.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sfem_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sfem_create", "sfem_setup", "sfem_apply", "sfem_diagonal", "sfem_pcg", "sfem_grad_nu",
              "sfem_set_coeffs", "sfem_load", "sfem_qpoint_coords", "sfem_destroy", "sfem_last_error"):
        assert n in names


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (the binding always loads torch's HIP runtime first)
    from paper_1910_03032_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsfem.so is not built: run `python -m paper_1910_03032_amd.build`")
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    from paper_1910_03032_amd import _lib
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_pure_host_calls(lib):
    assert lib.sfem_abi_version() == 10
    assert isinstance(lib.sfem_last_error(None), bytes)
    from paper_1910_03032_amd._lib import CtxInfo
    ci = CtxInfo()
    assert lib.sfem_get_info(None, C.byref(ci)) == -1  # SFEM_E_ARG on a NULL context
    assert lib.sfem_set_stream(None, None) == -1
    lib.sfem_destroy(None)  # no-op
    assert lib.sfem_apply_noalloc(None, 2, 0, 1, None, None) == -1
    assert lib.sfem_flow_step(None, None, None, None, None, None) == -1
    assert lib.sfem_flow_create(0, None, 2, 0, None, None, 0, None, None, None) == -1
    assert isinstance(lib.sfem_flow_last_error(None), bytes)
    lib.sfem_flow_destroy(None)  # no-op
    assert lib.sfem_lor_setup(None, 1, None) == -1
    assert lib.sfem_lor_apply(None, 1, None, None) == -1
    assert lib.sfem_lor_vcycle(None, 1, 0, None, None) == -1


def test_structs_match_header_layout():
    from paper_1910_03032_amd._lib import PcgOpts, PcgInfo
    # double, int, int, double, int, int, int, int, int -> 44 bytes, padded to 48
    assert C.sizeof(PcgOpts) == 48
    assert C.sizeof(PcgInfo) == 32
    from paper_1910_03032_amd._lib import CtxInfo
    # int, int, int64, int64, int, int, int64, int64, int64
    assert C.sizeof(CtxInfo) == 56
    from paper_1910_03032_amd._lib import FlowOpts, FlowInfo
    assert C.sizeof(FlowOpts) == 48  # 3 doubles, 6 ints
    assert C.sizeof(FlowInfo) == 136  # int (padded to 8), 4 sfem_pcg_info
    from paper_1910_03032_amd._lib import LorInfo
    assert C.sizeof(LorInfo) == 8 + 2 * 12 * 8 + 8 + 12 * 4


def test_library_is_gfx950_code_object():
    from paper_1910_03032_amd import _lib
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data

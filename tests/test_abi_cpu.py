"""CPU checks of the C ABI library: it loads, exports every symbol include/pp.h
declares, its struct layouts match the binding, and the binding refuses to run
without the built library.  No compute calls (there is no GPU here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pp.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pp_status|void|const char\*|uint64_t)\s+(pp_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_functions():
    from paper_1610_04398_amd import _binding
    assert _declared_functions() == sorted(_binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_1610_04398_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_binding.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1610_04398_amd import _binding
    with pytest.raises(_binding.LibraryMissing):
        _binding.load(str(tmp_path / "missing.so"))


def test_struct_layouts_match_header():
    from paper_1610_04398_amd import _binding
    # pp_params: int32 p; double theta; int32 leaf_max, precision, self_mode (natural alignment)
    assert ctypes.sizeof(_binding.pp_params) == 32
    assert _binding.pp_params.theta.offset == 8
    assert ctypes.sizeof(_binding.pp_stats) == 4 * 4 + 5 * 8 + 8 + 12 * 8


def test_status_strings_without_gpu():
    from paper_1610_04398_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.skip("library not built")
    lib = _binding.load()
    assert lib.pp_status_string(0) == b"ok"
    assert lib.pp_status_string(-2) == b"target outside the root square"
    assert lib.pp_last_error(None) == b"null context"


def test_array_ids_match_header():
    from paper_1610_04398_amd import _binding
    text = open(HEADER).read()
    for name, val in _binding.ARRAYS.items():
        m = re.search(r"PP_ARR_%s\s*=\s*(\d+)" % name, text)
        assert m and int(m.group(1)) == val, name


def test_footprint_estimate_is_monotone():
    """The admission estimate grows with grid size, target count and order (host-only function)."""
    from paper_1610_04398_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.skip("library not built")
    fe = _binding.pp_footprint_estimate
    a = fe(128, 128, 1024, 12, 64)
    assert 0 < a < fe(256, 256, 1024, 12, 64) < fe(512, 512, 1024, 12, 64)
    assert a < fe(128, 128, 8192, 12, 64)
    assert fe(512, 512, 4096, 8, 64) < fe(512, 512, 4096, 16, 64)
    assert fe(0, 128, 10, 12, 64) == 0
    # 4096^2 grid with 32K targets stays well inside one GPU's 288 GB
    assert fe(4096, 4096, 32768, 12, 64) < 32 << 30

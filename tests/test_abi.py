"""Host-only checks of the C-ABI library: it loads and exports every function
that include/rhosvd.h declares (no GPU work is done here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rhosvd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rhosvd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_12663_amd import rhosvd
    if not os.path.exists(rhosvd.LIB_PATH):
        from paper_2201_12663_amd import build
        build.build()
    return rhosvd.load()


def test_header_declares_expected_api():
    from paper_2201_12663_amd import rhosvd
    assert declared_functions() == sorted(rhosvd.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_version_and_null_handle_errors(lib):
    assert lib.rhosvd_version().decode().count(".") == 2
    # NULL handles are rejected before any device work
    assert lib.rhosvd_destroy(None) == -1
    assert lib.rhosvd_get(None, None, None, None, None, None, None) == -1
    assert lib.rhosvd_phase_ms(None, 0) == -1.0
    assert lib.rhosvd_create(None, None, None) == -1


def test_struct_layouts_match_header():
    from paper_2201_12663_amd import rhosvd
    assert ctypes.sizeof(rhosvd.Options) == 32
    # 4 doubles + 3 doubles + 3 int32 + 3 int32 = 56 + 24 = 80
    assert ctypes.sizeof(rhosvd.Report) == 80

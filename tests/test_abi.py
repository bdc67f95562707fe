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
    return sorted(set(re.findall(r"\b(rhosvd_[a-z0-9_]+)\s*\(", text)))


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
    assert ctypes.sizeof(rhosvd.Options) == 40
    # 4 doubles + 3 doubles + 3 int32 + 3 int32 + 2 doubles + 2 int32 = 56 + 24 + 16 + 8 = 104
    assert ctypes.sizeof(rhosvd.Report) == 112


def test_null_handle_batched(lib):
    assert lib.rhosvd_reduce_batched(None, 1, None) == -1
    assert lib.rhosvd_batch_uses_graph(None) == 0
    assert lib.rhosvd_last_core_tile(None) == 0


def test_network_size_and_null_handles(lib):
    assert lib.rhosvd_net_num_params() == 128 * 67 + 128 + 128 * 128 + 128 + 2 * 128 + 2
    assert lib.rhosvd_net_set_params(None, None) == -1
    assert lib.rhosvd_net_forward(None, 1, None, None) == -1
    assert lib.rhosvd_reduce_learned(None, 1, 1, None, None, None, None, 1e-3, None, 64, None, None) == -1


def test_struct_offsets_match_a_c_compiler(tmp_path):
    """Compile the header with the host C compiler and compare every field offset
    of the public structs with the ctypes mirrors of the binding."""
    import shutil
    import subprocess
    from paper_2201_12663_amd import rhosvd
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"rhosvd_options": rhosvd.Options, "rhosvd_report": rhosvd.Report, "rhosvd_allocator": rhosvd.Allocator,
               "rhosvd_problem": rhosvd.Problem, "rhosvd_learned_info": rhosvd.LearnedInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rhosvd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with the shared library absent, loading raises instead of
    running anything else in its place."""
    from paper_2201_12663_amd import rhosvd
    monkeypatch.setattr(rhosvd, "_lib", None)
    monkeypatch.setattr(rhosvd, "LIB_PATH", str(tmp_path / "librhosvd.so"))
    with pytest.raises(RuntimeError, match="missing"):
        rhosvd.load()

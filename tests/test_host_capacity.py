"""Host-side capacity checks of the learned path (csrc/capacity.hpp), compiled
and run on the CPU: ranks that fit their buffers pass, each kind of overflow is
caught (the library returns RHOSVD_ERR_DEVICE before any launch then)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_learned_mode_capacity_checks(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "capacity_check"
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", os.path.join(HERE, "host_capacity_check.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout

"""Host code under sanitizers: the library's geometry tables and the resident
kernel's patch partition (host C++) built with g++ -fsanitize=address,undefined
and exercised over many shapes, orders and both coordinate systems (no device
code is involved)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_geometry_tables_clean_under_asan_ubsan(tmp_path):
    exe = tmp_path / "geometry_driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "sanitize", "geometry_driver.cpp"),
           os.path.join(ROOT, "paper_2501_14030_amd", "csrc", "hr_geometry.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-2000:]
    assert "geometry tables checked" in r.stdout
    assert "resident partitions checked: 52" in r.stdout

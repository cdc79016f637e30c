"""Host logic: the geometry tables built by several host threads equal the
one-thread build (the threads take ranges of subdomains; their row sets are
concatenated in order).  Compiles the library's geometry source with the
host compiler and a small checker (tests/geometry_threads_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2503_10032_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_threaded_geometry_build_equals_sequential(tmp_path):
    exe = str(tmp_path / "geometry_threads_check")
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", "-I", CSRC,
                    os.path.join(HERE, "geometry_threads_check.cpp"), os.path.join(CSRC, "geometry.cpp"),
                    "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("OK")

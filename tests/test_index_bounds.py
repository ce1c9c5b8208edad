"""The MPM kernels' shared index arithmetic checked on the CPU: tests/
index_bounds.cpp includes the kernel headers, is built for the host (the
device pass compiles nothing, no kernel is instantiated) and runs there,
checking the XCD-aware block order, the velocity-grid node layout, the P2G
and G2P LDS tile layouts and the grid update's choice of covering tiles
exhaustively for both block edges (see the file's header)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_kernel_index_arithmetic(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path / "index_bounds"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-x", "hip", "-std=c++17", "-O1",
                        os.path.join(HERE, "index_bounds.cpp"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout[-2000:]

"""Bounds check of the kernels' geometry on the CPU: tests/geometry_check.hip is built as a
host program against the same geometry functions the kernels use (segment partition,
sub-segments, ghost reflection, workgroup -> tile map, y-sweep column tiles, tile staging
indices, whole-row / whole-line lane layout, LDS regions and tree slots) and checks them
exhaustively over line lengths. Skipped when hipcc is missing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_kernel_geometry_stays_in_bounds(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "geometry_check")
    b = subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17",
                        os.path.join(HERE, "geometry_check.hip"), "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "geometry check: ok" in r.stdout, r.stdout[-3000:]

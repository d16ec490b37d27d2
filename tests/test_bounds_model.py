"""The kernels' LDS and row index arithmetic, checked on the host: the index
functions the kernels call (Layout<G> in csrc/hqc_device.h) are evaluated by
tests/bounds_model.cpp, built host-only with hipcc, for every instantiated
geometry over every lane, product shift, tile size and RM pass, against the
LDS layout and the device row sizes; and the persistent grid's tile
schedule over segments of several sets with their own tile sizes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_index_bounds(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "bounds_model")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-host-only", "-std=c++17", "-O2",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2512_12904_amd", "csrc"),
                           "-o", exe, os.path.join(ROOT, "tests", "bounds_model.cpp")],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 8, r.stdout

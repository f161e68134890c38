"""Host-side checks of helpers compiled into the HIP library, built for the
host with hipcc from tests/host/*.cpp (no GPU is used):
- the tile traversals (QPass runs and the naive sub-box walk, Sec. 3.2) both
  enumerate exactly the union of the sub-box rects, each tile once;
- the per-entry row range that lets a render wave skip an entry contains
  every row where the binary32 cutoff of Eq. (4) passes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _run_host_check(tmp_path, name):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / name)
    src = os.path.join(HERE, "host", name + ".cpp")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-ffp-contract=off", "-o", exe,
                    src], check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0" in out.stdout


def test_traversals_enumerate_the_union_once(tmp_path):
    _run_host_check(tmp_path, "traversal_check")


def test_entry_row_range_is_conservative(tmp_path):
    _run_host_check(tmp_path, "rows_check")

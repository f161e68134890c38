"""Host-side check of the tile traversals compiled into the HIP library
(QPass runs and the naive sub-box walk, Sec. 3.2): both enumerate exactly the
union of the sub-box rects, each tile once.  Built for the host with hipcc
from tests/host/traversal_check.cpp; no GPU is used."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_traversals_enumerate_the_union_once(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "traversal_check")
    src = os.path.join(HERE, "host", "traversal_check.cpp")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-o", exe, src],
                   check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0" in out.stdout

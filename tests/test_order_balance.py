"""Host-side check of the XCD-balanced work-group order of the pair-space polarization.

Builds tests/native/order_balance.hip with hipcc and runs its host code only (no GPU needed): every
item of the order is dealt to exactly one work-group, and the working (upper-triangle) tiles are
spread over the 8 XCDs to within one tile.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_xcd_slices_cover_and_balance(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "order_balance"
    src = os.path.join(HERE, "native", "order_balance.hip")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", src, "-o", str(exe)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    print(out.stdout)
    lines = [ln for ln in out.stdout.splitlines() if ln.strip()]
    assert len(lines) == 8 and all(ln.startswith("ok ") for ln in lines), out.stdout
    assert out.returncode == 0

"""The hand-derived face-flux adjoints (WENO5-JS, HLLC/Einfeldt in all four
wave patterns, the dissipative flux) against fourth-order central differences
of the forward face code, compiled for the host CPU (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_face_adjoints_match_finite_differences(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "face_adjoint_check"
    src = os.path.join(HERE, "native", "face_adjoint_check.cpp")
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", "-o", str(exe), src], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE)
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert out.returncode == 0, out.stdout

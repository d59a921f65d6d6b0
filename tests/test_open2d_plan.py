"""Host logic of the one-launch 2D open-box step: how the ring is split into network segments
and which tile row holds each face node a ring cell pulls from.  The check program includes
the kernel header and runs on the CPU (hipcc compiles it; no GPU code is launched)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1601_08103_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_ring_segments_and_rows(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "open2d_plan_check")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "host", "open2d_plan_check.hip"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("checks ") and out.stdout.split()[-1] == "0"

"""The serving engine's host-only admission rule and arena (csrc/admission.h),
built with the host compiler into a small driver and run on the CPU: capacity
less the slot workspaces, rounding, waiting under fragmentation, failing when
the server stops with nothing in flight, head-of-line order, and which
requests a free stream slot launches together."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_cs_0308004_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "cpp", "admission_driver.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_admission_rule(tmp_path):
    exe = tmp_path / "admission_driver"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", f"-I{CSRC}", "-o", str(exe), DRIVER],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    lines = r.stdout.splitlines()
    assert lines and all(ln.startswith("ok ") for ln in lines), r.stdout
    assert r.returncode == 0
    assert len(lines) == 18

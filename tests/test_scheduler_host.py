"""The request loop's admission and batch hand-out policy, built with the
host compiler alone and run on the CPU (no HIP in the policy)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_policy(tmp_path):
    exe = tmp_path / "test_scheduler"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2105_13611_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "test_scheduler.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"

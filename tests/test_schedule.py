"""Host logic of the decode launch: the frame-to-wave assignment
(csrc/schedule.h), compiled with the host C++ compiler and checked for
exact coverage of every frame over many batch sizes and shapes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_frame_in_exactly_one_wave(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "schedule_check")
    subprocess.check_call([cxx, "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_2605_10433_amd", "csrc"),
                           os.path.join(ROOT, "tests", "helpers", "schedule_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr

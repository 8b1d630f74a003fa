"""Host logic of the decoder's LDS layout: the placement of padding lanes
(csrc/lds_pad.h), compiled with the host C++ compiler and checked on the
l = 63 code's gather patterns and on random rows."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_padding_lanes_add_no_bank_conflict(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "lds_pad_check")
    subprocess.check_call([cxx, "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_2605_10433_amd", "csrc"),
                           os.path.join(ROOT, "tests", "helpers", "lds_pad_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr

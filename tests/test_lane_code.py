"""The matrix and check order compiled into the one-lane layered kernel
(paper_2605_10433_amd/csrc/lane_code.h), checked on the host against the
oracle: the rows are those of the l = 63 code's H_Z (Section V, the
[[126, 28]] code; oracle/codes.py), and updating the checks in the compiled
order gives every variable its checks in the order of the first-fit layers
of oracle/layered.py (the layered schedule's definition), so the one-lane
kernel computes the layer-by-layer result."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from oracle import codes, layered

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dump(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("lane") / "lane_code_dump")
    subprocess.check_call([cxx, "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_2605_10433_amd", "csrc"),
                           os.path.join(ROOT, "tests", "helpers", "lane_code_dump.cpp"), "-o", exe])
    lines = subprocess.run([exe], capture_output=True, text=True, timeout=60, check=True).stdout.splitlines()
    m, n, dc = map(int, lines[0].split()[1:])
    rows = [list(map(int, l.split())) for l in lines[1:1 + m]]
    head = lines[1 + m].split()
    assert head[0] == "order"
    return m, n, dc, rows, int(head[1]), [int(x) for x in head[2:]]


def test_compiled_rows_are_the_l63_code(dump):
    m, n, dc, rows, _, _ = dump
    l, a, b = workloads.code("G63")
    hz = codes.gb_matrices(l, a, b)[1]
    assert hz.shape == (m, n) and all(len(r) == dc for r in rows)
    for c in range(m):
        assert sorted(rows[c]) == np.nonzero(hz[c])[0].tolist()


def test_compiled_order_keeps_the_layer_order(dump):
    m, n, _, rows, nlayers, order = dump
    l, a, b = workloads.code("G63")
    hz = codes.gb_matrices(l, a, b)[1]
    lay = layered.greedy_layers(hz)
    assert nlayers == len(lay)
    assert sorted(order) == list(range(m))
    # the flattened first-fit layers, layer by layer
    assert order == [c for layer in lay for c in layer]
    # and, as the property the kernel relies on, every variable meets its
    # checks in layer order
    layer_of = {c: i for i, layer in enumerate(lay) for c in layer}
    seen = {j: -1 for j in range(n)}
    for c in order:
        for j in np.nonzero(hz[c])[0]:
            assert layer_of[c] > seen[j]
            seen[j] = layer_of[c]

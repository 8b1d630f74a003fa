"""Oracle pins: Philox4x32-10, the depolarizing sampler, syndromes, packing.

Philox is pinned against rocRAND's independent implementation, evaluated on
the host by a small helper compiled here; the sampler against binomial
frequency bounds; the syndrome against columns of H_Z and the CSS condition.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import channel, codes, philox

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include", "-O1",
                    os.path.join(HERE, "helpers", "philox_rocrand.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(7)
    vals = rng.integers(0, 2 ** 32, size=(500, 6), dtype=np.uint64)
    vals[0] = 0
    vals[1] = 0xFFFFFFFF
    text = "\n".join(" ".join("%x" % int(v) for v in row) for row in vals) + "\n"
    out = subprocess.run([rocrand_philox], input=text, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t, 16) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    got = np.stack(philox.philox4x32(*[vals[:, i] for i in range(6)]), axis=1)
    assert ref.shape == got.shape
    assert (ref == got).all()


def test_philox_rounds_matter():
    a = philox.philox4x32(1, 2, 3, 4, 5, 6, rounds=10)
    b = philox.philox4x32(1, 2, 3, 4, 5, 6, rounds=9)
    assert any(int(x) != int(y) for x, y in zip(a, b))


def test_thresholds():
    assert channel.thresholds(0.0) == (0, 0, 0)
    tx, ty, tz = channel.thresholds(0.05)
    assert 0 < tx < ty < tz < 2 ** 32
    assert abs(tx / 2 ** 32 - 0.05 / 3) < 2 ** -32
    assert abs(ty / 2 ** 32 - 0.1 / 3) < 2 ** -32
    assert abs(tz / 2 ** 32 - 0.05) < 2 ** -32
    with pytest.raises(ValueError):
        channel.thresholds(1.0)


def test_sampler_frequencies():
    p, n, f = 0.06, 126, 8000
    tx, ty, tz = channel.thresholds(p)
    u = channel.uniforms(1, 2, 1000, f, n)
    N = u.size
    for lo, hi in ((0, tx), (tx, ty), (ty, tz)):
        cnt = int(((u >= lo) & (u < hi)).sum())
        mu = N * p / 3
        assert abs(cnt - mu) < 5 * math.sqrt(mu)
    # top nibble roughly uniform (chi-square, 15 dof, p ~ 1e-6 cut)
    hist = np.bincount((u >> np.uint64(28)).astype(np.int64).ravel(), minlength=16)
    chi2 = (((hist - N / 16) ** 2) / (N / 16)).sum()
    assert chi2 < 60
    ex, ez = channel.sample_paulis(1, 2, 1000, f, n, p)
    assert abs(ex.mean() - 2 * p / 3) < 5 * math.sqrt(2 * p / 3 / N)
    assert abs(ez.mean() - 2 * p / 3) < 5 * math.sqrt(2 * p / 3 / N)
    # Y errors (both bits) at rate p/3
    assert abs((ex & ez).mean() - p / 3) < 5 * math.sqrt(p / 3 / N)


def test_sampler_counter_layout():
    # frames are addressable: a sub-range equals the slice of a bigger draw
    a = channel.uniforms(9, 1, 0, 20, 126)
    b = channel.uniforms(9, 1, 7, 5, 126)
    assert (a[7:12] == b).all()
    # different streams and seeds give different draws
    assert (channel.uniforms(9, 2, 0, 20, 126) != a).any()
    assert (channel.uniforms(10, 1, 0, 20, 126) != a).any()
    # qubit q uses word q mod 4 of call q // 4
    w = philox.philox4x32(2, 5, 0, 1, 9, 0)
    assert int(a[5, 10]) == int(w[2])


def test_syndrome_properties():
    hx, hz = codes.gb_matrices(**codes.G63)
    n = hz.shape[1]
    eye = np.eye(n, dtype=np.uint8)
    assert (channel.syndrome(hz, eye) == hz.T).all()          # weight-1 errors give columns
    assert not channel.syndrome(hz, hx).any()                   # X stabilizers have zero syndrome
    rng = np.random.default_rng(0)
    e1 = rng.integers(0, 2, size=(10, n)).astype(np.uint8)
    e2 = rng.integers(0, 2, size=(10, n)).astype(np.uint8)
    assert (channel.syndrome(hz, e1 ^ e2) == channel.syndrome(hz, e1) ^ channel.syndrome(hz, e2)).all()


def test_pack_unpack():
    rng = np.random.default_rng(1)
    for nb in (1, 63, 64, 65, 126, 1022):
        bits = rng.integers(0, 2, size=(7, nb)).astype(np.uint8)
        pk = channel.pack(bits)
        assert pk.shape == (7, (nb + 63) // 64)
        assert (channel.unpack(pk, nb) == bits).all()
    one = np.zeros((1, 130), dtype=np.uint8)
    one[0, 70] = 1
    assert channel.pack(one)[0].tolist() == [0, 1 << 6, 0]


def test_prior_llr_closed_form():
    # 2p/3 = 1/30 at p = 0.05, so L0 = ln 29
    assert abs(channel.prior_llr(0.05) - math.log(29.0)) < 1e-12
    assert abs(channel.prior_llr(0.03) - math.log(49.0)) < 1e-12

"""Workload definitions and seeded input generators shared by the tests,
the bench and the oracle side of the parity checks.

Holds none of the decoding method's arithmetic: only code exponents (read
from codes.json, written by make_codes.py with the oracle), noise grids,
seeds / Philox stream assignment, and NumPy-seeded arbitrary syndromes for
edge-case decoding inputs.
"""
from __future__ import annotations

import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(_HERE, "codes.json")) as _fh:
    CODES = json.load(_fh)

# The l = 63 sweep: 2^20 frames per point over p = 0.02 .. 0.10, l_max = 100.
P_GRID = [0.02, 0.03, 0.04, 0.05, 0.06, 0.07, 0.08, 0.09, 0.10]
SWEEP_FRAMES = 1 << 20
SWEEP_LMAX = 100
SWEEP_SEED = 1
SMS_ALPHAS = [0.5, 0.625, 0.75, 0.875]
SAGMS_PARAMS = dict(alpha_min=0.30, alpha_max=0.50, eta=1.10)   # Section V setup

# The CPU calibration case: l = 63, p = 0.05, seed 1, stream 0, 10^4 frames, l_max = 50.
CALIB = dict(code="G63", p=0.05, seed=1, stream=0, frames=10_000, lmax=50)


# The mixed-code workload: 2^22 frames split 40 / 30 / 20 / 10 % over four GB
# codes of different length and degree (each share rounded to the nearest
# frame; the four sum to exactly 2^22), p = 0.04, l_max = 100.
MIX_CODES = ["G127", "G255w3", "G255w4", "G63"]
MIX_SHARES = [0.4, 0.3, 0.2, 0.1]
MIX_TOTAL = 1 << 22
MIX_FRAMES = [int(round(f * MIX_TOTAL)) for f in MIX_SHARES]
MIX_P = 0.04
MIX_LMAX = 100
MIX_SEED = 3
# The reduced-precision study runs the same mix at these noise levels.
PRECISION_P = [0.03, 0.05]


# The serving workload: requests of U{1..64} syndromes from one of five codes
# chosen uniformly, Poisson arrivals (seed 5), p = 0.04, l_max = 100.
SERVE_CODES = ["G63", "G127", "G255w3", "G255w4", "G511w5"]
SERVE_P = 0.04
SERVE_LMAX = 100
SERVE_SEED = 5
SERVE_MAX_FRAMES = 64
SERVE_LOADS = [0.5, 0.8]     # offered load, fraction of the measured batch throughput


def serve_trace(rate_per_s: float, nreq: int, seed: int = SERVE_SEED):
    """(code index, frames, arrival time in us) of nreq requests: Poisson
    arrivals at rate_per_s, codes uniform over SERVE_CODES, sizes U{1..64}."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1e6 / rate_per_s, nreq)
    code = rng.integers(0, len(SERVE_CODES), nreq).astype(np.int32)
    size = rng.integers(1, SERVE_MAX_FRAMES + 1, nreq).astype(np.int32)
    return code, size, np.cumsum(gaps)


def serve_stream(i: int) -> int:
    """Philox stream of the frame pool of serving code i."""
    return 200 + i


def mix_stream(i: int, p: float) -> int:
    """Philox stream of mix segment i at noise level p (distinct per pair)."""
    return 100 + 10 * i + int(round(p * 100))


def stream_of(p: float) -> int:
    """Philox stream of a sweep point: the index of p in the grid."""
    return P_GRID.index(p)


def code(name: str) -> tuple[int, list[int], list[int]]:
    c = CODES[name]
    return c["l"], list(c["a"]), list(c["b"])


def random_syndromes(m: int, nframes: int, seed: int, density: float = 0.5) -> np.ndarray:
    """Arbitrary syndrome bits [nframes, m] (uint8), not necessarily reachable by
    low-weight errors; frame 0 is all zero and frame 1 all one when nframes >= 2."""
    rng = np.random.default_rng(seed)
    s = (rng.random((nframes, m)) < density).astype(np.uint8)
    if nframes >= 2:
        s[0] = 0
        s[1] = 1
    return s

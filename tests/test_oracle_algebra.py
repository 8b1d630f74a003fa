"""Oracle pins: GF(2) algebra, GB codes, logical basis, judge.

Pinned against brute force over all vectors of small spaces and against the
paper's [[126,28]] code dimension (Section V setup).
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import codes, gf2, judge

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _span(rows):
    """All GF(2) combinations of the given rows, as a set of tuples."""
    rows = np.asarray(rows, dtype=np.uint8)
    out = set()
    for coef in itertools.product((0, 1), repeat=rows.shape[0]):
        v = np.zeros(rows.shape[1], dtype=np.uint8)
        for c, r in zip(coef, rows):
            if c:
                v ^= r
        out.add(tuple(int(x) for x in v))
    return out


@pytest.mark.parametrize("seed", range(12))
def test_rank_and_nullspace_brute_force(seed):
    rng = np.random.default_rng(seed)
    r, c = rng.integers(1, 7), rng.integers(1, 9)
    a = rng.integers(0, 2, size=(r, c)).astype(np.uint8)
    span = _span(a)
    assert len(span) == 2 ** gf2.rank(a)
    kernel = {v for v in itertools.product((0, 1), repeat=c)
              if not ((np.array(v) @ a.T.astype(int)) & 1).any()}
    ns = gf2.nullspace(a)
    assert len(kernel) == 2 ** ns.shape[0]
    assert _span(ns) == kernel if ns.shape[0] else kernel == {tuple([0] * c)}
    for v in itertools.product((0, 1), repeat=c):
        assert gf2.in_rowspace(a, np.array(v)) == (tuple(v) in span)


def test_g63_is_the_papers_126_28_code():
    hx, hz = codes.gb_matrices(**codes.G63)
    assert hx.shape == (63, 126) and hz.shape == (63, 126)
    assert not ((hx.astype(int) @ hz.T.astype(int)) & 1).any()          # CSS condition
    assert (hz.sum(axis=1) == 10).all() and (hz.sum(axis=0) == 5).all()  # d_c = 10, d_v = 5
    assert gf2.rank(hx) == 49 and gf2.rank(hz) == 49
    assert codes.dimension(hx, hz) == GOLD["gb126_k"]["value"]


def test_g127_dimension():
    hx, hz = codes.gb_matrices(**codes.G127)
    assert not ((hx.astype(int) @ hz.T.astype(int)) & 1).any()
    assert codes.dimension(hx, hz) == 28


def test_circulant_convention():
    a = codes.circulant(5, (0, 2))
    # row i is x^i a(x): ones at columns i and i+2 (mod 5)
    assert a[0].tolist() == [1, 0, 1, 0, 0]
    assert a[4].tolist() == [0, 1, 0, 0, 1]


@pytest.mark.parametrize("code", [dict(l=7, a=(0, 1), b=(0, 2)), dict(l=7, a=(0, 1, 3), b=(0, 2, 6))])
def test_logical_basis_brute_force_14_qubits(code):
    hx, hz = codes.gb_matrices(**code)
    lz = codes.logical_basis(hz, hx)
    k = codes.dimension(hx, hz)
    assert lz.shape[0] == k
    stab = _span(hx)
    for v in itertools.product((0, 1), repeat=hz.shape[1]):
        r = np.array(v, dtype=np.uint8)
        if ((hz.astype(int) @ r) & 1).any():
            continue                                  # only residuals with zero syndrome
        harmless = tuple(v) in stab
        assert harmless == (not ((lz.astype(int) @ r) & 1).any())


def test_small_code_dimensions():
    assert codes.dimension(*codes.gb_matrices(7, (0, 1), (0, 2))) == 2
    assert codes.dimension(*codes.gb_matrices(7, (0, 1, 3), (0, 2, 6))) == 6


def test_rank_and_logical_judges_agree():
    hx, hz = codes.gb_matrices(**codes.G63)
    lz = codes.logical_basis(hz, hx)
    rng = np.random.default_rng(3)
    # residuals that are stabilizers, logical operators and their sums
    stabs = (rng.integers(0, 2, size=(40, 63)) @ hx.astype(int)) & 1
    logs = (rng.integers(0, 2, size=(40, lz.shape[0])) @ lz.astype(int)) & 1
    r = np.vstack([stabs, logs, stabs ^ logs]).astype(np.uint8)
    ex = rng.integers(0, 2, size=r.shape).astype(np.uint8)
    ehat = ex ^ r
    conv = np.ones(r.shape[0], dtype=bool)
    conv[::7] = False
    a = judge.judge_rank(hx, ex, ehat, conv)
    b = judge.judge_logical(lz, ex, ehat, conv)
    assert (a == b).all()
    assert a[:40][conv[:40]].sum() == 0          # stabilizer residuals succeed


def test_draw_gb_reading():
    a, b, k, draws = codes.draw_gb(15, 3, seed=1)
    assert len(a) == 3 and len(b) == 3 and k >= 2
    assert codes.draw_gb(15, 3, seed=1) == (a, b, k, draws)
    assert codes.dimension(*codes.gb_matrices(15, a, b)) == k


@pytest.mark.parametrize("code", [codes.G63, codes.G127, dict(l=7, a=(0, 1, 3), b=(0, 2, 6))])
def test_gb_var_checks_are_the_columns_of_hz(code):
    hx, hz = codes.gb_matrices(**code)
    order = codes.gb_var_checks(**code)
    for j in range(hz.shape[1]):
        assert sorted(order[j]) == sorted(np.nonzero(hz[:, j])[0].tolist())

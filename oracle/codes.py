"""Generalized-bicycle (GB) CSS codes (test oracle).

A GB code of circulant size l is given by two polynomials a(x), b(x) over
GF(2) modulo x^l - 1 (Section II: codes of the generalized bicycle family;
Section V setup: the [[126,28]] GB code).  Convention used throughout this
project: the circulant of a(x) is the l x l matrix with

    A[i][j] = 1  iff  (j - i) mod l  is an exponent of a(x),

so row i is x^i a(x).  Then H_X = [A | B], H_Z = [B^T | A^T], n = 2l, and
H_X H_Z^T = AB + BA = 0 because circulants commute.  The X part of an error
is decoded on the Tanner graph of H_Z (its syndrome), and a residual is
harmless iff it lies in the rowspace of H_X.

Pinned by: H_X H_Z^T = 0, row/column weights, and k = 28 for the l = 63 code
(the paper's [[126,28]] code).
"""
from __future__ import annotations

import numpy as np

from . import gf2

# The l = 63 code of the paper's simulations (Section V setup) and the l = 127
# code of the mixed-size workload, as exponent lists of a(x) and b(x).
G63 = dict(l=63, a=(0, 1, 14, 16, 22), b=(0, 3, 13, 20, 42))
G127 = dict(l=127, a=(0, 15, 20, 28, 66), b=(0, 58, 59, 100, 121))


def circulant(l: int, exps) -> np.ndarray:
    """l x l circulant with A[i][j] = 1 iff (j - i) mod l is in exps."""
    a = np.zeros((l, l), dtype=np.uint8)
    for i in range(l):
        for e in exps:
            a[i, (i + e) % l] ^= 1
    return a


def gb_matrices(l: int, a, b) -> tuple[np.ndarray, np.ndarray]:
    """(H_X, H_Z) = ([A | B], [B^T | A^T]) of the GB code (a, b)."""
    A = circulant(l, a)
    B = circulant(l, b)
    hx = np.hstack([A, B])
    hz = np.hstack([B.T, A.T])
    return hx, hz


def gb_var_checks(l: int, a, b) -> list[list[int]]:
    """Checks of every variable of H_Z = [B^T | A^T], in polynomial-term order.

    Variable i of the first block meets check (i + b_t) mod l for each term
    b_t of b(x), variable l + i of the second block meets (i + a_t) mod l;
    listed in the order of the exponents as given.  This is the order in
    which a GB graph's FP32 posterior sums are taken.
    """
    first = [[(i + t) % l for t in b] for i in range(l)]
    second = [[(i + t) % l for t in a] for i in range(l)]
    return first + second


def dimension(hx, hz) -> int:
    """k = n - rank H_X - rank H_Z of a CSS code."""
    n = np.asarray(hx).shape[1]
    return n - gf2.rank(hx) - gf2.rank(hz)


def logical_basis(h_dec, h_other) -> np.ndarray:
    """Basis of ker(h_other) modulo rowspace(h_dec), k rows.

    When X errors are decoded on h_dec = H_Z, a residual r with H_Z r = 0
    is a stabilizer (harmless) iff r is in rowspace(H_X) = ker(H_X)^perp,
    i.e. iff r is orthogonal to ker(H_X); since r is already orthogonal to
    rowspace(H_Z) it suffices to test the rows returned here.
    """
    kernel = gf2.nullspace(h_other)
    acc = np.array(h_dec, dtype=np.uint8)
    acc_rank = gf2.rank(acc)
    picked = []
    for v in kernel:
        trial = np.vstack([acc, v[None, :]])
        r = gf2.rank(trial)
        if r > acc_rank:
            acc, acc_rank = trial, r
            picked.append(v)
    n = np.asarray(h_dec).shape[1]
    return np.array(picked, dtype=np.uint8).reshape(len(picked), n)


def draw_gb(l: int, w: int, seed: int, min_k: int = 2, max_draws: int = 100000):
    """Random weight-w GB pair drawn from `seed`, redrawn until k >= min_k.

    The paper gives no procedure for random exponents; this project's
    reading: a NumPy Generator seeded with `seed` draws w distinct exponents
    of a(x), then w of b(x) (each sorted), and keeps drawing pairs from the
    same stream until the code has k >= min_k.  Returns (a, b, k, draws).
    """
    rng = np.random.default_rng(seed)
    for t in range(1, max_draws + 1):
        a = tuple(sorted(int(v) for v in rng.choice(l, w, replace=False)))
        b = tuple(sorted(int(v) for v in rng.choice(l, w, replace=False)))
        hx, hz = gb_matrices(l, a, b)
        k = dimension(hx, hz)
        if k >= min_k:
            return a, b, k, t
    raise RuntimeError("no GB pair with k >= %d in %d draws" % (min_k, max_draws))

"""GF(2) linear algebra on dense 0/1 NumPy matrices (test oracle).

Used for the code dimension k = n - rank H_X - rank H_Z of a CSS code
(Section II, system model) and for the logical-failure judge (decoding
succeeds only if the residual error is a stabilizer, i.e. lies in the
rowspace of the other check matrix).  Plain Gaussian elimination, no
bit-packing.  Pinned by brute force over all vectors of small matrices.
"""
from __future__ import annotations

import numpy as np


def _as_gf2(a) -> np.ndarray:
    m = np.array(a, dtype=np.uint8, copy=True) & 1
    if m.ndim == 1:
        m = m[None, :]
    return m


def row_echelon(a) -> tuple[np.ndarray, list[int]]:
    """Reduced row-echelon form over GF(2) and the list of pivot columns."""
    m = _as_gf2(a)
    rows, cols = m.shape
    pivots: list[int] = []
    r = 0
    for c in range(cols):
        if r == rows:
            break
        nz = np.nonzero(m[r:, c])[0]
        if nz.size == 0:
            continue
        p = r + nz[0]
        if p != r:
            m[[r, p]] = m[[p, r]]
        # eliminate column c from every other row (reduced form)
        hit = np.nonzero(m[:, c])[0]
        hit = hit[hit != r]
        if hit.size:
            m[hit] ^= m[r]
        pivots.append(c)
        r += 1
    return m[:r], pivots


def rank(a) -> int:
    """Rank over GF(2)."""
    return len(row_echelon(a)[1])


def nullspace(a) -> np.ndarray:
    """Basis (rows) of {x : A x = 0 over GF(2)}."""
    m = _as_gf2(a)
    cols = m.shape[1]
    rref, piv = row_echelon(m)
    free = [c for c in range(cols) if c not in set(piv)]
    basis = np.zeros((len(free), cols), dtype=np.uint8)
    for t, f in enumerate(free):
        basis[t, f] = 1
        for r, pc in enumerate(piv):
            basis[t, pc] = rref[r, f]
    return basis


def in_rowspace(a, v) -> bool:
    """True iff v is a GF(2) combination of the rows of A (rank test)."""
    return rank(np.vstack([_as_gf2(a), _as_gf2(v)])) == rank(a)


def matvec(a, x) -> np.ndarray:
    """A x over GF(2); x may be a batch of row vectors [F, cols]."""
    a = _as_gf2(a).astype(np.int64)
    x = np.asarray(x, dtype=np.int64)
    return ((x @ a.T) & 1).astype(np.uint8)

"""Logical-failure judge (test oracle).

Decoding succeeds when the residual syndrome is zero (Section II, after
eq. (resid)).  This project also counts a converged frame as a logical
failure when the residual error r = e_x xor e_hat is not a stabilizer, i.e.
not in the rowspace of the other check matrix H_X.  Two forms:

  judge_rank     fail iff not converged, or rank [H_X; r] > rank H_X
                 (plain GF(2) rank test, one elimination per frame)
  judge_logical  fail iff not converged, or L r != 0 over GF(2), where L is
                 a basis of ker(H_X) modulo rowspace(H_Z)
                 (codes.logical_basis); equivalent whenever H_Z r = 0.
"""
from __future__ import annotations

import numpy as np

from . import gf2


def judge_rank(h_other, ex, ehat, converged) -> np.ndarray:
    ex = np.asarray(ex, dtype=np.uint8)
    ehat = np.asarray(ehat, dtype=np.uint8)
    fail = ~np.asarray(converged, dtype=bool)
    base = gf2.rank(h_other)
    for f in range(ex.shape[0]):
        if fail[f]:
            continue
        r = ex[f] ^ ehat[f]
        if r.any() and gf2.rank(np.vstack([h_other, r[None, :]])) > base:
            fail[f] = True
    return fail


def judge_logical(lbasis, ex, ehat, converged) -> np.ndarray:
    r = (np.asarray(ex, dtype=np.int64) ^ np.asarray(ehat, dtype=np.int64))
    lb = np.asarray(lbasis, dtype=np.int64)
    bad = ((r @ lb.T) & 1).any(axis=1) if lb.size else np.zeros(r.shape[0], dtype=bool)
    return ~np.asarray(converged, dtype=bool) | bad

"""Closed forms of the paper's analysis (test oracle; not on the decode path).

  transfer functions       eq. (transfer_all): CN output magnitude when all
                           d_c - 1 inputs equal kappa (uniform message
                           approximation)
  BP-matching ratio        eq. (alphastar), exact and large-L0 forms
  scalability penalty      eq. (mismatch), Proposition 1
  weighted op count        eq. (complexity) and Table 1, weights (1,1,1,10)
"""
from __future__ import annotations

import math


def phi(x: float) -> float:
    """Gallager phi(x) = -ln tanh(x/2), an involution on (0, inf)."""
    return -math.log(math.tanh(x / 2.0))


def t_bp(kappa: float, dc: int) -> float:
    """T_BP4(kappa) = phi^-1((d_c - 1) phi(kappa)), with phi^-1 = phi."""
    return phi((dc - 1) * phi(kappa))


def t_ms(kappa: float) -> float:
    return kappa


def t_sms(kappa: float, alpha: float) -> float:
    return alpha * kappa


def t_sagms(kappa: float, alpha_eff: float) -> float:
    return alpha_eff * kappa


def alpha_star(l0: float, dc: int) -> float:
    """Exact BP-matching ratio (2 / L0) atanh(tanh(L0/2)^(d_c - 1))."""
    return 2.0 * math.atanh(math.tanh(l0 / 2.0) ** (dc - 1)) / l0


def alpha_star_approx(l0: float, dc: int) -> float:
    """Large-L0 form 1 - ln(d_c - 1) / L0 (uses phi(x) ~ 2 e^-x)."""
    return 1.0 - math.log(dc - 1) / l0


def delta_alpha(dc_ref: int, dc_new: int, l0: float) -> float:
    """Scalability penalty ln((d_new - 1)/(d_ref - 1)) / L0, eq. (mismatch)."""
    return math.log((dc_new - 1) / (dc_ref - 1)) / l0


def gf4_prior(eps0: float) -> float:
    """The paper's GF(4) prior L0 = ln((1 - e0)/(e0/3)) (Section II notation)."""
    return math.log((1.0 - eps0) / (eps0 / 3.0))


# Table 1 rows: (additions, multiplications, comparisons, transcendentals)
def table1_ops(dc: int) -> dict:
    return {
        "BP4": (dc - 2, dc - 1, 0, 2 * dc - 1),
        "MS": (0, dc - 1, dc - 2, 0),
        "SAGMS": (3, dc + 1, dc - 1, 0),
    }


def weighted_cost(ops, weights=(1, 1, 1, 10)) -> int:
    return sum(o * w for o, w in zip(ops, weights))


def complexity(dc: int) -> dict:
    """Per-CN-output weighted cost of eq. (complexity); SMS = MS + one scale."""
    rows = table1_ops(dc)
    ms = weighted_cost(rows["MS"])
    return {"BP4": weighted_cost(rows["BP4"]), "SMS": ms + 1, "SAGMS": weighted_cost(rows["SAGMS"])}

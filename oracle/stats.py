"""Monte Carlo statistics (test oracle).

Section V setup: FER points are reported with a 95 % Wilson score interval;
Section V results quote a two-sample log-ratio interval for the ratio of
two FERs.  The Wilson interval is pinned by its closed form at the paper's
stopping rule (500 failures give about +-9 % relative half-width).
"""
from __future__ import annotations

import math

Z95 = 1.959963984540054  # two-sided 95 % standard-normal quantile


def wilson(failures: int, frames: int, z: float = Z95) -> tuple[float, float]:
    """Wilson score interval (lo, hi) for a binomial proportion."""
    if frames <= 0:
        raise ValueError("frames must be positive")
    phat = failures / frames
    z2 = z * z
    denom = 1.0 + z2 / frames
    centre = (phat + z2 / (2.0 * frames)) / denom
    half = (z / denom) * math.sqrt(phat * (1.0 - phat) / frames + z2 / (4.0 * frames * frames))
    return max(0.0, centre - half), min(1.0, centre + half)


def log_ratio_interval(f1: int, n1: int, f2: int, n2: int, z: float = Z95) -> tuple[float, float, float]:
    """Ratio FER1/FER2 with the log-method (Katz) interval: (ratio, lo, hi)."""
    if min(f1, f2) <= 0:
        raise ValueError("both samples need at least one failure")
    p1, p2 = f1 / n1, f2 / n2
    ratio = p1 / p2
    se = math.sqrt((1.0 - p1) / f1 + (1.0 - p2) / f2)
    return ratio, ratio * math.exp(-z * se), ratio * math.exp(z * se)

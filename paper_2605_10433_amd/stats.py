"""Reporting statistics of the Monte Carlo frame-error rate (host side).

FER points carry a 95 % Wilson score interval, as in the paper's setup
(Section V): the interval is the set of proportions q whose score statistic
|phat - q| / sqrt(q (1 - q) / n) is at most z, i.e. the roots of a quadratic.
"""
import math

Z95 = 1.959963984540054


def wilson(failures: int, frames: int, z: float = Z95):
    """95 % Wilson score interval (lo, hi) of failures / frames."""
    if frames <= 0:
        raise ValueError("frames must be positive")
    n, x = float(frames), float(failures)
    # (n + z^2) q^2 - (2x + z^2) q + x^2 / n = 0
    qa = n + z * z
    qb = 2.0 * x + z * z
    qc = x * x / n
    disc = max(qb * qb - 4.0 * qa * qc, 0.0)
    root = math.sqrt(disc)
    return max(0.0, (qb - root) / (2.0 * qa)), min(1.0, (qb + root) / (2.0 * qa))


def fer_ratio_interval(f1: int, n1: int, f2: int, n2: int, z: float = Z95):
    """FER1 / FER2 with the 95 % log-method interval of the ratio of two
    binomial proportions (Section V reports a FER ratio with such an
    interval): log(ratio) +- z * sqrt(1/f1 - 1/n1 + 1/f2 - 1/n2).
    Returns (ratio, lo, hi); both samples need a failure."""
    if f1 < 1 or f2 < 1:
        raise ValueError("both samples need at least one failure")
    lr = math.log(f1) - math.log(n1) - math.log(f2) + math.log(n2)
    se = math.sqrt(1.0 / f1 - 1.0 / n1 + 1.0 / f2 - 1.0 / n2)
    return math.exp(lr), math.exp(lr - z * se), math.exp(lr + z * se)

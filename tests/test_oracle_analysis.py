"""Oracle pins: the paper's printed analytical numbers (Sections IV and V)."""
import json
import math
import os

import pytest

from oracle import analysis, stats

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_gf4_prior_value():
    g = GOLD["gf4_prior_eps0"]
    assert analysis.gf4_prior(g["value"]) == pytest.approx(g["L0_printed"], abs=g["tol"])


@pytest.mark.parametrize("key", ["alpha_star_approx_dc10", "alpha_star_approx_dc16"])
def test_alpha_star_printed(key):
    g = GOLD[key]
    l0 = analysis.gf4_prior(0.10)
    assert analysis.alpha_star_approx(l0, g["dc"]) == pytest.approx(g["value"], abs=g["tol"])


def test_delta_alpha_and_sms_excess():
    l0 = analysis.gf4_prior(0.10)
    g = GOLD["delta_alpha_10_16"]
    assert analysis.delta_alpha(10, 16, l0) == pytest.approx(g["value"], abs=g["tol"])
    # the penalty is the difference of the large-L0 forms (Proposition 1 proof)
    assert analysis.delta_alpha(10, 16, l0) == pytest.approx(
        analysis.alpha_star_approx(l0, 10) - analysis.alpha_star_approx(l0, 16), rel=1e-12)
    e = GOLD["sms_excess_over_alpha_star_dc16"]
    assert e["alpha"] - analysis.alpha_star_approx(l0, 16) == pytest.approx(e["value"], abs=e["tol"])


@pytest.mark.parametrize("l0", [1.5, 2.64, 3.2958, 4.3, 7.0])
def test_alpha_star_exact_decreases_in_dc(l0):
    # Proposition 1, checked on the exact form (not only its approximation)
    vals = [analysis.alpha_star(l0, dc) for dc in range(2, 30)]
    assert vals[0] == pytest.approx(1.0)
    assert all(b < a for a, b in zip(vals, vals[1:]))
    # exact alpha* is the BP transfer function at kappa = L0 divided by L0
    for dc in (4, 10, 16):
        assert analysis.alpha_star(l0, dc) == pytest.approx(analysis.t_bp(l0, dc) / l0, rel=1e-9)


def test_alpha_star_approx_is_large_l0_limit():
    # the neglected terms are O(exp(-L0)); at L0 = 20 they are below 1e-6
    for dc in (4, 10, 16):
        assert analysis.alpha_star(20.0, dc) == pytest.approx(analysis.alpha_star_approx(20.0, dc), abs=1e-6)
        assert abs(analysis.alpha_star(3.0, dc) - analysis.alpha_star_approx(3.0, dc)) > 1e-4


def test_complexity_table():
    g = GOLD["complexity_dc10"]
    c = analysis.complexity(g["dc"])
    assert (c["BP4"], c["SMS"], c["SAGMS"]) == (g["BP4"], g["SMS"], g["SAGMS"])
    for dc in range(2, 20):
        c = analysis.complexity(dc)
        assert c == {"BP4": 22 * dc - 13, "SMS": 2 * dc - 2, "SAGMS": 2 * dc + 3}


def test_wilson_half_width_at_500_failures():
    g = GOLD["wilson_500"]
    for frames in (10 ** 4, 10 ** 5, 10 ** 6, 2 * 10 ** 7):
        lo, hi = stats.wilson(g["failures"], frames)
        fer = g["failures"] / frames
        assert (hi - lo) / 2 / fer <= g["max_rel_half_width"]
    # and the Wilson interval covers its point estimate, shrinking with n
    lo1, hi1 = stats.wilson(5, 100)
    lo2, hi2 = stats.wilson(50, 1000)
    assert lo1 < 0.05 < hi1 and (hi2 - lo2) < (hi1 - lo1)


def test_wilson_matches_scipy_binomtest():
    from scipy.stats import binomtest
    for x, n in ((0, 50), (3, 100), (500, 10 ** 6), (97, 97)):
        ci = binomtest(x, n).proportion_ci(confidence_level=0.95, method="wilson")
        lo, hi = stats.wilson(x, n)
        assert lo == pytest.approx(ci.low, abs=1e-12) and hi == pytest.approx(ci.high, abs=1e-12)


def test_sagms_setup_satisfies_stability():
    g = GOLD["sagms_setup"]
    assert g["alpha_max"] * g["eta"] == pytest.approx(g["alpha_max_eta"])
    assert g["alpha_max"] * g["eta"] <= 1.0


def test_log_ratio_interval():
    r, lo, hi = stats.log_ratio_interval(400, 10 ** 7, 500, 10 ** 7)
    assert lo < r < hi and r == pytest.approx(0.8)
    assert math.log(hi / r) == pytest.approx(math.log(r / lo))


def test_log_ratio_interval_coverage():
    """The interval's defining property, by simulation: over many pairs of
    binomial samples with known FERs it covers the true ratio about 95 % of
    the time, and its width shrinks as 1 / sqrt(failures)."""
    import numpy as np
    rng = np.random.default_rng(7)
    for q1, q2, n in ((0.01, 0.02, 40_000), (0.2, 0.1, 4_000), (0.05, 0.05, 20_000)):
        f1 = rng.binomial(n, q1, 4000)
        f2 = rng.binomial(n, q2, 4000)
        hit = [lo <= q1 / q2 <= hi for (_, lo, hi) in (stats.log_ratio_interval(a, n, b, n) for a, b in zip(f1, f2))]
        assert 0.935 <= np.mean(hit) <= 0.965
    w1 = stats.log_ratio_interval(100, 10 ** 6, 100, 10 ** 6)
    w4 = stats.log_ratio_interval(400, 4 * 10 ** 6, 400, 4 * 10 ** 6)
    assert math.log(w1[2] / w1[1]) == pytest.approx(2 * math.log(w4[2] / w4[1]), rel=1e-3)

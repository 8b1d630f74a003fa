"""Oracle pins: check-node rules, decoders, exact marginals and ML bounds.

  * CN rules against brute force over the configurations of one check
    (min-sum output = min-marginal difference; BP output = log-ratio of the
    parity-constrained probability sums), and against the closed transfer
    functions of eq. (transfer_all).
  * Decoders on tree-shaped Tanner graphs against exact marginals (BP) and
    exact min-marginals (MS), by enumeration.
  * Brute-force maximum-likelihood decoding of 14-qubit GB codes: every
    decoder's exact FER is at least the ML FER; the Monte Carlo FER of the
    oracle's sampler + decoder lies in the Wilson interval of the exact FER.
  * Special cases and invariants: SMS(1) = MS, SAGMS(a, a, 1) = SMS(a),
    zero syndrome, converged => H e_hat = s, round-1 closed form.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import analysis, channel, codes, decoders, judge, stats
from oracle.decoders import DecoderParams, TannerGraph


# ---------------------------------------------------------------- CN rules
def _configs(d, parity):
    return [c for c in itertools.product((0, 1), repeat=d) if sum(c) % 2 == parity]


def brute_cn_minsum(llrs, s):
    """Min-sum CN message to one edge: min cost with x_j = 1 minus x_j = 0."""
    def best(par):
        return min(sum(x * l for x, l in zip(c, llrs)) for c in _configs(len(llrs), par))
    # x_j = 0 needs the others' parity = s, x_j = 1 needs s xor 1
    return best(s ^ 1) - best(s)


def brute_cn_bp(llrs, s):
    p1 = [1.0 / (1.0 + math.exp(l)) for l in llrs]     # P(x = 1) from the LLR

    def mass(par):
        return sum(math.prod(p if x else 1 - p for x, p in zip(c, p1)) for c in _configs(len(llrs), par))
    return math.log(mass(s) / mass(s ^ 1))


@pytest.mark.parametrize("seed", range(30))
def test_cn_minsum_brute_force(seed):
    rng = np.random.default_rng(seed)
    d = int(rng.integers(2, 9))
    v = rng.normal(0, 3, size=d)
    if seed % 3 == 0:                       # exact ties and zeros
        v[: d // 2] = np.round(v[: d // 2])
        v[0] = 0.0
        v[-1] = -abs(v[1])
    s = int(rng.integers(0, 2))
    out = decoders.cn_minsum(v[None, None, :], np.array([[s]]), np.ones((1, 1)))[0, 0]
    for j in range(d):
        ref = brute_cn_minsum([v[k] for k in range(d) if k != j], s)
        if ref == 0.0:
            assert out[j] == 0.0
        else:
            assert out[j] == pytest.approx(ref, abs=1e-12)


@pytest.mark.parametrize("seed", range(20))
def test_cn_bp_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 8))
    v = rng.normal(0, 2.5, size=d)
    s = int(rng.integers(0, 2))
    out = decoders.cn_bp(v[None, None, :], np.array([[s]]))[0, 0]
    for j in range(d):
        ref = brute_cn_bp([v[k] for k in range(d) if k != j], s)
        assert out[j] == pytest.approx(ref, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("dc", [2, 4, 10, 16])
@pytest.mark.parametrize("kappa", [0.3, 1.0, 3.37, 8.0])
def test_cn_transfer_functions(dc, kappa):
    # eq. (transfer_all): every other input equal to kappa (UMA)
    v = np.full((1, 1, dc), kappa)
    s0 = np.zeros((1, 1), dtype=np.uint8)
    assert decoders.cn_minsum(v, s0, np.ones((1, 1)))[0, 0, 0] == kappa
    assert decoders.cn_minsum(v, s0, np.full((1, 1), 0.75))[0, 0, 0] == pytest.approx(0.75 * kappa)
    bp = decoders.cn_bp(v, s0)[0, 0, 0]
    assert bp == pytest.approx(analysis.t_bp(kappa, dc), rel=1e-9)
    assert bp <= kappa                       # T_BP4 <= kappa (Section II)
    # syndrome bit flips the sign
    assert decoders.cn_minsum(v, np.ones((1, 1), dtype=np.uint8), np.ones((1, 1)))[0, 0, 0] == -kappa


def test_bp_output_cap():
    v = np.full((1, 1, 4), 60.0)
    out = decoders.cn_bp(v, np.zeros((1, 1), dtype=np.uint8))[0, 0, 0]
    assert np.isfinite(out) and out == pytest.approx(2 * math.atanh(1 - 2.0 ** -40), rel=1e-6)


# ------------------------------------------------------- tree-shaped graphs
def random_tree_graph(rng, checks):
    """Tanner graph with no cycles: each new check meets one old variable."""
    rows, nvar = [], 0
    first = int(rng.integers(2, 4))
    rows.append(list(range(first)))
    nvar = first
    for _ in range(checks - 1):
        anchor = int(rng.integers(0, nvar))
        new = int(rng.integers(1, 3))
        rows.append([anchor] + list(range(nvar, nvar + new)))
        nvar += new
    h = np.zeros((checks, nvar), dtype=np.uint8)
    for i, r in enumerate(rows):
        h[i, r] = 1
    return h


def exact_marginals(h, s, llr):
    m, n = h.shape
    lp = np.full(n, -np.inf)
    lq = np.full(n, -np.inf)
    best1 = np.full(n, np.inf)
    best0 = np.full(n, np.inf)
    for e in itertools.product((0, 1), repeat=n):
        e = np.array(e)
        if (((h.astype(int) @ e) & 1) != s).any():
            continue
        logp = sum(-math.log1p(math.exp(l)) if x else -math.log1p(math.exp(-l)) for x, l in zip(e, llr))
        cost = float((e * llr).sum())
        for j in range(n):
            if e[j]:
                lq[j] = np.logaddexp(lq[j], logp)
                best1[j] = min(best1[j], cost)
            else:
                lp[j] = np.logaddexp(lp[j], logp)
                best0[j] = min(best0[j], cost)
    return lp - lq, best1 - best0


@pytest.mark.parametrize("seed", range(12))
def test_tree_bp_exact_and_ms_min_marginals(seed):
    rng = np.random.default_rng(seed)
    h = random_tree_graph(rng, int(rng.integers(3, 6)))
    m, n = h.shape
    assert n <= 16
    e = rng.integers(0, 2, size=n)
    s = ((h.astype(int) @ e) & 1).astype(np.uint8)
    llr = rng.uniform(0.3, 2.5, size=n) * rng.choice([1, 1, 1, -1], size=n)
    lbp, lms = exact_marginals(h, s, llr)
    g = TannerGraph(h)
    rounds = 2 * m + 2                      # beyond the tree's diameter
    rb = decoders.decode(g, s[None], llr, DecoderParams(kind="bp", lmax=rounds), early_exit=False)
    assert np.allclose(rb.posterior[0], lbp, rtol=1e-9, atol=1e-9)
    rm = decoders.decode(g, s[None], llr, DecoderParams(kind="ms", lmax=rounds), early_exit=False)
    assert np.allclose(rm.posterior[0], lms, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------- 14-qubit ML pins
def exact_fers(code, p, params_list):
    hx, hz = codes.gb_matrices(**code)
    n = hz.shape[1]
    lz = codes.logical_basis(hz, hx)
    q = 2 * p / 3
    errs = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.uint8)
    w = errs.sum(axis=1)
    prob = q ** w * (1 - q) ** (n - w)
    synd = channel.syndrome(hz, errs)
    skey = channel.pack(synd)[:, 0]
    cls = channel.pack(((errs.astype(int) @ lz.T.astype(int)) & 1).astype(np.uint8))[:, 0]
    # maximum likelihood: most probable logical class per syndrome
    table = {}
    for sk, c, pr in zip(skey, cls, prob):
        table.setdefault(int(sk), {}).setdefault(int(c), 0.0)
        table[int(sk)][int(c)] += pr
    fer_ml = 1.0 - sum(max(d.values()) for d in table.values())
    # deterministic decoders: decode every distinct syndrome once
    uniq, inv = np.unique(skey, return_inverse=True)
    s_uniq = channel.unpack(uniq[:, None], hz.shape[0])
    g = TannerGraph(hz)
    llr = np.full(n, channel.prior_llr(p))
    out = []
    for prm in params_list:
        r = decoders.decode(g, s_uniq, llr, prm)
        fail = judge.judge_logical(lz, errs, r.ehat[inv], r.converged[inv])
        out.append(float((prob * fail).sum()))
    return fer_ml, out, table, lz, hz


@pytest.mark.parametrize("code", [dict(l=7, a=(0, 1), b=(0, 2)), dict(l=7, a=(0, 1, 3), b=(0, 2, 6))])
def test_ml_lower_bounds_every_decoder(code):
    p = 0.08
    prms = [DecoderParams(kind="ms", lmax=30), DecoderParams(kind="sms", alpha=0.75, lmax=30),
            DecoderParams(kind="sagms", lmax=30), DecoderParams(kind="bp", lmax=30)]
    fer_ml, fers, *_ = exact_fers(code, p, prms)
    assert 0.0 < fer_ml < 0.5
    for f in fers:
        assert f >= fer_ml - 1e-12


def test_ml_corrects_weight_one_on_distance_three_code():
    code = dict(l=7, a=(0, 1), b=(0, 2))
    _, _, table, lz, hz = exact_fers(code, 0.05, [])
    n = hz.shape[1]
    for j in range(n):
        e = np.zeros((1, n), dtype=np.uint8)
        e[0, j] = 1
        sk = int(channel.pack(channel.syndrome(hz, e))[0, 0])
        c = int(channel.pack(((e.astype(int) @ lz.T.astype(int)) & 1).astype(np.uint8))[0, 0])
        best = max(table[sk].items(), key=lambda kv: kv[1])[0]
        assert best == c


def test_monte_carlo_fer_inside_wilson_of_exact():
    code = dict(l=7, a=(0, 1), b=(0, 2))
    p = 0.1
    prm = DecoderParams(kind="sagms", lmax=30)
    _, (fer_exact,), _, lz, hz = exact_fers(code, p, [prm])
    f = 20000
    ex, _ = channel.sample_paulis(11, 0, 0, f, hz.shape[1], p)
    r = decoders.decode(TannerGraph(hz), channel.syndrome(hz, ex), np.full(14, channel.prior_llr(p)), prm)
    fails = int(judge.judge_logical(lz, ex, r.ehat, r.converged).sum())
    lo, hi = stats.wilson(fails, f, z=4.0)
    assert lo <= fer_exact <= hi


# ------------------------------------------------ invariants, special cases
@pytest.fixture(scope="module")
def g63_batch():
    hx, hz = codes.gb_matrices(**codes.G63)
    p = 0.06
    ex, _ = channel.sample_paulis(1, 5, 0, 600, 126, p)
    s = channel.syndrome(hz, ex)
    return TannerGraph(hz), hz, s, np.full(126, channel.prior_llr(p))


@pytest.mark.parametrize("arith", ["fp64", "fp32"])
def test_sms_one_is_ms_and_sagms_constant_is_sms(g63_batch, arith):
    g, hz, s, llr = g63_batch
    a = decoders.decode(g, s, llr, DecoderParams(kind="ms", lmax=40), arith)
    b = decoders.decode(g, s, llr, DecoderParams(kind="sms", alpha=1.0, lmax=40), arith)
    assert (a.ehat == b.ehat).all() and (a.iters == b.iters).all() and (a.posterior == b.posterior).all()
    c = decoders.decode(g, s, llr, DecoderParams(kind="sms", alpha=0.625, lmax=40), arith)
    d = decoders.decode(g, s, llr, DecoderParams(kind="sagms", alpha_min=0.625, alpha_max=0.625,
                                                 eta=1.0, lmax=40), arith)
    assert (c.ehat == d.ehat).all() and (c.iters == d.iters).all() and (c.posterior == d.posterior).all()


@pytest.mark.parametrize("kind", ["ms", "sms", "sagms", "bp"])
@pytest.mark.parametrize("arith", ["fp64", "fp32"])
def test_frame_invariants(g63_batch, kind, arith):
    g, hz, s, llr = g63_batch
    s = s.copy()
    s[:5] = 0                                   # zero syndromes
    prm = DecoderParams(kind=kind, lmax=25)
    r = decoders.decode(g, s, llr, prm, arith)
    assert (r.iters[:5] == 0).all() and not r.ehat[:5].any() and r.converged[:5].all()
    resid = s ^ channel.syndrome(hz, r.ehat)
    assert not resid[r.converged].any()         # converged => H e_hat = s
    assert (r.iters[~r.converged] == prm.lmax).all()
    assert ((r.iters >= 1) | ~s.any(axis=1)).all()


def test_round_one_closed_form(g63_batch):
    # After one round from v2c = L0 (uniform), every CN output is
    # (-1)^{s_i} * prod sgn(L0) * alpha_i * L0 = (-1)^{s_i} alpha_i L0.
    g, hz, s, llr = g63_batch
    prm = DecoderParams(kind="sagms", lmax=1)
    r = decoders.decode(g, s[:20], llr, prm, trace=True, early_exit=False)
    rd = r.trace[0]
    w = s[:20].sum(axis=1)
    gfac = 0.50 - 0.20 * w / 63
    for f in range(20):
        for e in range(g.E):
            i = g.e_check[e]
            a = gfac[f] * (1.10 if s[f, i] else 1.0)
            expect = (-1.0 if s[f, i] else 1.0) * a * llr[0]
            assert rd["c2v"][f, e] == pytest.approx(expect, rel=1e-15)


def test_gain_never_exceeds_one():
    prm = DecoderParams(kind="sagms", alpha_min=0.3, alpha_max=0.5, eta=2.0)
    rng = np.random.default_rng(0)
    sres = rng.integers(0, 2, size=(200, 63)).astype(np.uint8)
    gains = decoders.check_gains(prm, sres, 63)
    assert gains.max() <= 1.0 and gains.min() >= 0.3 - 1e-15
    with pytest.raises(ValueError):
        DecoderParams(kind="sagms", alpha_max=0.6, eta=2.0).validate()


@pytest.mark.parametrize("kind,kw,tol", [("sagms", {}, 1e-5), ("sms", dict(alpha=0.625), 1e-5),
                                         ("ms", {}, 1e-5), ("sms", dict(alpha=0.875), 2e-4)])
def test_fp32_messages_track_fp64(g63_batch, kind, kw, tol):
    """Over the first 10 rounds, FP32 messages stay within tol (relative,
    floor L0) of FP64 on frames whose FP64 trajectory avoids the tie band
    1e-4 L0; tol follows the per-round error gain gain * (d_v - 1)."""
    g, hz, s, llr = g63_batch
    prm = DecoderParams(kind=kind, lmax=10, **kw)
    a = decoders.decode(g, s[:300], llr, prm, "fp64", early_exit=False, trace=True)
    b = decoders.decode(g, s[:300], llr, prm, "fp32", early_exit=False, trace=True)
    L0 = llr[0]
    near = np.zeros(300, dtype=bool)
    for ra in a.trace:
        near |= (np.abs(ra["post"]).min(axis=1) <= 1e-4 * L0) | (np.abs(ra["v2c"]).min(axis=1) <= 1e-4 * L0)
    ok = ~near
    # min-sum posteriors are integer combinations of a uniform L0, so MS frames
    # meet exact zeros (ties) often; the other decoders rarely do
    assert ok.sum() >= (10 if kind == "ms" else 100)
    for ra, rb in zip(a.trace, b.trace):
        assert ((ra["post"][ok] < 0) == (rb["post"][ok] < 0)).all()
        for key in ("c2v", "v2c", "post"):
            x64, x32 = ra[key][ok], rb[key][ok].astype(np.float64)
            assert (np.abs(x64 - x32) <= tol * np.maximum(np.abs(x64), L0)).all(), key


def test_decoder_frame_independence(g63_batch):
    g, hz, s, llr = g63_batch
    prm = DecoderParams(kind="sagms", lmax=30)
    full = decoders.decode(g, s[:64], llr, prm, "fp32")
    part = decoders.decode(g, s[20:40], llr, prm, "fp32")
    assert (full.ehat[20:40] == part.ehat).all() and (full.iters[20:40] == part.iters).all()


def test_min_sum_exact_ties_with_a_short_prior():
    """Min-sum with a uniform prior makes every message an integer combination
    of L0.  When L0 has few significant bits (a float32 value) FP64 sums are
    exact, posteriors hit exact zeros, and with sgn(0) = +1 the decoder
    stalls in many frames; rounding residues (a full-precision FP64 prior, or
    FP32 sums) break those ties instead.  The paper does not address ties;
    this records the reading's consequence."""
    hx, hz = codes.gb_matrices(**codes.G63)
    lz = codes.logical_basis(hz, hx)
    tg = TannerGraph(hz)
    p = 0.05
    ex, _ = channel.sample_paulis(1, 4, 0, 800, 126, p)
    s = channel.syndrome(hz, ex)
    prm = DecoderParams(kind="ms", lmax=100)
    short = np.full(126, channel.prior_llr(p), dtype=np.float32)
    full = np.full(126, channel.prior_llr(p))
    fer = {}
    for name, llr, arith in (("exact", short, "fp64"), ("fp64", full, "fp64"), ("fp32", short, "fp32")):
        r = decoders.decode(tg, s, llr, prm, arith)
        fer[name] = judge.judge_logical(lz, ex, r.ehat, r.converged).mean()
    assert fer["exact"] > 3 * fer["fp64"] and fer["exact"] > 3 * fer["fp32"]
    lo, hi = stats.wilson(int(round(fer["fp64"] * 800)), 800, z=3.0)
    assert lo <= fer["fp32"] <= hi


def test_var_order_changes_only_fp32_rounding():
    """An explicit per-variable check order leaves FP64 results unchanged
    (exclusive sums are definitional) and changes FP32 posteriors by
    rounding only; a bad order is rejected."""
    hx, hz = codes.gb_matrices(**codes.G63)
    ga = TannerGraph(hz)
    gb = TannerGraph(hz, codes.gb_var_checks(**codes.G63))
    p = 0.05
    ex, _ = channel.sample_paulis(1, 4, 0, 300, 126, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(126, channel.prior_llr(p), dtype=np.float32)
    prm = DecoderParams(kind="sagms", lmax=8)
    a64 = decoders.decode(ga, s, llr, prm, "fp64", early_exit=False)
    b64 = decoders.decode(gb, s, llr, prm, "fp64", early_exit=False)
    assert np.allclose(a64.posterior, b64.posterior, rtol=1e-13, atol=1e-12)
    a32 = decoders.decode(ga, s, llr, prm, "fp32", early_exit=False)
    b32 = decoders.decode(gb, s, llr, prm, "fp32", early_exit=False)
    assert (a32.posterior != b32.posterior).any()
    assert np.allclose(a32.posterior, b32.posterior, rtol=1e-4, atol=1e-4 * llr[0])
    bad = codes.gb_var_checks(**codes.G63)
    bad[0] = bad[1]
    with pytest.raises(ValueError):
        TannerGraph(hz, bad)


def test_quantizers():
    x = np.array([0.0, 0.1, 0.125, 0.375, 1.0 / 3, 15.74, 15.9, 100.0, -0.125, -0.375, -7.3], dtype=np.float32)
    q6 = decoders.quantize(x, "int6")
    assert q6.tolist() == [0.0, 0.0, 0.0, 0.5, 0.25, 15.75, 15.75, 15.75, -0.0, -0.5, -7.25]
    assert (np.abs(q6) <= 15.75).all() and ((q6 * 4) == np.round(q6 * 4)).all()
    q16 = decoders.quantize(x, "fp16")
    assert (q16 == x.astype(np.float16).astype(np.float32)).all()
    big = decoders.quantize(np.array([7e4, -1e30, np.float32(65519.0)], dtype=np.float32), "fp16")
    assert big.tolist() == [65504.0, -65504.0, 65504.0]                          # saturating
    assert decoders.quantize(np.float32(1 + 2 ** -11), "fp16") == 1.0          # ties to even
    assert decoders.quantize(np.float32(1 + 3 * 2 ** -11), "fp16") == np.float32(1 + 2 ** -9)


@pytest.mark.parametrize("arith", ["fp16", "int6"])
def test_quantized_modes_track_fp32(g63_batch, arith):
    """Reduced-precision messages: every message lies on the format's grid,
    the FER stays close to FP32, and zero / invariant cases still hold."""
    g, hz, s, llr = g63_batch
    prm = DecoderParams(kind="sagms", lmax=40)
    tr = decoders.decode(g, s[:100], llr, prm, arith, early_exit=False, trace=True)
    for rd in tr.trace:
        for key in ("c2v", "v2c"):
            assert (decoders.quantize(rd[key], arith) == rd[key]).all()
    r = decoders.decode(g, s, llr, prm, arith)
    r32 = decoders.decode(g, s, llr, prm, "fp32")
    assert abs(int(r.converged.sum()) - int(r32.converged.sum())) <= 0.1 * len(s)
    resid = s ^ channel.syndrome(hz, r.ehat)
    assert not resid[r.converged].any()
    with pytest.raises(ValueError):
        decoders.decode(g, s[:2], llr, DecoderParams(kind="bp"), arith)


def test_int6_posteriors_are_exact_sums():
    """int6: posteriors are sums of grid values, computed exactly in FP32."""
    hx, hz = codes.gb_matrices(**codes.G63)
    g = TannerGraph(hz)
    ex, _ = channel.sample_paulis(2, 0, 0, 50, 126, 0.06)
    s = channel.syndrome(hz, ex)
    llr = np.full(126, channel.prior_llr(0.06), dtype=np.float32)
    r = decoders.decode(g, s, llr, DecoderParams(kind="sms", alpha=0.75, lmax=12), "int6", trace=True)
    for rd in r.trace:
        assert ((rd["post"] * 4) == np.round(rd["post"] * 4)).all()


def test_grid24():
    x = np.array([3.5835189, -0.7, 1e-9, -1e-9, 2.0 ** -25, 3 * 2.0 ** -25, 123.456, -0.0], dtype=np.float32)
    y = decoders.grid24(x)
    assert y[0] == x[0] and y[6] == x[6]                                   # |x| >= 1: unchanged
    assert ((y.astype(np.float64) * 2.0 ** 24) == np.round(y.astype(np.float64) * 2.0 ** 24)).all()
    assert y[2] == 0.0 and y[3] == 0.0 and not np.signbit(y[3]) and not np.signbit(y[7])
    assert y[4] == 0.0 and y[5] == 2.0 ** -23                              # ties to even
    assert abs(float(y[1]) - (-0.7)) <= 2.0 ** -25


@pytest.mark.parametrize("arith", ["fp16", "int6"])
def test_check_outputs_need_only_output_rounding(arith):
    """The message rounding is monotone and keeps signs, so a check update on
    rounded v2c messages equals: signs of the unrounded messages, exclusive
    minima of the unrounded magnitudes, rounded, times the gain, rounded.
    Inputs are on the format's grid before rounding (multiples of 2^-24 for
    FP16, of 1/4 for INT6: the values the decoder produces), with ties,
    zeros and magnitudes beyond the format's range."""
    rng = np.random.default_rng(5)
    step = 2.0 ** -24 if arith == "fp16" else 0.25
    for trial in range(300):
        d = int(rng.integers(2, 12))
        scale = [1e-6, 1e-3, 1.0, 30.0, 1e5][trial % 5]
        v = (np.round(rng.normal(0, scale, size=(4, 3, d)) / step) * step).astype(np.float32)
        v[0, 0, :2] = v[0, 0, 2] if d > 2 else v[0, 0, 0]                 # exact ties
        v[1, 1, 0] = 0.0
        v[2, 2, :] = np.abs(v[2, 2, :])
        s = rng.integers(0, 2, size=(4, 3)).astype(np.uint8)
        gain = rng.choice([0.3, 0.5, 0.55, 1.0], size=(4, 3)).astype(np.float32)
        ref = decoders.cn_minsum(decoders.quantize(v, arith), s, gain, arith)
        mag = np.abs(v)
        other = ~np.eye(d, dtype=bool)
        excl = np.where(other, mag[..., None, :], np.inf).min(axis=-1)
        out = decoders.quantize(gain[..., None] * decoders.quantize(excl, arith), arith)
        neg = ((v < 0)[..., None, :] & other).sum(axis=-1) + s[..., None]
        out = np.where(neg & 1, -out, out)
        assert (out.view(np.uint32) == ref.view(np.uint32)).all(), (trial, arith)

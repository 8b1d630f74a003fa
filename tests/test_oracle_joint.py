"""Oracle pins of the joint (quaternary, scalar-message) decoders.

The joint decoders of oracle/joint.py are checked against what the paper and
the mathematics fix, not against themselves:
  * the scalarization against brute-force sums over the four Paulis of one
    qubit (BP: log-ratio of commuting / anticommuting probability; MS: the
    min-marginal difference), and its closed forms under a uniform prior
    (MS: L0 exactly, the message of Algorithm 1's initialisation and
    Remark 1; BP: the binary marginal LLR);
  * BP on tree-shaped quaternary graphs (X, Y and Z entries, non-uniform
    priors) against exact posterior marginals ln P(E_j = I | s) /
    P(E_j = W | s) by enumeration of all 4^n Pauli errors, and MS against
    exact min-marginals;
  * brute-force maximum-likelihood decoding of the [[14,2,3]] GB code in
    joint form (degenerate ML over logical classes, by meet-in-the-middle
    enumeration of all 4^14 errors): every joint decoder's exact FER is at
    least the ML FER, the Monte Carlo FER (Philox frames) lies in the Wilson
    interval of the exact FER, and ML corrects every weight-1 error;
  * Remark 1's round-1 closed forms (min-sum family: outputs +-gain * L0;
    BP: +-T_BP4 of eq. (transfer_all));
  * a reduction: a graph of Z-type rows only, with a positive uniform prior,
    decodes exactly as the binary decoder of decoders.py (dyadic gains and
    integer priors, so both run in exact arithmetic);
  * the [[126,28]] GB code in the overcomplete form of the Section V setup:
    m = 126, d_c = d_v = 10, rows pairwise commuting, 2k = 56 logicals;
  * the two judges agree; converged frames satisfy the syndrome; FP32 mode
    within tolerance of FP64 over the first rounds.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import analysis, channel, codes, decoders, gf2, joint, stats
from oracle.decoders import DecoderParams

PAULIS = (joint.PX, joint.PY, joint.PZ)


def anticommutes(w, p):
    """Two single-qubit Paulis (codes 0..3) anticommute iff both are
    non-identity and different."""
    return w != 0 and p != 0 and w != p


# ------------------------------------------------------------- scalarization
@pytest.mark.parametrize("seed", range(20))
def test_scalarize_brute_force(seed):
    rng = np.random.default_rng(seed)
    g = rng.normal(1.0, 2.0, size=3)
    if seed % 4 == 0:
        g[1] = g[0]                                   # ties
    for p in PAULIS:
        # probabilities relative to I: P(W) / P(I) = exp(-Gamma^W)
        w = {0: 1.0, joint.PX: math.exp(-g[0]), joint.PY: math.exp(-g[1]), joint.PZ: math.exp(-g[2])}
        comm = sum(v for k, v in w.items() if not anticommutes(k, p))
        anti = sum(v for k, v in w.items() if anticommutes(k, p))
        lam_bp = joint.scalarize(g[None, :], np.array([p]), "bp")[0]
        assert lam_bp == pytest.approx(math.log(comm / anti), rel=1e-12, abs=1e-12)
        cost = {0: 0.0, joint.PX: g[0], joint.PY: g[1], joint.PZ: g[2]}
        best_comm = min(v for k, v in cost.items() if not anticommutes(k, p))
        best_anti = min(v for k, v in cost.items() if anticommutes(k, p))
        lam_ms = joint.scalarize(g[None, :], np.array([p]), "ms")[0]
        assert lam_ms == pytest.approx(best_anti - best_comm, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("eps", [0.01, 0.05, 0.1, 0.2])
def test_scalarize_uniform_prior_closed_forms(eps):
    """Uniform prior L0 (Section II): the min-sum message is L0 itself (so
    Algorithm 1's initialisation L_{j->i} = L0 and Remark 1 are literal for
    the min-sum family), and the BP message is the binary marginal LLR of the
    depolarizing channel, ln((1 - 2e/3) / (2e/3))."""
    L0 = joint.depolarizing_prior(eps)
    assert L0 == pytest.approx(math.log(3 * (1 - eps) / eps), rel=1e-15)
    g = np.full((3, 3), L0)
    lam_ms = joint.scalarize(g, np.array(PAULIS), "ms")
    assert (lam_ms == L0).all()
    lam_bp = joint.scalarize(g, np.array(PAULIS), "bp")
    assert lam_bp == pytest.approx(np.full(3, channel.prior_llr(eps)), rel=1e-13)
    assert lam_bp == pytest.approx(np.full(3, math.log((math.exp(L0) + 1) / 2)), rel=1e-13)
    # fp32: exactly L0 as well
    assert (joint.scalarize(g.astype(np.float32), np.array(PAULIS), "ms") == np.float32(L0)).all()


def test_hard_decision_tie_rule():
    """argmin over (I, X, Y, Z) of (0, G^X, G^Y, G^Z), first minimum."""
    rng = np.random.default_rng(3)
    vals = rng.integers(-2, 3, size=(500, 3)).astype(np.float64)
    xh, zh = joint.hard_decision(vals)
    for v, x, z in zip(vals, xh, zh):
        full = [0.0] + list(v)
        best = full.index(min(full))                  # first minimum
        assert x == (best in (joint.PX, joint.PY)) and z == (best in (joint.PY, joint.PZ))


# ----------------------------------------------------------------- trees
def random_tree_graph(rng, nchecks):
    """A tree-shaped quaternary Tanner graph: every check has degree >= 2,
    every new check shares exactly one variable with the graph so far, and
    the edge Paulis are random in {X, Y, Z}."""
    rows = []
    nvar = 0
    for c in range(nchecks):
        d = int(rng.integers(2, 4))
        if c == 0:
            vs = list(range(d))
            nvar = d
        else:
            vs = [int(rng.integers(0, nvar))] + list(range(nvar, nvar + d - 1))
            nvar += d - 1
        rows.append({v: int(rng.integers(1, 4)) for v in vs})
    sx = np.zeros((nchecks, nvar), dtype=np.uint8)
    sz = np.zeros((nchecks, nvar), dtype=np.uint8)
    for i, r in enumerate(rows):
        for v, p in r.items():
            sx[i, v] = p in (joint.PX, joint.PY)
            sz[i, v] = p in (joint.PY, joint.PZ)
    return sx, sz


def all_paulis(n):
    """Every Pauli error on n qubits: (e_x, e_z, codes) arrays [4^n, n]."""
    codes_ = np.array(list(itertools.product(range(4), repeat=n)), dtype=np.int64)
    ex = ((codes_ == joint.PX) | (codes_ == joint.PY)).astype(np.uint8)
    ez = ((codes_ == joint.PY) | (codes_ == joint.PZ)).astype(np.uint8)
    return ex, ez, codes_


def cost_of(codes_, prior):
    """sum_j Lambda_j^{E_j} (Lambda^I = 0): minus log-probability relative to all-I."""
    full = np.hstack([np.zeros((prior.shape[0], 1)), prior])     # [n, 4]
    return full[np.arange(codes_.shape[1])[None, :], codes_].sum(axis=1)


@pytest.mark.parametrize("seed", range(8))
def test_bp_exact_marginals_on_trees(seed):
    rng = np.random.default_rng(100 + seed)
    sx, sz = random_tree_graph(rng, int(rng.integers(2, 5)))
    g = joint.PauliGraph(sx, sz)
    n = g.n
    assert n <= 9
    prior = rng.uniform(0.3, 4.0, size=(n, 3))
    ex, ez, cds = all_paulis(n)
    e0 = int(rng.integers(0, len(cds)))
    s = joint.symplectic_syndrome(sx, sz, ex[e0:e0 + 1], ez[e0:e0 + 1])
    r = joint.decode_joint(g, s, prior, DecoderParams(kind="bp", lmax=2 * g.m + 2), "fp64", early_exit=False)
    syn = joint.symplectic_syndrome(sx, sz, ex, ez)
    ok = (syn == s[0]).all(axis=1)
    w = np.exp(-cost_of(cds[ok], prior))
    for j in range(n):
        pi = w[cds[ok][:, j] == 0].sum()
        for k, W in enumerate(PAULIS):
            pw = w[cds[ok][:, j] == W].sum()
            assert r.gamma[0, j, k] == pytest.approx(math.log(pi / pw), rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("seed", range(8))
def test_ms_exact_min_marginals_on_trees(seed):
    rng = np.random.default_rng(200 + seed)
    sx, sz = random_tree_graph(rng, int(rng.integers(2, 5)))
    g = joint.PauliGraph(sx, sz)
    n = g.n
    prior = np.round(rng.uniform(0.3, 4.0, size=(n, 3)), 3)
    ex, ez, cds = all_paulis(n)
    e0 = int(rng.integers(0, len(cds)))
    s = joint.symplectic_syndrome(sx, sz, ex[e0:e0 + 1], ez[e0:e0 + 1])
    r = joint.decode_joint(g, s, prior, DecoderParams(kind="ms", lmax=2 * g.m + 2), "fp64", early_exit=False)
    syn = joint.symplectic_syndrome(sx, sz, ex, ez)
    ok = (syn == s[0]).all(axis=1)
    c = cost_of(cds[ok], prior)
    for j in range(n):
        ci = c[cds[ok][:, j] == 0].min()
        for k, W in enumerate(PAULIS):
            cw = c[cds[ok][:, j] == W].min()
            assert r.gamma[0, j, k] == pytest.approx(cw - ci, rel=1e-9, abs=1e-9)


# ------------------------------------------------- ML on the [[14,2,3]] code
L7 = dict(l=7, a=(0, 1), b=(0, 2))


def _keys(sx, sz, lops, ex, ez):
    """(syndrome, logical class) of every error as one integer."""
    s = joint.symplectic_syndrome(sx, sz, ex, ez).astype(np.int64)
    n = ex.shape[1]
    cls = ((ez.astype(np.int64) @ lops[:, :n].T.astype(np.int64) +
            ex.astype(np.int64) @ lops[:, n:].T.astype(np.int64)) & 1)
    bits = np.hstack([s, cls])
    return (bits << np.arange(bits.shape[1], dtype=np.int64)).sum(axis=1), s.shape[1], cls.shape[1]


def _wht(v):
    v = v.copy()
    h = 1
    while h < v.size:
        v = v.reshape(-1, 2, h)
        a, b = v[:, 0, :].copy(), v[:, 1, :].copy()
        v[:, 0, :], v[:, 1, :] = a + b, a - b
        v = v.reshape(-1)
        h *= 2
    return v


def class_probabilities(sx, sz, lops, eps):
    """P(syndrome, logical class) of the depolarizing channel, exactly, by
    enumerating the 4^7 errors of each half of the 14 qubits and XOR-
    convolving the two halves' distributions (Walsh-Hadamard transform)."""
    n = sx.shape[1]
    half = n // 2
    ex, ez, cds = all_paulis(half)
    nbits = None
    dists = []
    for side in (0, 1):
        fx = np.zeros((len(cds), n), dtype=np.uint8)
        fz = np.zeros((len(cds), n), dtype=np.uint8)
        cols = slice(0, half) if side == 0 else slice(half, n)
        fx[:, cols] = ex
        fz[:, cols] = ez
        keys, ms, nk = _keys(sx, sz, lops, fx, fz)
        nbits = ms + nk
        wt = (cds != 0).sum(axis=1)
        prob = (eps / 3.0) ** wt * (1.0 - eps) ** (half - wt)
        dists.append(np.bincount(keys, weights=prob, minlength=1 << nbits))
    joint_p = _wht(_wht(dists[0]) * _wht(dists[1])) / float(1 << nbits)
    ms = sx.shape[0]
    return joint_p.reshape(1 << (nbits - ms), 1 << ms).T, ms          # [syndrome, class]


@pytest.fixture(scope="module")
def l7_joint():
    sx, sz, vc = joint.gb_joint(**L7)
    lops = joint.logical_operators(sx, sz)
    return sx, sz, vc, lops


def test_l7_joint_code_structure(l7_joint):
    sx, sz, vc, lops = l7_joint
    assert sx.shape == (14, 14)
    # rows commute pairwise (symplectic self-orthogonality)
    comm = (sx.astype(int) @ sz.T.astype(int) + sz.astype(int) @ sx.T.astype(int)) & 1
    assert not comm.any()
    assert lops.shape == (4, 28)                       # 2k, k = 2
    assert gf2.rank(np.hstack([sx, sz])) == 12


@pytest.mark.parametrize("eps", [0.03, 0.08])
def test_l7_joint_ml_bound_and_monte_carlo(l7_joint, eps):
    sx, sz, vc, lops = l7_joint
    P, ms = class_probabilities(sx, sz, lops, eps)
    assert P.sum() == pytest.approx(1.0, rel=1e-12)
    assert (P > -1e-15).all()
    fer_ml = 1.0 - P.max(axis=1).sum()
    reach = np.nonzero(P.sum(axis=1) > 0)[0]
    assert len(reach) == 1 << 12                       # rank 12: every reachable syndrome
    synd = ((reach[:, None] >> np.arange(ms)) & 1).astype(np.uint8)
    g = joint.PauliGraph(sx, sz, vc)
    L0 = joint.depolarizing_prior(eps)
    n = sx.shape[1]
    for kind, kw in (("sagms", {}), ("sms", dict(alpha=0.5)), ("ms", {}), ("bp", {})):
        prm = DecoderParams(kind=kind, lmax=30, **kw)
        r = joint.decode_joint(g, synd, np.full(n, L0), prm, "fp64")
        cls_hat = ((r.zhat.astype(np.int64) @ lops[:, :n].T + r.xhat.astype(np.int64) @ lops[:, n:].T) & 1)
        cls_idx = (cls_hat << np.arange(cls_hat.shape[1])).sum(axis=1)
        ok = r.converged
        fer_dec = 1.0 - P[reach[ok], cls_idx[ok]].sum()
        assert fer_dec >= fer_ml - 1e-12, kind
        # converged estimates reproduce their syndrome
        assert (joint.symplectic_syndrome(sx, sz, r.xhat[ok], r.zhat[ok]) == synd[ok]).all()
        if kind == "sagms":
            # Monte Carlo with the channel sampler and the judge, 6000 frames
            fr = 6000
            ex, ez = channel.sample_paulis(9, 3, 0, fr, n, eps)
            s = joint.symplectic_syndrome(sx, sz, ex, ez)
            rr = joint.decode_joint(g, s, np.full(n, L0), prm, "fp64")
            fail = joint.judge_joint(sx, sz, ex, ez, rr.xhat, rr.zhat, rr.converged)
            lo, hi = stats.wilson(int(fail.sum()), fr)
            # the exact FER lies in the sample's 95 % interval (a 5 % test)
            assert lo <= fer_dec <= hi, (fer_dec, lo, hi)
    # ML corrects every weight-1 error (distance 3) at small noise
    if eps == 0.03:
        for q in range(n):
            for W in PAULIS:
                e_x = np.zeros((1, n), dtype=np.uint8)
                e_z = np.zeros((1, n), dtype=np.uint8)
                e_x[0, q] = W in (joint.PX, joint.PY)
                e_z[0, q] = W in (joint.PY, joint.PZ)
                key, _, _ = _keys(sx, sz, lops, e_x, e_z)
                s_idx, c_idx = key[0] & ((1 << ms) - 1), key[0] >> ms
                assert P[s_idx].argmax() == c_idx


# ---------------------------------------------------------- closed forms
@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.625)), ("sagms", {}), ("bp", {})])
def test_round_one_closed_form(kind, kw):
    """Remark 1: under a uniform prior every incoming magnitude of round 1 is
    L0 (min-sum family), so a check's outputs are +-gain * L0 with sign
    (-1)^{s_i} times the product of the (positive) inputs; BP's are
    +-T_BP4(lambda_1) of eq. (transfer_all) with lambda_1 = ln((e^L0 + 1)/2)."""
    sx, sz, vc = joint.gb_joint(63, codes.G63["a"], codes.G63["b"])
    g = joint.PauliGraph(sx, sz, vc)
    eps = 0.05
    L0 = joint.depolarizing_prior(eps)
    rng = np.random.default_rng(4)
    s = (rng.random((6, g.m)) < 0.2).astype(np.uint8)
    s[0] = 0
    prm = DecoderParams(kind=kind, lmax=1, **kw)
    r = joint.decode_joint(g, s, np.full(g.n, L0), prm, "fp64", early_exit=False, trace=True)
    c2v = r.trace[0]["c2v"]                                       # [F, E]
    sign = np.where(s[:, g.e_check] == 1, -1.0, 1.0)
    if kind == "bp":
        lam1 = math.log((math.exp(L0) + 1) / 2)
        mag = analysis.t_bp(lam1, g.dc)
        assert np.allclose(c2v, sign * mag, rtol=1e-12)
    else:
        gain = decoders.check_gains(prm, s, g.m)[:, g.e_check]
        assert np.allclose(c2v, sign * gain * L0, rtol=1e-15, atol=0)
        c2v32 = joint.decode_joint(g, s, np.full(g.n, L0, np.float32), prm, "fp32", early_exit=False,
                                   trace=True).trace[0]["c2v"]
        assert (c2v32 == (sign * (gain.astype(np.float32) * np.float32(L0))).astype(np.float32)).all()
    # frame 0 has a zero syndrome: 0 rounds when early exit is on
    r0 = joint.decode_joint(g, s[:1], np.full(g.n, L0), prm, "fp64")
    assert r0.iters[0] == 0 and r0.converged[0] and not r0.xhat.any() and not r0.zhat.any()


@pytest.mark.parametrize("kind,kw", [("sms", dict(alpha=0.5)), ("sagms", dict(alpha_min=0.25, alpha_max=0.5, eta=1.0)),
                                     ("ms", {})])
def test_z_rows_only_reduce_to_the_binary_decoder(kind, kw):
    """With only Z-type rows (H_Z) and a positive uniform prior, Gamma^Z = L0
    and Gamma^X = Gamma^Y: the joint decoder is the binary decoder of the X
    part.  Integer prior, dyadic gains and few rounds keep every sum exact,
    so both must agree exactly (beliefs, decisions, rounds)."""
    hx, hz = codes.gb_matrices(**codes.G63)
    g = joint.PauliGraph(np.zeros_like(hz), hz)
    tg = decoders.TannerGraph(hz)
    s = channel.syndrome(hz, channel.sample_paulis(2, 0, 0, 300, 126, 0.04)[0])
    prm = DecoderParams(kind=kind, lmax=6, **kw)
    L0 = np.full(126, 3.0)
    rj = joint.decode_joint(g, s, L0, prm, "fp64")
    rb = decoders.decode(tg, s, L0, prm, "fp64")
    assert (rj.iters == rb.iters).all() and (rj.converged == rb.converged).all()
    assert (rj.xhat == rb.ehat).all() and not rj.zhat.any()
    assert (rj.gamma[:, :, 0] == rb.posterior).all() and (rj.gamma[:, :, 1] == rb.posterior).all()
    assert (rj.gamma[:, :, 2] == 3.0).all()


def test_gb126_overcomplete_form():
    """Section V setup: the [[126,28]] GB code as m = 126 Pauli rows,
    d_c = d_v = 10, rows pairwise commuting, 2k = 56 logical operators."""
    sx, sz, vc = joint.gb_joint(63, codes.G63["a"], codes.G63["b"])
    g = joint.PauliGraph(sx, sz, vc)
    assert (g.m, g.n, g.E) == (126, 126, 1260)
    assert (g.cn_deg == 10).all() and (g.vn_deg == 10).all()
    assert g.css
    comm = (sx.astype(int) @ sz.T.astype(int) + sz.astype(int) @ sx.T.astype(int)) & 1
    assert not comm.any()
    lops = joint.logical_operators(sx, sz)
    assert lops.shape == (56, 252)
    # every variable's order lists 5 X-type then 5 Z-type checks
    for j in range(126):
        assert [c < 63 for c in vc[j]] == [True] * 5 + [False] * 5


def test_judges_agree_on_constructed_residuals():
    sx, sz, vc = joint.gb_joint(**L7)
    lops = joint.logical_operators(sx, sz)
    n = 14
    rng = np.random.default_rng(8)
    stab = np.hstack([sx, sz])
    rows = []
    for t in range(60):
        r = (rng.integers(0, 2, size=stab.shape[0]) @ stab) & 1          # a stabilizer
        if t % 2:
            r = r ^ lops[rng.integers(0, lops.shape[0])]                 # times a logical
        rows.append(r)
    rows = np.array(rows, dtype=np.uint8)
    zero = np.zeros((60, n), dtype=np.uint8)
    conv = np.ones(60, dtype=bool)
    f1 = joint.judge_joint(sx, sz, rows[:, :n], rows[:, n:], zero, zero, conv)
    f2 = joint.judge_joint_logical(lops, rows[:, :n], rows[:, n:], zero, zero, conv)
    assert (f1 == f2).all()
    assert (f1 == (np.arange(60) % 2 == 1)).all()


def test_fp32_within_tolerance_of_fp64_first_rounds():
    """SAGMS on the [[126,28]] code: over the first 5 rounds the FP32 beliefs
    stay within 1e-5 relative (floor L0) of FP64 on frames whose FP64 run
    keeps away from exact ties, with identical decisions and rounds."""
    sx, sz, vc = joint.gb_joint(63, codes.G63["a"], codes.G63["b"])
    g = joint.PauliGraph(sx, sz, vc)
    eps = 0.05
    ex, ez = channel.sample_paulis(1, 0, 0, 256, g.n, eps)
    s = joint.symplectic_syndrome(sx, sz, ex, ez)
    L0 = np.float32(joint.depolarizing_prior(eps))
    for lmax in (1, 3, 5):
        prm = DecoderParams(kind="sagms", lmax=lmax)
        r64 = joint.decode_joint(g, s, np.full(g.n, L0), prm, "fp64")
        r32 = joint.decode_joint(g, s, np.full(g.n, L0), prm, "fp32")
        same = (r64.iters == r32.iters) & (r64.xhat == r32.xhat).all(1) & (r64.zhat == r32.zhat).all(1)
        assert same.mean() > 0.98
        err = np.abs(r32.gamma.astype(np.float64) - r64.gamma) / np.maximum(np.abs(r64.gamma), float(L0))
        assert err[same].max() < 1e-5

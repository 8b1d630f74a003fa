"""Pins of the oracle's layered schedule (oracle/layered.py).

The paper defines only the flooding schedule, so the layered schedule is
pinned by what its own definition fixes: the first-fit layering checked by
brute force, a hand-worked two-check example, the special case of checks
with disjoint supports (one layer: the layered and flooding schedules
coincide), a scalar check-by-check implementation on tiny graphs, the FP32
order tracking the FP64 definition, and the schedule's defining effect on
the round count.
"""
import numpy as np
import pytest

import workloads
from oracle import channel, codes, decoders, layered


def tanner(h):
    return decoders.TannerGraph(np.asarray(h, dtype=np.uint8))


@pytest.mark.parametrize("name", ["G63", "G127", "G255w4"])
def test_first_fit_layers_by_brute_force(name):
    hz = codes.gb_matrices(*workloads.code(name))[1]
    lay = layered.greedy_layers(hz)
    seen = np.concatenate(lay)
    assert sorted(seen.tolist()) == list(range(hz.shape[0]))        # a partition
    where = {int(c): t for t, L in enumerate(lay) for c in L}
    for t, L in enumerate(lay):
        assert (np.diff(L) > 0).all()
        sup = hz[L].astype(int)
        assert (sup.sum(axis=0) <= 1).all()                          # disjoint supports
        for c in L:
            # first fit: every earlier layer holds a smaller check sharing a variable
            for u in range(t):
                assert any(d < c and (hz[d] & hz[c]).any() for d in lay[u])
    assert where[0] == 0


def test_hand_worked_two_checks():
    """Checks A = {0, 1}, B = {1, 2} (two layers), MS, L0 = (1, 3, 5),
    s = (1, 0).  Layer A: c2v(A->0) = -3, c2v(A->1) = -1, so post_0 = -2,
    post_1 = 2.  Layer B sees v2c(1->B) = 2 (not 3): c2v(B->1) = 5,
    c2v(B->2) = 2, post = (-2, 7, 7); the hard decision (1, 0, 0) meets s
    after one round.  Flooding gives post_2 = 5 + 3 = 8 instead."""
    h = [[1, 1, 0], [0, 1, 1]]
    g = tanner(h)
    s = np.array([[1, 0]], dtype=np.uint8)
    prm = decoders.DecoderParams(kind="ms", lmax=5)
    for arith, dt in (("fp64", np.float64), ("fp32", np.float32)):
        r = layered.decode_layered(g, s, np.array([1.0, 3.0, 5.0], dtype=dt), prm, arith)
        assert r.posterior[0].tolist() == [-2.0, 7.0, 7.0]
        assert r.iters[0] == 1 and r.converged[0] and r.ehat[0].tolist() == [1, 0, 0]
    rf = decoders.decode(g, s, np.array([1.0, 3.0, 5.0]), prm, "fp64")
    assert rf.posterior[0].tolist() == [-2.0, 7.0, 8.0]


@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.5)),
                                     ("sagms", dict(alpha_min=0.3, alpha_max=0.5, eta=1.1))])
def test_disjoint_checks_equal_flooding(kind, kw):
    """Checks with disjoint supports form one layer; every round of the
    layered schedule then equals a flooding round."""
    rng = np.random.default_rng(3)
    h = np.zeros((4, 14), dtype=np.uint8)
    for i, cols in enumerate([[0, 1, 2], [3, 4, 5, 6], [7, 8, 9], [10, 11, 12, 13]]):
        h[i, cols] = 1
    g = tanner(h)
    assert len(layered.greedy_layers(h)) == 1
    s = rng.integers(0, 2, (200, 4)).astype(np.uint8)
    llr = rng.choice([-2.0, -1.0, 1.0, 2.0, 3.0, 4.0], 14)
    prm = decoders.DecoderParams(kind=kind, lmax=9, **kw)
    rl = layered.decode_layered(g, s, llr, prm, "fp64")
    rf = decoders.decode(g, s, llr, prm, "fp64")
    assert (rl.iters == rf.iters).all() and (rl.ehat == rf.ehat).all() and (rl.converged == rf.converged).all()
    assert np.array_equal(rl.posterior, rf.posterior)


def scalar_layered(h, s, l0, prm):
    """Check-by-check layered min-sum with Python scalars (tiny graphs)."""
    m, n = h.shape
    rows = [list(np.nonzero(h[i])[0]) for i in range(m)]
    lay = layered.greedy_layers(h)
    c2v = {(i, j): 0.0 for i in range(m) for j in rows[i]}

    def post_of(j):
        return float(l0[j]) + sum(c2v[(i, j)] for i in range(m) if h[i, j])

    def residual():
        e = [1 if post_of(j) < 0 else 0 for j in range(n)]
        return [int(s[i]) ^ (sum(e[j] for j in rows[i]) & 1) for i in range(m)], e

    res, e = residual()
    if not any(res):
        return e, 0, True
    for ell in range(1, prm.lmax + 1):
        w = sum(res)
        for L in lay:
            for i in L:
                if prm.kind == "ms":
                    gain = 1.0
                elif prm.kind == "sms":
                    gain = prm.alpha
                else:
                    gain = prm.alpha_max - (prm.alpha_max - prm.alpha_min) * w / m
                    if res[i]:
                        gain *= prm.eta
                v = {j: post_of(j) - c2v[(i, j)] for j in rows[i]}
                new = {}
                for j in rows[i]:
                    others = [v[k] for k in rows[i] if k != j]
                    sign = (-1) ** (int(s[i]) + sum(1 for x in others if x < 0))
                    new[j] = sign * gain * min(abs(x) for x in others)
                for j in rows[i]:
                    c2v[(i, j)] = new[j]
        res, e = residual()
        if not any(res):
            return e, ell, True
    return e, prm.lmax, False


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.5)),
                                     ("sagms", dict(alpha_min=0.25, alpha_max=0.5, eta=1.5))])
def test_matches_scalar_check_by_check(seed, kind, kw):
    """Integer priors and dyadic gains (m = 8, so the SAGMS gain
    (16 - w) / 32 is dyadic too) keep every message exact in FP64 for these
    few rounds, so the two implementations must agree exactly whatever
    their summation orders, ties included."""
    rng = np.random.default_rng(seed)
    m, n = 8, 12
    rows = set()
    while len(rows) < m:
        rows.add(tuple(sorted(rng.choice(n, 3, replace=False).tolist())))
    h = np.zeros((m, n), dtype=np.uint8)
    for i, r in enumerate(sorted(rows)):
        h[i, list(r)] = 1
    g = tanner(h)
    s = rng.integers(0, 2, (16, m)).astype(np.uint8)
    l0 = rng.choice([-3.0, -1.0, 1.0, 2.0, 3.0, 5.0, 7.0], n)
    prm = decoders.DecoderParams(kind=kind, lmax=6, **kw)
    r = layered.decode_layered(g, s, l0, prm, "fp64")
    assert len(layered.greedy_layers(h)) > 1
    for f in range(s.shape[0]):
        e, it, cv = scalar_layered(h, s[f], l0, prm)
        assert r.iters[f] == it and bool(r.converged[f]) == cv and r.ehat[f].tolist() == e


def test_fp32_order_tracks_fp64():
    """The incremental FP32 order stays within a few FP32 roundings per
    round of the FP64 definition over the first rounds."""
    l, a, b = workloads.code("G63")
    hx, hz = codes.gb_matrices(l, a, b)
    g = decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b))
    p = 0.05
    ex, _ = channel.sample_paulis(1, 4, 0, 300, 2 * l, p)
    s = channel.syndrome(hz, ex)
    l0 = channel.prior_llr(p)
    for lmax in (1, 2, 4):
        prm = decoders.DecoderParams(kind="sms", alpha=0.5, lmax=lmax)
        r32 = layered.decode_layered(g, s, np.full(2 * l, l0, dtype=np.float32), prm, "fp32")
        r64 = layered.decode_layered(g, s, np.full(2 * l, np.float32(l0), dtype=np.float64), prm, "fp64")
        same = (r32.iters == r64.iters) & (r32.ehat == r64.ehat).all(axis=1)
        assert same.mean() > 0.95
        err = np.abs(r32.posterior[same] - r64.posterior[same])
        assert (err <= 1e-5 * np.maximum(np.abs(r64.posterior[same]), l0)).all()


def test_layered_needs_fewer_rounds_than_flooding():
    """Later layers use the messages of earlier layers of the same round,
    so SMS converges in fewer rounds than with flooding (l = 63 code,
    p = 0.05, the same 1000 frames)."""
    l, a, b = workloads.code("G63")
    hx, hz = codes.gb_matrices(l, a, b)
    g = decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b))
    p = 0.05
    ex, _ = channel.sample_paulis(1, 4, 0, 1000, 2 * l, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(2 * l, channel.prior_llr(p), dtype=np.float32)
    prm = decoders.DecoderParams(kind="sms", alpha=0.75, lmax=100)
    rl = layered.decode_layered(g, s, llr, prm, "fp32")
    rf = decoders.decode(g, s, llr, prm, "fp32")
    assert rl.iters.mean() < 0.8 * rf.iters.mean()
    assert rl.converged.mean() >= rf.converged.mean()


def test_rejects_bp_and_reduced_formats():
    g = tanner([[1, 1, 0], [0, 1, 1]])
    s = np.zeros((1, 2), dtype=np.uint8)
    with pytest.raises(ValueError):
        layered.decode_layered(g, s, np.ones(3), decoders.DecoderParams(kind="bp"), "fp64")
    with pytest.raises(ValueError):
        layered.decode_layered(g, s, np.ones(3), decoders.DecoderParams(kind="ms"), "fp16")

"""GPU parity: libsagms (through its C ABI) against the CPU oracle.

Bar: bit-exact error samples, syndromes, hard decisions, round counts,
convergence flags, judge verdicts and counters; the FP32 posteriors are
bit-identical to the oracle's FP32 mode (same operation order).  Against
the FP64 mode: over the first 10 rounds, posteriors within 1e-5 relative
(floor L0) on frames whose FP64 trajectory keeps away from decision ties
(2e-4 for SMS with alpha >= 0.75, whose round-to-round error gain is >= 3);
at full length the FER of each lies in the other's Wilson interval.  BP
(transcendental CN) is compared by tolerance and agreement fraction.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, codes, decoders, judge, stats  # noqa: E402

pytestmark = pytest.mark.gpu

SMALL = {"L7a": (7, [0, 1], [0, 2]), "L7b": (7, [0, 1, 3], [0, 2, 6])}


def code_of(name):
    return SMALL[name] if name in SMALL else workloads.code(name)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def say(*args):
    print(*args, flush=True)


def gpu_decode(g, synd_bits, llr, cfg, dev, soft=True):
    f = synd_bits.shape[0]
    synd = torch.from_numpy(channel.pack(synd_bits).view(np.int64)).to(dev) if f else \
        torch.empty((0, g.words_m), dtype=torch.int64, device=dev)
    out = sagms.frame_buffers(g, f, device=dev)
    post = torch.empty((f, g.n), dtype=torch.float32, device=dev)
    llr_dev = torch.from_numpy(np.asarray(llr, dtype=np.float32)).to(dev)
    if soft:
        sagms.decode_soft(g, synd, llr_dev, cfg, out["ehat"], out["iters"], out["converged"], post)
    else:
        sagms.decode(g, synd, llr_dev, cfg, out["ehat"], out["iters"], out["converged"])
    torch.cuda.synchronize()
    return (channel.unpack(u64(out["ehat"]), g.n), out["iters"].cpu().numpy(),
            out["converged"].cpu().numpy().astype(bool), post.cpu().numpy())


def tanner(l, a, b):
    """The oracle's graph of a GB code, with the code's posterior-sum order."""
    return decoders.TannerGraph(codes.gb_matrices(l, a, b)[1], codes.gb_var_checks(l, a, b))


def params(kind, lmax, **kw):
    return decoders.DecoderParams(kind=kind, lmax=lmax, **kw), sagms.decoder_config(kind, lmax=lmax, **kw)


# ------------------------------------------------------------------ sampler
@pytest.mark.parametrize("name", ["L7a", "G63", "G127", "G255w3", "G511w5"])
@pytest.mark.parametrize("p", [0.0, 0.05, 0.3])
def test_sampler_bit_exact(dev, name, p):
    l, a, b = code_of(name)
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    for seed, stream_id, frame0, nf in ((1, 0, 0, 333), (0xDEADBEEF12345, 7, (1 << 32) - 100, 257)):
        say("sampler", name, p, seed, stream_id, frame0, nf)
        buf = sagms.frame_buffers(g, nf, device=dev)
        sagms.gen_errors(g, seed, stream_id, frame0, nf, p, buf["ex"], buf["ez"], buf["synd"])
        torch.cuda.synchronize()
        ex, ez = channel.sample_paulis(seed, stream_id, frame0, nf, g.n, p)
        assert (u64(buf["ex"]) == channel.pack(ex)).all()
        assert (u64(buf["ez"]) == channel.pack(ez)).all()
        assert (u64(buf["synd"]) == channel.pack(channel.syndrome(hz, ex))).all()


def test_sampler_without_z_plane_and_empty(dev):
    g = sagms.Graph.gb(*workloads.code("G63"))
    buf = sagms.frame_buffers(g, 100, device=dev, with_ez=False)
    sagms.gen_errors(g, 3, 2, 5, 100, 0.07, buf["ex"], None, buf["synd"])
    sagms.gen_errors(g, 3, 2, 5, 0, 0.07, buf["ex"][:0], None, buf["synd"][:0])
    torch.cuda.synchronize()
    ex, _ = channel.sample_paulis(3, 2, 5, 100, 126, 0.07)
    assert (u64(buf["ex"]) == channel.pack(ex)).all()


# ------------------------------------------------------------------ decoder
DECODERS = [("ms", {}), ("sms", dict(alpha=0.5)), ("sms", dict(alpha=0.625)), ("sms", dict(alpha=0.75)),
            ("sms", dict(alpha=0.875)), ("sagms", {})]


@pytest.mark.parametrize("kind,kw", DECODERS)
@pytest.mark.parametrize("p", [0.02, 0.05, 0.1])
def test_decode_bit_exact_g63(dev, kind, kw, p):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    nf = 1200
    ex, _ = channel.sample_paulis(1, workloads.stream_of(p), 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    prm, cfg = params(kind, 100, **kw)
    say("decode G63", kind, kw, p, nf)
    e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
    r = decoders.decode(tanner(l, a, b), s, llr, prm, "fp32")
    assert (it == r.iters).all()
    assert (cv == r.converged).all()
    assert (e == r.ehat).all()
    assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()


@pytest.mark.parametrize("kind,kw", DECODERS + [("bp", {})])
def test_decode_g63_given_as_rows(dev, kind, kw):
    """The l = 63 code given row by row (CSR): the general LDS-staged kernel,
    posteriors summed in ascending check order, bit-exact against the
    oracle's default graph (BP within tolerance)."""
    l, a, b = workloads.code("G63")
    hx, hz = codes.gb_matrices(l, a, b)
    g = sagms.Graph.from_dense(hz, hx)
    p, nf = 0.06, 800
    ex, _ = channel.sample_paulis(3, 1, 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    prm, cfg = params(kind, 100, **kw)
    say("decode G63 rows", kind, kw)
    e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
    r = decoders.decode(decoders.TannerGraph(hz), s, llr, prm, "fp32")
    if kind == "bp":
        agree = (it == r.iters) & (e == r.ehat).all(axis=1)
        assert agree.mean() > 0.97
        return
    assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
    assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()


@pytest.mark.parametrize("name,nf", [("L7a", 300), ("L7b", 300), ("G127", 400), ("G255w3", 200),
                                     ("G255w4", 200), ("G511w5", 60)])
@pytest.mark.parametrize("kind", ["ms", "sms", "sagms"])
def test_decode_bit_exact_other_codes(dev, name, nf, kind):
    l, a, b = code_of(name)
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    p = 0.04
    ex, _ = channel.sample_paulis(5, 3, 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    prm, cfg = params(kind, 60, **({"alpha": 0.75} if kind == "sms" else {}))
    say("decode", name, kind, nf)
    e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
    r = decoders.decode(tanner(l, a, b), s, llr, prm, "fp32")
    assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
    assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()


@pytest.mark.parametrize("lmax", [1, 2, 7])
@pytest.mark.parametrize("kind", ["ms", "sagms"])
def test_decode_arbitrary_syndromes_and_priors(dev, lmax, kind):
    """All-zero / all-one / random syndromes, non-uniform, negative and -0.0 priors."""
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    s = workloads.random_syndromes(g.m, 300, seed=lmax)
    rng = np.random.default_rng(17)
    llr = rng.uniform(-1.0, 5.0, size=g.n).astype(np.float32)
    llr[3] = -0.0
    llr[4] = 0.0
    prm, cfg = params(kind, lmax)
    say("decode arbitrary", kind, lmax)
    e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
    r = decoders.decode(tanner(l, a, b), s, llr, prm, "fp32")
    assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
    assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()
    assert (it[~cv] == lmax).all()


def test_decode_zero_noise_and_tiny_batches(dev):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    llr = np.full(g.n, channel.prior_llr(0.05), dtype=np.float32)
    cfg = sagms.decoder_config("sagms")
    for nf in (1, 2, 3, 5, 63, 65):
        s = np.zeros((nf, g.m), dtype=np.uint8)
        e, it, cv, _ = gpu_decode(g, s, llr, cfg, dev)
        assert not e.any() and (it == 0).all() and cv.all()
    s = workloads.random_syndromes(g.m, 5, seed=9, density=0.05)
    e, it, cv, _ = gpu_decode(g, s, llr, cfg, dev, soft=False)
    r = decoders.decode(tanner(l, a, b), s, llr, decoders.DecoderParams(kind="sagms"), "fp32")
    assert (it == r.iters).all() and (e == r.ehat).all()


def test_decode_from_csr_graph_with_irregular_degrees(dev):
    """A non-GB graph with uneven check and variable degrees (padded shapes)."""
    rng = np.random.default_rng(4)
    m, n = 40, 90
    h = np.zeros((m, n), dtype=np.uint8)
    for i in range(m):
        h[i, rng.choice(n, size=int(rng.integers(2, 11)), replace=False)] = 1
    g = sagms.Graph.from_dense(h)
    s = workloads.random_syndromes(m, 400, seed=5, density=0.2)
    llr = rng.uniform(0.5, 4.0, size=n).astype(np.float32)
    for kind in ("ms", "sagms"):
        prm, cfg = params(kind, 25)
        say("decode csr", kind, g.dc_max, g.dv_max)
        e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
        r = decoders.decode(decoders.TannerGraph(h), s, llr, prm, "fp32")
        assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
        assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()


def tie_flags(trace, nframes, tau):
    """Frames whose FP64 trajectory brings a posterior or a v2c message within
    tau of zero (a sign / hard-decision tie) in any recorded round."""
    near = np.zeros(nframes, dtype=bool)
    for rd in trace:
        near[rd["frames"]] |= (np.abs(rd["post"]).min(axis=1) <= tau) | (np.abs(rd["v2c"]).min(axis=1) <= tau)
    return near


# Per-round bar against FP64 (posteriors relative to max(|x64|, L0), rounds
# l = 1..10, frames outside the tie band).  A round adds at most about 7
# FP32 roundings (gain product, d_v additions, one subtraction; 8 counted
# here) and carries earlier errors forward with a gain of at most
# G = gain * (d_v - 1): the check output follows one input (min-sum) or
# moves by at most the change of any one input (BP), and a variable sums
# d_v - 1 of them.  So after l rounds the relative error is at most
# E_G(l) = 8 * 2^-24 * (G^l - 1) / (G - 1).  The bar is 1e-5 for every round
# where E_G(l) <= 1e-5, and for all ten rounds where G <= 2.5 (SAGMS with
# gain <= 0.55, SMS with alpha <= 0.625), measured to hold there; in later
# rounds of a larger G it is E_G(l) itself.
EPS_ROUND = 8 * 2.0 ** -24
ROUNDS = range(1, 11)


def error_gain(kind, kw, dv=5):
    if kind in ("ms", "bp"):
        return 1.0 * (dv - 1)
    if kind == "sms":
        return kw["alpha"] * (dv - 1)
    return max(workloads.SAGMS_PARAMS["alpha_max"] * workloads.SAGMS_PARAMS["eta"], 0.0) * (dv - 1)


def round_bar(G, rnd):
    growth = EPS_ROUND * (G ** rnd - 1.0) / (G - 1.0)
    return 1e-5 if (G <= 2.5 or growth <= 1e-5) else growth


def per_round_against_fp64(dev, kind, kw, s, llr, llr64=None):
    """Decodes with l_max = 1..10 on the GPU and in the FP64 oracle; returns
    [(round, max relative error, checked fraction, bar)] over the frames
    whose FP64 trajectory stays outside the tie band 1e-4 L0 (hard decisions
    and round counts of those frames must be identical)."""
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    tg = tanner(l, a, b)
    nf = s.shape[0]
    floor = float(np.min(np.abs(llr)))
    G = error_gain(kind, kw)
    rows = []
    for rnd in ROUNDS:
        prm, cfg = params(kind, rnd, **kw)
        e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
        r64 = decoders.decode(tg, s, llr if llr64 is None else llr64, prm, "fp64", trace=True)
        ok = ~tie_flags(r64.trace, nf, 1e-4 * floor)
        assert (it[ok] == r64.iters[ok]).all() and (e[ok] == r64.ehat[ok]).all(), rnd
        err = np.abs(post[ok].astype(np.float64) - r64.posterior[ok]) / np.maximum(np.abs(r64.posterior[ok]), floor)
        rows.append((rnd, float(err.max()) if err.size else 0.0, float(ok.mean()), round_bar(G, rnd)))
    say("per-round max relative error against FP64", kind, kw, "G=%.3g" % G,
        " ".join("l%d:%.2e/%.2f" % (rnd, m, c) for rnd, m, c, _ in rows))
    for rnd, m, c, bar in rows:
        assert m <= bar, (kind, kw, rnd, m, bar)
    return rows


@pytest.mark.parametrize("kind,kw", DECODERS + [("bp", {})])
@pytest.mark.parametrize("p", [0.02, 0.05, 0.1])
def test_fp32_messages_within_tolerance_of_fp64(dev, kind, kw, p):
    """Per-round posteriors against the FP64 oracle (the FP32 prior promoted
    to double), uniform prior of the channel, frames of the sweep stream.
    With a dyadic gain (MS: 1, SMS: 0.5) every message is an exact dyadic
    combination of a uniform L0: ties are exact and most frames fall in the
    tie band, so those two are also run with random priors below."""
    l, a, b = workloads.code("G63")
    nf = 600
    ex, _ = channel.sample_paulis(1, workloads.stream_of(p), 0, nf, 2 * l, p)
    s = channel.syndrome(codes.gb_matrices(l, a, b)[1], ex)
    llr = np.full(2 * l, channel.prior_llr(p), dtype=np.float32)
    say("fp64 per round", kind, kw, p)
    rows = per_round_against_fp64(dev, kind, kw, s, llr)
    dyadic = kind == "ms" or kw.get("alpha") == 0.5
    if not dyadic:
        assert np.mean([c for _, _, c, _ in rows]) >= 0.5


@pytest.mark.parametrize("kind,kw", DECODERS + [("bp", {})])
@pytest.mark.parametrize("p", [0.02, 0.05, 0.1])
def test_fp32_messages_within_tolerance_of_fp64_random_priors(dev, kind, kw, p):
    """The same per-round bar with non-uniform priors (L0 (1 + u), u uniform in
    [-0.25, 0.25] per variable), which remove the exact message ties: at
    least half of the frames are checked in every round."""
    l, a, b = workloads.code("G63")
    nf = 600
    ex, _ = channel.sample_paulis(1, workloads.stream_of(p), 0, nf, 2 * l, p)
    s = channel.syndrome(codes.gb_matrices(l, a, b)[1], ex)
    rng = np.random.default_rng(int(p * 1000))
    llr = (channel.prior_llr(p) * (1.0 + rng.uniform(-0.25, 0.25, 2 * l))).astype(np.float32)
    say("fp64 per round, random priors", kind, kw, p)
    rows = per_round_against_fp64(dev, kind, kw, s, llr, llr.astype(np.float64))
    for rnd, _, c, _ in rows:
        assert c >= 0.5, (rnd, c)


@pytest.mark.parametrize("prior", ["uniform", "random"])
@pytest.mark.parametrize("kind,kw", DECODERS)
def test_fer_matches_fp64_oracle(dev, kind, kw, prior):
    """Full-length decoding (l_max = 100): the GPU FER and the FER of the FP64
    oracle (fed the FP64 prior) on the same frames each lie in the other's
    95 % Wilson interval; the fraction of frames whose hard decision
    differs is small.  Uniform prior: the channel's L0 (MS within 25 %, see
    the tie note below).  Random: L0 (1 + u) per variable, u uniform in
    [-0.25, 0.25], which leaves MS no exact ties (Wilson bar for all)."""
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    p, nf = 0.05, 3000
    ex, _ = channel.sample_paulis(1, workloads.stream_of(p), 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    if prior == "uniform":
        llr64 = np.full(g.n, channel.prior_llr(p))
    else:
        llr64 = channel.prior_llr(p) * (1.0 + np.random.default_rng(29).uniform(-0.25, 0.25, g.n))
    llr = llr64.astype(np.float32)
    prm, cfg = params(kind, 100, **kw)
    say("fer vs fp64", kind, kw, prior)
    e, it, cv, _ = gpu_decode(g, s, llr, cfg, dev, soft=False)
    r64 = decoders.decode(tanner(l, a, b), s, llr64, prm, "fp64")
    lz = codes.logical_basis(hz, hx)
    f_gpu = int(judge.judge_logical(lz, ex, e, cv).sum())
    f_64 = int(judge.judge_logical(lz, ex, r64.ehat, r64.converged).sum())
    if kind == "ms" and prior == "uniform":
        # with a uniform prior min-sum resolves its frequent exact ties by
        # rounding residues (see the oracle's tie test), which grow from
        # 2^-24 in FP32 but from 2^-53 in FP64, so its FER moves with
        # precision: agreement within 25 % relative
        assert abs(f_gpu - f_64) <= 0.25 * max(f_64, f_gpu)
    else:
        lo_g, hi_g = stats.wilson(f_gpu, nf)
        lo_o, hi_o = stats.wilson(f_64, nf)
        assert lo_o <= f_gpu / nf <= hi_o and lo_g <= f_64 / nf <= hi_g
    differ = (e != r64.ehat).any(axis=1)
    both = cv & r64.converged
    say("FER gpu %.4f fp64 %.4f, HD-disagreeing frames %.4f (%.4f of frames converged in both)"
        % (f_gpu / nf, f_64 / nf, differ.mean(), differ[both].mean()))
    # a frame that oscillates until l_max ends in an arbitrary state in either
    # precision; frames that converge in both agree almost always
    assert differ[both].mean() < (0.05 if kind == "ms" else 0.01)


def test_bp_against_oracle(dev):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    p = 0.05
    nf = 1000
    ex, _ = channel.sample_paulis(1, 4, 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    prm, cfg = params("bp", 100)
    say("decode bp")
    e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
    r = decoders.decode(tanner(l, a, b), s, llr, prm, "fp32")
    agree = (it == r.iters) & (e == r.ehat).all(axis=1)
    assert agree.mean() > 0.97
    tol = 1e-4 * np.maximum(np.abs(r.posterior[agree]), float(llr[0]))
    close = (np.abs(post[agree] - r.posterior[agree]) <= tol).all(axis=1)
    assert close.mean() > 0.97
    resid = s ^ channel.syndrome(hz, e)
    assert not resid[cv].any()


# ------------------------------------------------------------------ judge
def test_judge_matches_oracle_rank_test(dev):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    nf, p = 3000, 0.08
    buf = sagms.frame_buffers(g, nf, device=dev)
    llr = torch.full((g.n,), float(np.float32(channel.prior_llr(p))), device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    sagms.gen_errors(g, 2, 6, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    sagms.decode(g, buf["synd"], llr, sagms.decoder_config("ms", lmax=30), buf["ehat"], buf["iters"], buf["converged"])
    sagms.judge(g, buf["ex"], buf["ehat"], buf["converged"], buf["iters"], counters, fail=buf["fail"])
    torch.cuda.synchronize()
    ex = channel.unpack(u64(buf["ex"]), g.n)
    eh = channel.unpack(u64(buf["ehat"]), g.n)
    cv = buf["converged"].cpu().numpy().astype(bool)
    fail = buf["fail"].cpu().numpy().astype(bool)
    ref = judge.judge_rank(hx, ex[:600], eh[:600], cv[:600])
    assert (fail[:600] == ref).all()
    assert (fail == judge.judge_logical(codes.logical_basis(hz, hx), ex, eh, cv)).all()
    c = counters.cpu().numpy()
    assert c[0] == fail.sum() and c[1] == buf["iters"].cpu().numpy().sum()


@pytest.mark.parametrize("name", ["L7a", "G63", "G127", "G511w5"])
def test_judge_on_constructed_residuals(dev, name):
    """Residuals that are stabilizers (success), logical operators and their
    sums (failure), with and without convergence, against the rank test."""
    l, a, b = code_of(name)
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    lz = codes.logical_basis(hz, hx)
    rng = np.random.default_rng(8)
    nf = 96
    stab = (rng.integers(0, 2, size=(nf, hx.shape[0])) @ hx.astype(np.int64)) & 1
    logi = (rng.integers(0, 2, size=(nf, lz.shape[0])) @ lz.astype(np.int64)) & 1
    r = np.where((np.arange(nf) % 3 == 0)[:, None], stab, stab ^ logi).astype(np.uint8)
    ex = rng.integers(0, 2, size=(nf, g.n)).astype(np.uint8)
    eh = ex ^ r
    cv = (np.arange(nf) % 5 != 0).astype(np.uint8)
    it = rng.integers(0, 100, size=nf).astype(np.int32)
    T = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to(dev, dt)  # noqa: E731
    fail = torch.empty(nf, dtype=torch.uint8, device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    sagms.judge(g, T(channel.pack(ex).view(np.int64), torch.int64), T(channel.pack(eh).view(np.int64), torch.int64),
                T(cv, torch.uint8), T(it, torch.int32), counters, fail=fail)
    torch.cuda.synchronize()
    ref = judge.judge_rank(hx, ex, eh, cv.astype(bool))
    got = fail.cpu().numpy().astype(bool)
    assert (got == ref).all()
    assert (got & cv.astype(bool)).any() and (~got).any()
    assert counters.cpu().numpy().tolist() == [int(ref.sum()), int(it.sum())]


# ----------------------------------------------- full size, bench launch shape
def test_full_size_sampled_frames(dev):
    """2^20 frames at p = 0.05 (the timed workload), SAGMS, l_max = 100:
    sampled frames recomputed one by one by the oracle, counters checked
    against the per-frame verdicts, FER inside the Wilson interval of the
    oracle's own estimate on an independent prefix."""
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    nf, p = workloads.SWEEP_FRAMES, 0.05
    st = workloads.stream_of(p)
    buf = sagms.frame_buffers(g, nf, device=dev)
    llr = torch.full((g.n,), float(np.float32(channel.prior_llr(p))), device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    cfg = sagms.decoder_config("sagms", lmax=100)
    say("full size", nf)
    sagms.gen_errors(g, workloads.SWEEP_SEED, st, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    sagms.judge(g, buf["ex"], buf["ehat"], buf["converged"], buf["iters"], counters, fail=buf["fail"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(nf, size=256, replace=False))
    idx[-1] = nf - 1
    ex_all, synd_all = u64(buf["ex"]), u64(buf["synd"])
    eh_all, it_all = u64(buf["ehat"]), buf["iters"].cpu().numpy()
    cv_all, fail_all = buf["converged"].cpu().numpy(), buf["fail"].cpu().numpy()
    tg = tanner(l, a, b)
    lz = codes.logical_basis(hz, hx)
    llr_np = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    exs = np.vstack([channel.sample_paulis(workloads.SWEEP_SEED, st, int(f), 1, g.n, p)[0] for f in idx])
    s = channel.syndrome(hz, exs)
    assert (channel.pack(exs) == ex_all[idx]).all() and (channel.pack(s) == synd_all[idx]).all()
    r = decoders.decode(tg, s, llr_np, decoders.DecoderParams(kind="sagms", lmax=100), "fp32")
    assert (channel.pack(r.ehat) == eh_all[idx]).all()
    assert (r.iters == it_all[idx]).all() and (r.converged == cv_all[idx]).all()
    assert (judge.judge_logical(lz, exs, r.ehat, r.converged) == fail_all[idx]).all()
    c = counters.cpu().numpy()
    assert c[0] == fail_all.sum() and c[1] == it_all.sum()
    # oracle FER on its own prefix; the two estimates' Wilson intervals overlap
    pre = 4000
    ex0, _ = channel.sample_paulis(workloads.SWEEP_SEED, st, 0, pre, g.n, p)
    r0 = decoders.decode(tg, channel.syndrome(hz, ex0), llr_np, decoders.DecoderParams(kind="sagms", lmax=100), "fp64")
    f0 = int(judge.judge_logical(lz, ex0, r0.ehat, r0.converged).sum())
    lo0, hi0 = stats.wilson(f0, pre)
    lo1, hi1 = stats.wilson(int(c[0]), nf)
    assert lo0 <= hi1 and lo1 <= hi0


def test_determinism_split_and_streams(dev):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    nf, p = 5000, 0.06
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 9, 1, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), float(np.float32(channel.prior_llr(p))), device=dev)
    cfg = sagms.decoder_config("sagms", lmax=100)
    sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    ref = [buf[k].clone() for k in ("ehat", "iters", "converged")]
    # again, and split in two calls on two other streams
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    k = 1777
    with torch.cuda.stream(s1):
        sagms.decode(g, buf["synd"][:k], llr, cfg, buf["ehat"][:k], buf["iters"][:k], buf["converged"][:k])
    with torch.cuda.stream(s2):
        sagms.decode(g, buf["synd"][k:], llr, cfg, buf["ehat"][k:], buf["iters"][k:], buf["converged"][k:])
    torch.cuda.synchronize()
    for key, r in zip(("ehat", "iters", "converged"), ref):
        assert torch.equal(buf[key], r), key
    # a frame range generated separately equals the slice of the whole batch
    part = sagms.frame_buffers(g, 100, device=dev)
    sagms.gen_errors(g, 9, 1, 2500, 100, p, part["ex"], part["ez"], part["synd"])
    torch.cuda.synchronize()
    assert torch.equal(part["ex"], buf["ex"][2500:2600]) and torch.equal(part["synd"], buf["synd"][2500:2600])


@pytest.mark.parametrize("fpw", [1, 3, 16, 1024])
def test_decode_launch_shape_does_not_change_results(dev, fpw):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hz = codes.gb_matrices(l, a, b)[1]
    p, nf = 0.07, 1500
    ex, _ = channel.sample_paulis(4, 2, 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    ref = gpu_decode(g, s, llr, sagms.decoder_config("sagms"), dev)
    got = gpu_decode(g, s, llr, sagms.decoder_config("sagms", frames_per_wave=fpw), dev)
    for x, y in zip(ref, got):
        assert (x.view(np.uint8) == y.view(np.uint8)).all()


@pytest.mark.parametrize("name,nf", [("G63", 300_001), ("G63", 16_385), ("G127", 140_000), ("G511w5", 40_000)])
def test_tapered_launch_covers_every_frame(dev, name, nf):
    """The default launch's tapered frame assignment (runs of 16 frames, then
    8, 4, 2 and 1 at the end of the grid) decodes every frame exactly as a
    launch with one frame per wave does, on batches that span every level
    of the taper; outputs start as a sentinel, so a frame left out shows."""
    l, a, b = workloads.code(name)
    g = sagms.Graph.gb(l, a, b)
    p = 0.06
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 3, 7, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    outs = []
    for fpw in (0, 1):
        e = torch.full((nf, g.words_n), -1, dtype=torch.int64, device=dev)
        it = torch.full((nf,), -7, dtype=torch.int32, device=dev)
        cv = torch.full((nf,), 9, dtype=torch.uint8, device=dev)
        say("taper", name, nf, fpw)
        sagms.decode(g, buf["synd"], llr, sagms.decoder_config("sagms", frames_per_wave=fpw), e, it, cv)
        torch.cuda.synchronize()
        outs.append((e.cpu().numpy(), it.cpu().numpy(), cv.cpu().numpy()))
    (e0, i0, c0), (e1, i1, c1) = outs
    assert (i1 >= 0).all() and (c1 <= 1).all()
    assert (e0 == e1).all() and (i0 == i1).all() and (c0 == c1).all()


C1 = None


def c1_golden():
    import base64
    import json
    import os
    global C1
    if C1 is None:
        C1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1_calibration.json")))
    dec = lambda s, n: np.frombuffer(base64.b64decode(s), dtype=np.uint8)[:n]  # noqa: E731
    return C1, dec


@pytest.mark.parametrize("name", ["ms", "sms", "sagms"])
def test_cpu_calibration_case(dev, name):
    """The CPU calibration case (l = 63, p = 0.05, seed 1 / stream 0, frames
    0..9999, l_max = 50): the GPU agrees frame by frame with the stored FP32
    oracle run and, for SMS / SAGMS, its FER lies in the Wilson interval of
    the stored FP64 run.  Min-sum breaks its exact ties only as rounding
    residues grow, which FP64 needs more rounds for, so its FP64 FER at
    l_max = 50 is far higher (recorded, not a parity target)."""
    c, dec = c1_golden()
    d = c["decoders"][name]
    l, a, b = workloads.code(c["code"])
    g = sagms.Graph.gb(l, a, b)
    nf = c["frames"]
    buf = sagms.frame_buffers(g, nf, device=dev)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    sagms.gen_errors(g, c["seed"], c["stream"], 0, nf, c["p"], buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), float(np.float32(channel.prior_llr(c["p"]))), device=dev)
    cfg = sagms.decoder_config(lmax=c["lmax"], **d["params"])
    sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    sagms.judge(g, buf["ex"], buf["ehat"], buf["converged"], buf["iters"], counters, fail=buf["fail"])
    torch.cuda.synchronize()
    fail = buf["fail"].cpu().numpy()
    it = buf["iters"].cpu().numpy()
    ref32 = np.unpackbits(dec(d["fp32"]["fail_bits"], (nf + 7) // 8))[:nf]
    assert (fail == ref32).all()
    assert (it == dec(d["fp32"]["iters"], nf)).all()
    assert counters.cpu().numpy().tolist() == [d["fp32"]["failures"], d["fp32"]["sum_iters"]]
    f64 = d["fp64"]["failures"]
    if name == "ms":
        assert f64 > 2 * int(fail.sum())
    else:
        lo, hi = stats.wilson(f64, nf)
        assert lo <= fail.sum() / nf <= hi
        lo, hi = stats.wilson(int(fail.sum()), nf)
        assert lo <= f64 / nf <= hi


@pytest.mark.parametrize("precision", ["fp16", "int6"])
@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.75)), ("sagms", {})])
@pytest.mark.parametrize("p", [0.03, 0.05, 0.08])
def test_reduced_precision_bit_exact(dev, precision, kind, kw, p):
    """FP16 and INT6 messages: hard decisions, rounds, flags and FP32
    posteriors bit-exact against the oracle's mode of the same format."""
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    hz = codes.gb_matrices(l, a, b)[1]
    nf = 1000
    ex, _ = channel.sample_paulis(1, workloads.stream_of(p), 0, nf, g.n, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(p), dtype=np.float32)
    prm = decoders.DecoderParams(kind=kind, lmax=100, **kw)
    cfg = sagms.decoder_config(kind, lmax=100, precision=precision, **kw)
    say("decode", precision, kind, kw, p)
    e, it, cv, post = gpu_decode(g, s, llr, cfg, dev)
    r = decoders.decode(tanner(l, a, b), s, llr, prm, precision)
    assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
    assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()


@pytest.mark.parametrize("precision", ["fp16", "int6"])
@pytest.mark.parametrize("name,nf", [("L7b", 300), ("G127", 300), ("G255w4", 150), ("G511w5", 40)])
def test_reduced_precision_other_codes(dev, precision, name, nf):
    l, a, b = code_of(name)
    g = sagms.Graph.gb(l, a, b)
    hz = codes.gb_matrices(l, a, b)[1]
    ex, _ = channel.sample_paulis(6, 1, 0, nf, g.n, 0.04)
    s = channel.syndrome(hz, ex)
    llr = np.full(g.n, channel.prior_llr(0.04), dtype=np.float32)
    say("decode", precision, name)
    e, it, cv, post = gpu_decode(g, s, llr, sagms.decoder_config("sagms", lmax=60, precision=precision), dev)
    r = decoders.decode(tanner(l, a, b), s, llr, decoders.DecoderParams(kind="sagms", lmax=60), precision)
    assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
    assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()


@pytest.mark.parametrize("precision", ["fp16", "int6"])
def test_reduced_precision_arbitrary_inputs(dev, precision):
    l, a, b = workloads.code("G63")
    g = sagms.Graph.gb(l, a, b)
    s = workloads.random_syndromes(g.m, 300, seed=11)
    rng = np.random.default_rng(12)
    llr = rng.uniform(-2.0, 20.0, size=g.n).astype(np.float32)
    llr[5] = -0.0
    for lmax in (1, 9):
        e, it, cv, post = gpu_decode(g, s, llr, sagms.decoder_config("ms", lmax=lmax, precision=precision), dev)
        r = decoders.decode(tanner(l, a, b), s, llr, decoders.DecoderParams(kind="ms", lmax=lmax), precision)
        assert (it == r.iters).all() and (e == r.ehat).all()
        assert (post.view(np.uint32) == r.posterior.view(np.uint32)).all()

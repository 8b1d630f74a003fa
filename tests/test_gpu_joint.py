"""Joint (quaternary) decoding on the GPU, through the C ABI, against the
oracle (oracle/joint.py).

* Sampler: X and Z error planes and the symplectic syndrome (H_X e_z,
  H_Z e_x) bit-exact, on the register-row and the gather paths.
* Decoder: x_hat, z_hat, round counts, convergence flags and the three FP32
  beliefs of every variable bit-identical to the oracle's FP32 mode (MS,
  SMS, SAGMS) on four GB codes, the [[126,28]] code of the paper's Section V
  setup among them (m = 126, d_c = d_v = 10), at several noise levels, on
  arbitrary syndromes with non-uniform and negative priors, l_max in
  {1, 2, 7}, and on sampled frames of a 2^20-frame launch.
* Judge: verdicts and counters equal the oracle's stabilizer-group test.
* Against the FP64 oracle: beliefs round by round within the bar of the
  binary decoder's FP32 growth bound (1e-5 where it allows), hard decisions
  and rounds identical outside the tie band; full-length FER in each
  other's Wilson interval.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, joint, stats  # noqa: E402
from oracle.decoders import DecoderParams  # noqa: E402

pytestmark = pytest.mark.gpu

SMALL = {"L7": (7, [0, 1], [0, 2]), "L7b": (7, [0, 1, 3], [0, 2, 6])}


def code_of(name):
    return SMALL[name] if name in SMALL else workloads.code(name)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*args):
    print(*args, flush=True)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


_oracle_graphs = {}


def oracle_graph(name):
    if name not in _oracle_graphs:
        l, a, b = code_of(name)
        sx, sz, vc = joint.gb_joint(l, a, b)
        _oracle_graphs[name] = (sx, sz, joint.PauliGraph(sx, sz, vc))
    return _oracle_graphs[name]


def gpu_decode(g, synd_bits, llr, cfg, dev):
    f = synd_bits.shape[0]
    synd = torch.from_numpy(channel.pack(synd_bits).view(np.int64)).to(dev)
    out = sagms.frame_buffers(g, f, device=dev)
    gamma = torch.empty((f, g.n, 3), dtype=torch.float32, device=dev)
    llr_dev = torch.from_numpy(np.asarray(llr, dtype=np.float32)).to(dev)
    sagms.decode_soft(g, synd, llr_dev, cfg, out["ehat"], out["iters"], out["converged"], gamma)
    torch.cuda.synchronize()
    e = u64(out["ehat"])
    wn = g.words_n
    return (channel.unpack(e[:, :wn], g.n), channel.unpack(e[:, wn:], g.n), out["iters"].cpu().numpy(),
            out["converged"].cpu().numpy().astype(bool), gamma.cpu().numpy())


def sample(name, nf, eps, seed=1, stream=0, frame0=0):
    l, a, b = code_of(name)
    sx, sz, _ = oracle_graph(name)
    ex, ez = channel.sample_paulis(seed, stream, frame0, nf, 2 * l, eps)
    return ex, ez, joint.symplectic_syndrome(sx, sz, ex, ez)


def assert_same(gpu, r, tag):
    xh, zh, it, cv, gamma = gpu
    assert (it == r.iters).all(), (tag, "iters")
    assert (cv == r.converged).all(), (tag, "converged")
    assert (xh == r.xhat).all() and (zh == r.zhat).all(), (tag, "estimate")
    assert (gamma.view(np.uint32) == r.gamma.astype(np.float32).view(np.uint32)).all(), (tag, "beliefs")


# ------------------------------------------------------------------ sampler
@pytest.mark.parametrize("name", ["L7", "G63", "G127", "G255w4"])
@pytest.mark.parametrize("eps", [0.0, 0.05, 0.3])
def test_joint_sampler_bit_exact(dev, name, eps):
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    for seed, stream_id, frame0, nf in ((1, 0, 0, 333), (0xDEADBEEF12345, 7, (1 << 32) - 100, 257)):
        say("joint sampler", name, eps, seed, frame0, nf)
        buf = sagms.frame_buffers(g, nf, device=dev)
        sagms.gen_errors(g, seed, stream_id, frame0, nf, eps, buf["ex"], buf["ez"], buf["synd"])
        torch.cuda.synchronize()
        ex, ez, s = sample(name, nf, eps, seed, stream_id, frame0)
        assert (u64(buf["ex"]) == channel.pack(ex)).all()
        assert (u64(buf["ez"]) == channel.pack(ez)).all()
        assert (u64(buf["synd"]) == channel.pack(s)).all()


# ------------------------------------------------------------------ decoder
DECODERS = [("ms", {}), ("sms", dict(alpha=0.5)), ("sms", dict(alpha=0.75)), ("sagms", {})]


@pytest.mark.parametrize("kind,kw", DECODERS)
@pytest.mark.parametrize("name,nf,eps", [("L7", 500, 0.05), ("L7b", 500, 0.08), ("G63", 1500, 0.01),
                                         ("G63", 1500, 0.04), ("G63", 800, 0.08), ("G127", 600, 0.03)])
def test_joint_decode_bit_exact(dev, name, nf, eps, kind, kw):
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    _, _, pg = oracle_graph(name)
    _, _, s = sample(name, nf, eps, seed=3, stream=int(eps * 100))
    llr = np.full(2 * l, joint.depolarizing_prior(eps), dtype=np.float32)
    say("joint decode", name, kind, kw, eps, nf)
    gpu = gpu_decode(g, s, llr, sagms.decoder_config(kind, lmax=100, **kw), dev)
    r = joint.decode_joint(pg, s, llr, DecoderParams(kind=kind, lmax=100, **kw), "fp32")
    assert_same(gpu, r, (name, kind, kw, eps))
    say("  FER-free stats: converged %.4f mean rounds %.2f" % (gpu[3].mean(), gpu[2].mean()))


@pytest.mark.parametrize("lmax", [1, 2, 7])
@pytest.mark.parametrize("kind", ["ms", "sagms"])
def test_joint_decode_arbitrary_syndromes_and_priors(dev, lmax, kind):
    """All-zero / all-one / random syndromes, non-uniform, negative and -0.0 priors."""
    name = "G63"
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    _, _, pg = oracle_graph(name)
    s = workloads.random_syndromes(2 * l, 300, seed=lmax)
    rng = np.random.default_rng(23)
    llr = rng.uniform(-1.0, 5.0, size=2 * l).astype(np.float32)
    llr[3] = -0.0
    llr[4] = 0.0
    say("joint arbitrary", kind, lmax)
    gpu = gpu_decode(g, s, llr, sagms.decoder_config(kind, lmax=lmax), dev)
    r = joint.decode_joint(pg, s, llr, DecoderParams(kind=kind, lmax=lmax), "fp32")
    assert_same(gpu, r, (kind, lmax))
    assert (gpu[2][~gpu[3]] == lmax).all()


def test_joint_zero_noise_tiny_batches_and_launch_shapes(dev):
    name = "G63"
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    _, _, pg = oracle_graph(name)
    llr = np.full(2 * l, joint.depolarizing_prior(0.02), dtype=np.float32)
    for nf in (1, 2, 3, 63, 65):
        xh, zh, it, cv, _ = gpu_decode(g, np.zeros((nf, 2 * l), dtype=np.uint8), llr,
                                       sagms.decoder_config("sagms"), dev)
        assert not xh.any() and not zh.any() and (it == 0).all() and cv.all()
    _, _, s = sample(name, 700, 0.05, seed=8)
    r = joint.decode_joint(pg, s, llr, DecoderParams(kind="sagms", lmax=100), "fp32")
    for fpw in (0, 1, 3, 64, 1024):
        gpu = gpu_decode(g, s, llr, sagms.decoder_config("sagms", frames_per_wave=fpw), dev)
        assert_same(gpu, r, ("frames_per_wave", fpw))


# ------------------------------------------------------------------ judge
@pytest.mark.parametrize("name", ["L7", "G63"])
def test_joint_judge_matches_oracle(dev, name):
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    sx, sz, pg = oracle_graph(name)
    nf, eps = 2000, 0.06
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 4, 2, 0, nf, eps, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), joint.depolarizing_prior(eps), dtype=torch.float32, device=dev)
    cfg = sagms.decoder_config("sagms", lmax=40)
    sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    sagms.judge_joint(g, buf["ex"], buf["ez"], buf["ehat"], buf["converged"], buf["iters"], counters,
                      fail=buf["fail"])
    torch.cuda.synchronize()
    ex = channel.unpack(u64(buf["ex"]), g.n)
    ez = channel.unpack(u64(buf["ez"]), g.n)
    e = u64(buf["ehat"])
    xh = channel.unpack(e[:, :g.words_n], g.n)
    zh = channel.unpack(e[:, g.words_n:], g.n)
    conv = buf["converged"].cpu().numpy().astype(bool)
    want = joint.judge_joint(sx, sz, ex, ez, xh, zh, conv)
    got = buf["fail"].cpu().numpy().astype(bool)
    assert (got == want).all()
    c = counters.cpu().numpy()
    assert c[0] == want.sum() and c[1] == buf["iters"].cpu().numpy().astype(np.int64).sum()
    # converged estimates satisfy the syndrome
    assert not (joint.symplectic_syndrome(sx, sz, xh, zh)[conv] ^ channel.unpack(u64(buf["synd"]), g.m)[conv]).any()
    say("joint judge", name, "failures", int(c[0]), "of", nf)


def test_joint_full_size_sampled_frames(dev):
    """2^20 frames of the [[126,28]] code in one launch of the default shape:
    256 sampled frames (the last among them) recomputed by the oracle."""
    name = "G63"
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    sx, sz, pg = oracle_graph(name)
    nf, eps = 1 << 20, 0.03
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 1, 9, 0, nf, eps, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), joint.depolarizing_prior(eps), dtype=torch.float32, device=dev)
    sagms.decode(g, buf["synd"], llr, sagms.decoder_config("sagms", lmax=100), buf["ehat"], buf["iters"],
                 buf["converged"])
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    sagms.judge_joint(g, buf["ex"], buf["ez"], buf["ehat"], buf["converged"], buf["iters"], counters,
                      fail=buf["fail"])
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([np.random.default_rng(5).choice(nf, 255, replace=False), [nf - 1]]))
    ex = np.zeros((len(idx), 2 * l), dtype=np.uint8)
    ez = np.zeros_like(ex)
    for i, f in enumerate(idx):
        x1, z1 = channel.sample_paulis(1, 9, int(f), 1, 2 * l, eps)
        ex[i], ez[i] = x1[0], z1[0]
    s = joint.symplectic_syndrome(sx, sz, ex, ez)
    assert (u64(buf["synd"])[idx] == channel.pack(s)).all()
    r = joint.decode_joint(pg, s, np.full(2 * l, joint.depolarizing_prior(eps), np.float32),
                           DecoderParams(kind="sagms", lmax=100), "fp32")
    e = u64(buf["ehat"])[idx]
    assert (e[:, :g.words_n] == channel.pack(r.xhat)).all() and (e[:, g.words_n:] == channel.pack(r.zhat)).all()
    assert (buf["iters"].cpu().numpy()[idx] == r.iters).all()
    fail = joint.judge_joint(sx, sz, ex, ez, r.xhat, r.zhat, r.converged)
    assert (buf["fail"].cpu().numpy()[idx].astype(bool) == fail).all()
    c = counters.cpu().numpy()
    say("joint 2^20 frames at eps = 0.03: FER %.3e, mean rounds %.3f" % (c[0] / nf, c[1] / nf))


# ------------------------------------------------------------------ FP64
EPS_ROUND = 8 * 2.0 ** -24


def round_bar(G, rnd):
    growth = EPS_ROUND * (G ** rnd - 1.0) / (G - 1.0)
    return 1e-5 if (G <= 2.5 or growth <= 1e-5) else growth


def margins(trace, nframes):
    """Smallest decision margin of every frame's FP64 trajectory over the
    recorded rounds: a belief's distance to 0 or to another belief of the
    same variable (hard-decision ties), or a message's distance to 0 (sign
    ties)."""
    marg = np.full(nframes, np.inf)
    for rd in trace:
        gm = rd["gamma"]
        pair = np.minimum(np.minimum(np.abs(gm[..., 0] - gm[..., 1]), np.abs(gm[..., 0] - gm[..., 2])),
                          np.abs(gm[..., 1] - gm[..., 2]))
        mm = np.minimum(np.minimum(np.abs(gm).min(axis=(1, 2)), pair.min(axis=1)), np.abs(rd["v2c"]).min(axis=1))
        marg[rd["frames"]] = np.minimum(marg[rd["frames"]], mm)
    return marg


@pytest.mark.parametrize("kind,kw", DECODERS)
@pytest.mark.parametrize("eps", [0.02, 0.05])
def test_joint_beliefs_within_tolerance_of_fp64(dev, kind, kw, eps):
    """Beliefs after l = 1..10 rounds against the FP64 oracle (FP32 prior
    promoted), random priors L0 (1 + u), u in [-0.25, 0.25].

    Frames checked in round l: those whose FP64 decision margin (margins())
    exceeds both 1e-4 L0 and 4 times the frame's own largest belief
    deviation, i.e. frames where rounding cannot explain another decision;
    their hard decisions and rounds must be identical.  Belief bar: a message
    to a check carries the errors of the variable's d_v - 1 other outputs
    (in Gamma^A - own) and of the d_v / 2 outputs in min(0, Gamma^P), so a
    round's error gain is at most G = gain * (3 d_v / 2 - 1) = 14 * gain
    here: 1e-5 where 8 2^-24 (G^l - 1)/(G - 1) allows it, that bound after.
    At least half of the frames are checked in every round, for unscaled MS
    (whose FP32 and FP64 trajectories separate by about x3 per round on this
    graph) in rounds 1-7."""
    name = "G63"
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    _, _, pg = oracle_graph(name)
    nf = 400
    _, _, s = sample(name, nf, eps, seed=6)
    rng = np.random.default_rng(int(eps * 1000))
    llr = (joint.depolarizing_prior(eps) * (1.0 + rng.uniform(-0.25, 0.25, 2 * l))).astype(np.float32)
    floor = float(llr.min())
    gain = {"ms": 1.0, "sms": kw.get("alpha", 1.0), "sagms": 0.55}[kind]
    G = gain * (3 * g.dv_max // 2 - 1)
    rows = []
    for rnd in range(1, 11):
        xh, zh, it, cv, gamma = gpu_decode(g, s, llr, sagms.decoder_config(kind, lmax=rnd, **kw), dev)
        r64 = joint.decode_joint(pg, s, llr.astype(np.float64), DecoderParams(kind=kind, lmax=rnd, **kw), "fp64",
                                 trace=True)
        dev_f = np.abs(gamma.astype(np.float64) - r64.gamma).max(axis=(1, 2))
        ok = margins(r64.trace, nf) > np.maximum(1e-4 * floor, 4.0 * dev_f)
        assert (it[ok] == r64.iters[ok]).all() and (xh[ok] == r64.xhat[ok]).all() and (zh[ok] == r64.zhat[ok]).all()
        err = np.abs(gamma[ok].astype(np.float64) - r64.gamma[ok]) / np.maximum(np.abs(r64.gamma[ok]), floor)
        rows.append((rnd, float(err.max()) if err.size else 0.0, float(ok.mean()), round_bar(G, rnd)))
    say("joint per-round max relative error against FP64", kind, kw, eps, "G=%.3g" % G,
        " ".join("l%d:%.2e/%.2f" % (rnd, m, c) for rnd, m, c, _ in rows))
    for rnd, m, c, bar in rows:
        assert m <= bar, (rnd, m, bar)
        if kind != "ms" or rnd <= 7:
            assert c >= 0.5, (rnd, c)


@pytest.mark.parametrize("prior", ["uniform", "random"])
@pytest.mark.parametrize("kind,kw", DECODERS)
def test_joint_fer_matches_fp64(dev, kind, kw, prior):
    """Full-length decoding (l_max = 100) of 4000 frames at eps = 0.05: GPU FER
    (FP32 prior) and FP64-oracle FER (FP64 prior) in each other's 95 % Wilson
    interval; frames converged in both agree on >= 99 %.  Priors: the
    channel's L0, or L0 (1 + u), u uniform in [-0.25, 0.25].  Compared
    within 30 % relative instead: unscaled MS, which on this graph carries
    FP32 rounding forward with a gain of up to 14 per round (measured about
    x3), so that its frames that take many rounds end differently in the two
    precisions with either prior (random prior: the oracle's own FP32 mode
    0.108, FP64 0.086); and, with the uniform prior, SMS, whose dyadic gain
    makes every message an exact combination of L0: exact ties, broken by
    rounding residues that differ between FP32 and FP64 (as for min-sum on
    the binary graph)."""
    name = "G63"
    l, a, b = code_of(name)
    g = sagms.Graph.gb_joint(l, a, b)
    sx, sz, pg = oracle_graph(name)
    nf, eps = 4000, 0.05
    ex, ez, s = sample(name, nf, eps, seed=7)
    L0 = joint.depolarizing_prior(eps)
    llr64 = np.full(2 * l, L0) if prior == "uniform" else L0 * (1.0 + np.random.default_rng(31).uniform(-0.25, 0.25,
                                                                                                        2 * l))
    xh, zh, it, cv, _ = gpu_decode(g, s, llr64.astype(np.float32), sagms.decoder_config(kind, lmax=100, **kw), dev)
    r64 = joint.decode_joint(pg, s, llr64, DecoderParams(kind=kind, lmax=100, **kw), "fp64")
    f_gpu = int(joint.judge_joint(sx, sz, ex, ez, xh, zh, cv).sum())
    f_64 = int(joint.judge_joint(sx, sz, ex, ez, r64.xhat, r64.zhat, r64.converged).sum())
    lo_g, hi_g = stats.wilson(f_gpu, nf)
    lo_o, hi_o = stats.wilson(f_64, nf)
    differ = (xh != r64.xhat).any(axis=1) | (zh != r64.zhat).any(axis=1)
    both = cv & r64.converged
    say("joint FER gpu %.4f fp64 %.4f, frames converged in both that differ %.4f" %
        (f_gpu / nf, f_64 / nf, differ[both].mean()), kind, kw, prior)
    if kind == "ms" or (kind == "sms" and prior == "uniform"):
        assert abs(f_gpu - f_64) <= 0.30 * max(f_gpu, f_64)
    else:
        assert lo_o <= f_gpu / nf <= hi_o and lo_g <= f_64 / nf <= hi_g
    assert differ[both].mean() < 0.01

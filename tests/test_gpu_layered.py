"""GPU parity of the layered schedule (SAGMS_LAYERED) through the C ABI.

Bar: hard decisions, round counts, flags and FP32 posteriors bit-exact
against the oracle's layered FP32 mode (oracle/layered.py) on every code of
the workloads, MS / SMS / SAGMS, arbitrary syndromes and priors, several
l_max, batch sizes from 1 to thousands; at 2^20 frames the launch's frame
assignment is checked by sampled frames and by split batches.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, codes, decoders, layered  # noqa: E402

pytestmark = pytest.mark.gpu

KINDS = [("ms", {}), ("sms", dict(alpha=0.75)), ("sagms", dict(workloads.SAGMS_PARAMS))]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def gpu_layered(g, synd_bits, llr, cfg, dev):
    f = synd_bits.shape[0]
    synd = torch.from_numpy(channel.pack(synd_bits).view(np.int64)).to(dev) if f else \
        torch.empty((0, g.words_m), dtype=torch.int64, device=dev)
    out = sagms.frame_buffers(g, f, device=dev)
    out["ehat"].fill_(-1)
    out["iters"].fill_(-7)
    post = torch.full((f, g.n), float("nan"), dtype=torch.float32, device=dev)
    sagms.decode_soft(g, synd, torch.from_numpy(np.asarray(llr, np.float32)).to(dev), cfg, out["ehat"], out["iters"],
                      out["converged"], post)
    torch.cuda.synchronize()
    return (channel.unpack(out["ehat"].cpu().numpy().view(np.uint64), g.n), out["iters"].cpu().numpy(),
            out["converged"].cpu().numpy().astype(bool), post.cpu().numpy())


def check_against_oracle(name, kind, kw, s, llr, lmax, dev):
    l, a, b = workloads.code(name)
    hz = codes.gb_matrices(l, a, b)[1]
    g = sagms.Graph.gb(l, a, b)
    prm = decoders.DecoderParams(kind=kind, lmax=lmax, **kw)
    r = layered.decode_layered(decoders.TannerGraph(hz), s, np.asarray(llr, np.float32), prm, "fp32")
    say("layered", name, kind, s.shape[0], lmax)
    e, it, cv, post = gpu_layered(g, s, llr, sagms.decoder_config(kind, lmax=lmax, schedule="layered", **kw), dev)
    assert (it == r.iters).all()
    assert (cv == r.converged).all()
    assert (e == r.ehat).all()
    ref = np.asarray(r.posterior, np.float32)
    # unscaled min-sum can overflow FP32 on frames that never converge
    # (messages grow without a gain below 1): inf - inf then gives a NaN
    # whose sign and payload differ between the GPU and the host; NaNs must
    # sit at the same places, every other posterior matches bit for bit
    nan = np.isnan(ref)
    assert (np.isnan(post) == nan).all()
    assert (post.view(np.uint32)[~nan] == ref.view(np.uint32)[~nan]).all()
    return r


@pytest.mark.parametrize("name,nf,p", [("G63", 1500, 0.05), ("G127", 500, 0.04), ("G255w3", 300, 0.04),
                                       ("G255w4", 300, 0.04), ("G511w5", 80, 0.03)])
@pytest.mark.parametrize("kind,kw", KINDS)
def test_layered_bit_exact(dev, name, nf, p, kind, kw):
    l, a, b = workloads.code(name)
    hz = codes.gb_matrices(l, a, b)[1]
    ex, _ = channel.sample_paulis(2, 6, 0, nf, 2 * l, p)
    s = channel.syndrome(hz, ex)
    r = check_against_oracle(name, kind, kw, s, np.full(2 * l, channel.prior_llr(p), np.float32), 100, dev)
    assert r.converged.mean() > 0.3


@pytest.mark.parametrize("lmax", [1, 2, 7])
@pytest.mark.parametrize("kind,kw", KINDS)
def test_layered_arbitrary_inputs(dev, lmax, kind, kw):
    """Random, all-zero and all-one syndromes; priors with negative entries
    and signed zeros."""
    l, a, b = workloads.code("G63")
    rng = np.random.default_rng(lmax)
    s = rng.integers(0, 2, (200, l)).astype(np.uint8)
    s[0] = 0
    s[1] = 1
    llr = rng.normal(2.0, 1.5, 2 * l).astype(np.float32)
    llr[:5] = [-0.0, 0.0, -1.0, -2.5, 0.25]
    check_against_oracle("G63", kind, kw, s, llr, lmax, dev)


@pytest.mark.parametrize("nf", [0, 1, 2, 7, 8, 9, 15, 16, 17, 63, 65])
@pytest.mark.parametrize("name", ["G127", "G63"])
def test_layered_small_batches(dev, name, nf):
    l, a, b = workloads.code(name)
    hz = codes.gb_matrices(l, a, b)[1]
    ex, _ = channel.sample_paulis(5, 1, 0, max(nf, 1), 2 * l, 0.05)
    s = channel.syndrome(hz, ex)[:nf]
    if nf == 0:
        g = sagms.Graph.gb(l, a, b)
        e, it, cv, post = gpu_layered(g, s, np.full(2 * l, 3.0, np.float32),
                                      sagms.decoder_config("sagms", schedule="layered"), dev)
        assert it.size == 0
        return
    check_against_oracle(name, "sagms", dict(workloads.SAGMS_PARAMS), s,
                         np.full(2 * l, channel.prior_llr(0.05), np.float32), 100, dev)


def test_layered_full_size(dev):
    """2^20 frames of the l = 63 workload in the default launch: 256 sampled
    frames (with the first and last) recomputed by the oracle; the same
    frames decoded as two halves on two streams give identical outputs."""
    l, a, b = workloads.code("G63")
    hz = codes.gb_matrices(l, a, b)[1]
    g = sagms.Graph.gb(l, a, b)
    p, nf = 0.05, 1 << 20
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 1, workloads.stream_of(p), 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    cfg = sagms.decoder_config("sagms", schedule="layered", **workloads.SAGMS_PARAMS)
    say("layered full size")
    sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    half = nf // 2
    e2 = torch.empty_like(buf["ehat"])
    i2 = torch.empty_like(buf["iters"])
    c2 = torch.empty_like(buf["converged"])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        sagms.decode(g, buf["synd"][:half], llr, cfg, e2[:half], i2[:half], c2[:half], stream=s1)
    with torch.cuda.stream(s2):
        sagms.decode(g, buf["synd"][half:], llr, cfg, e2[half:], i2[half:], c2[half:], stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(e2, buf["ehat"]) and torch.equal(i2, buf["iters"]) and torch.equal(c2, buf["converged"])
    rng = np.random.default_rng(11)
    pick = np.unique(np.concatenate([[0, nf - 1], rng.integers(0, nf, 254)]))
    s = channel.unpack(buf["synd"][torch.from_numpy(pick).to(dev)].cpu().numpy().view(np.uint64), l)
    prm = decoders.DecoderParams(kind="sagms", lmax=100, **workloads.SAGMS_PARAMS)
    r = layered.decode_layered(decoders.TannerGraph(hz), s, np.full(2 * l, sagms.prior_llr(p), np.float32), prm,
                               "fp32")
    e = channel.unpack(buf["ehat"].cpu().numpy().view(np.uint64)[pick], g.n)
    assert (e == r.ehat).all()
    assert (buf["iters"].cpu().numpy()[pick] == r.iters).all()
    assert (buf["converged"].cpu().numpy()[pick].astype(bool) == r.converged).all()


@pytest.mark.parametrize("kind,kw", KINDS)
def test_layered_general_kernel_on_the_l63_code(dev, kind, kw):
    """The l = 63 matrix with its rows permuted is not the compiled matrix of
    the one-lane kernel, so it runs on the general kernel (groups of lanes):
    against the oracle's layered FP32 mode on the permuted matrix."""
    l, a, b = workloads.code("G63")
    hz = codes.gb_matrices(l, a, b)[1]
    perm = np.random.default_rng(8).permutation(l)
    h = hz[perm]
    g = sagms.Graph.from_dense(h)
    assert g.layered_group >= 8
    ex, _ = channel.sample_paulis(3, 6, 0, 700, 2 * l, 0.05)
    s = channel.syndrome(h, ex)
    llr = np.full(2 * l, channel.prior_llr(0.05), np.float32)
    prm = decoders.DecoderParams(kind=kind, lmax=100, **kw)
    r = layered.decode_layered(decoders.TannerGraph(h), s, llr, prm, "fp32")
    say("layered general kernel, permuted l = 63 rows", kind)
    e, it, cv, post = gpu_layered(g, s, llr, sagms.decoder_config(kind, lmax=100, schedule="layered", **kw), dev)
    assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
    ref = np.asarray(r.posterior, np.float32)
    nan = np.isnan(ref)
    assert (np.isnan(post) == nan).all()
    assert (post.view(np.uint32)[~nan] == ref.view(np.uint32)[~nan]).all()


@pytest.mark.parametrize("alpha", [0.5, 0.625, 0.875, 1.0])
def test_layered_lane_kernel_sms_gains(dev, alpha):
    """SMS with the other gains of the paper's SMS sweep (and 1.0, plain
    min-sum through the SMS path) on the one-lane kernel of the l = 63 code,
    two noise levels: bit-exact against the oracle's layered FP32 mode."""
    l, a, b = workloads.code("G63")
    hz = codes.gb_matrices(l, a, b)[1]
    for p, seed in ((0.04, 11), (0.08, 12)):
        ex, _ = channel.sample_paulis(seed, 6, 0, 800, 2 * l, p)
        s = channel.syndrome(hz, ex)
        check_against_oracle("G63", "sms", dict(alpha=alpha), s, np.full(2 * l, channel.prior_llr(p), np.float32),
                             100, dev)


def test_layered_lane_kernel_ragged_launch(dev):
    """The one-lane kernel of the l = 63 code over 2^16 + 37 frames (runs of
    frames per wavefront that do not divide evenly, a last wavefront with
    fewer frames than lanes): hard decisions, rounds, flags and posteriors of
    300 sampled frames, the last 37 among them, against the oracle."""
    l, a, b = workloads.code("G63")
    hz = codes.gb_matrices(l, a, b)[1]
    g = sagms.Graph.gb(l, a, b)
    assert g.layered_group == 1
    p, nf = 0.06, (1 << 16) + 37
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 4, 7, 1 << 33, nf, p, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    post = torch.full((nf, g.n), float("nan"), dtype=torch.float32, device=dev)
    cfg = sagms.decoder_config("sagms", schedule="layered", **workloads.SAGMS_PARAMS)
    say("layered one-lane kernel, ragged launch", nf)
    sagms.decode_soft(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"], post)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    pick = np.unique(np.concatenate([np.arange(nf - 37, nf), rng.integers(0, nf, 263)]))
    s = channel.unpack(buf["synd"][torch.from_numpy(pick).to(dev)].cpu().numpy().view(np.uint64), l)
    prm = decoders.DecoderParams(kind="sagms", lmax=100, **workloads.SAGMS_PARAMS)
    r = layered.decode_layered(decoders.TannerGraph(hz), s, np.full(2 * l, sagms.prior_llr(p), np.float32), prm,
                               "fp32")
    e = channel.unpack(buf["ehat"].cpu().numpy().view(np.uint64)[pick], g.n)
    assert (e == r.ehat).all()
    assert (buf["iters"].cpu().numpy()[pick] == r.iters).all()
    assert (buf["converged"].cpu().numpy()[pick].astype(bool) == r.converged).all()
    got = post.cpu().numpy()[pick]
    assert (got.view(np.uint32) == np.asarray(r.posterior, np.float32).view(np.uint32)).all()
    assert (buf["iters"].cpu().numpy() >= 0).all()  # every frame written


def test_layered_layer_wider_than_a_wavefront(dev):
    """80 checks with disjoint supports (one layer, wider than a wavefront,
    so it spans several passes whatever the group size) plus 10 checks
    across them (further layers), degree 6, n = 480: against the oracle's
    layered FP32 mode."""
    rng = np.random.default_rng(21)
    m0, n = 80, 480
    h = np.zeros((m0 + 10, n), dtype=np.uint8)
    for i in range(m0):
        h[i, 6 * i:6 * i + 6] = 1
    for i in range(10):
        blocks = rng.choice(m0, 6, replace=False)
        h[m0 + i, 6 * blocks + rng.integers(0, 6, 6)] = 1
    assert h.sum(axis=0).max() <= 3 and (h.sum(axis=1) == 6).all()
    lay = layered.greedy_layers(h)
    assert len(lay[0]) > 64 and len(lay) > 1
    g = sagms.Graph.from_dense(h)
    assert g.layered_passes * g.layered_group >= m0 + 10 and g.layered_passes > 1
    s = rng.integers(0, 2, (96, h.shape[0])).astype(np.uint8)
    llr = rng.uniform(1.0, 4.0, n).astype(np.float32)
    for kind, kw in KINDS:
        prm = decoders.DecoderParams(kind=kind, lmax=30, **kw)
        r = layered.decode_layered(decoders.TannerGraph(h), s, llr, prm, "fp32")
        say("layered wide layer", kind)
        e, it, cv, post = gpu_layered(g, s, llr, sagms.decoder_config(kind, lmax=30, schedule="layered", **kw), dev)
        assert (it == r.iters).all() and (cv == r.converged).all() and (e == r.ehat).all()
        ref = np.asarray(r.posterior, np.float32)
        nan = np.isnan(ref)
        assert (np.isnan(post) == nan).all()
        assert (post.view(np.uint32)[~nan] == ref.view(np.uint32)[~nan]).all()


def test_layered_refused_where_not_built(dev):
    g = sagms.Graph.gb(*workloads.code("G63"))
    synd = torch.zeros((4, g.words_m), dtype=torch.int64, device=dev)
    out = sagms.frame_buffers(g, 4, device=dev)
    llr = torch.full((g.n,), 3.0, dtype=torch.float32, device=dev)
    with pytest.raises(sagms.SagmsError):
        sagms.decode(g, synd, llr, sagms.decoder_config("bp", schedule="layered"), out["ehat"], out["iters"],
                     out["converged"])
    # a graph with checks of different degrees
    h = np.zeros((4, 12), dtype=np.int32)
    for i, cols in enumerate([[0, 1, 2, 3, 4, 5], [2, 3, 6, 7, 8, 9], [4, 5, 8, 9, 10, 11], [0, 1, 6, 7]]):
        h[i, cols] = 1
    g2 = sagms.Graph.from_dense(h)
    synd2 = torch.zeros((4, g2.words_m), dtype=torch.int64, device=dev)
    out2 = sagms.frame_buffers(g2, 4, device=dev)
    llr2 = torch.full((g2.n,), 3.0, dtype=torch.float32, device=dev)
    with pytest.raises(sagms.SagmsError, match="same degree"):
        sagms.decode(g2, synd2, llr2, sagms.decoder_config("ms", schedule="layered"), out2["ehat"], out2["iters"],
                     out2["converged"])

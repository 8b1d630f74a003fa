"""Paper-faithful variants on the GPU: derived SAGMS gains (Corollary 1),
channel mismatch (decoding with the prior of p0 != p, Section V) and the
Monte Carlo stopping rule of the Section V setup (500 failures or a frame
cap) of the sweep tool.  Decoding results bit-exact against the oracle's
FP32 mode; the stopping rule against its definition.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import analysis, channel, codes, decoders  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run(g, hz, l, a, b, p, p0, cfg, prm, dev, nf=400, stream_id=9):
    ex, _ = channel.sample_paulis(1, stream_id, 0, nf, 2 * l, p)
    s = channel.syndrome(hz, ex)
    llr = np.full(2 * l, channel.prior_llr(p0), dtype=np.float32)
    r = decoders.decode(decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b)), s, llr, prm, "fp32")
    synd = torch.from_numpy(channel.pack(s).view(np.int64)).to(dev)
    out = sagms.frame_buffers(g, nf, device=dev)
    post = torch.empty((nf, g.n), dtype=torch.float32, device=dev)
    sagms.decode_soft(g, synd, torch.from_numpy(llr).to(dev), cfg, out["ehat"], out["iters"], out["converged"], post)
    torch.cuda.synchronize()
    assert (out["ehat"].cpu().numpy().view(np.uint64) == channel.pack(r.ehat)).all()
    assert (out["iters"].cpu().numpy() == r.iters).all()
    assert (out["converged"].cpu().numpy() == r.converged).all()
    assert (post.cpu().numpy().view(np.uint32) == np.asarray(r.posterior, np.float32).view(np.uint32)).all()
    return r


@pytest.mark.parametrize("name", ["G63", "G255w3"])
@pytest.mark.parametrize("eta", [0.0, 1.1])
@pytest.mark.parametrize("p", [0.03, 0.06])
def test_derived_gains_bit_exact(dev, name, eta, p):
    l, a, b = workloads.code(name)
    hx, hz = codes.gb_matrices(l, a, b)
    g = sagms.Graph.gb(l, a, b)
    l0 = channel.prior_llr(p)
    cfg = sagms.derived_config(l0, g.dc_max, ratio=0.6, eta=eta, lmax=60)
    amax = analysis.alpha_star(l0, g.dc_max)
    assert cfg.alpha_max == pytest.approx(amax, rel=1e-12)
    prm = decoders.DecoderParams(kind="sagms", lmax=60, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max, eta=cfg.eta)
    print("derived", name, eta, p, cfg.alpha_min, cfg.alpha_max, cfg.eta, flush=True)
    run(g, hz, l, a, b, p, p, cfg, prm, dev)


@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.5)), ("sagms", {})])
@pytest.mark.parametrize("p", [0.01, 0.03])
def test_mismatched_prior_bit_exact(dev, kind, kw, p):
    l, a, b = workloads.code("G63")
    hx, hz = codes.gb_matrices(l, a, b)
    g = sagms.Graph.gb(l, a, b)
    cfg = sagms.decoder_config(kind, lmax=50, **kw)
    prm = decoders.DecoderParams(kind=kind, lmax=50, **kw)
    print("mismatch", kind, p, flush=True)
    run(g, hz, l, a, b, p, 0.1, cfg, prm, dev, stream_id=11)


def test_sweep_stopping_rule(dev):
    from paper_2605_10433_amd import sweep
    g = sagms.Graph.gb(*workloads.code("G63"))
    r = sweep.run_point(g, "G63", 0.08, 3, "ms", 30, until_failures=200, max_frames=3 << 20)
    assert r["failures"] >= 200 and r["frames"] <= 3 << 20
    # the rule is checked after every chunk of up to 2^20 frames
    r2 = sweep.run_point(g, "G63", 0.08, 3, "ms", 30, frames=r["frames"])
    assert r2["failures"] == r["failures"] and r2["mean_iters"] == r["mean_iters"]
    r3 = sweep.run_point(g, "G63", 0.01, 3, "sagms", 30, until_failures=10 ** 9, max_frames=1 << 19)
    assert r3["frames"] == 1 << 19                                             # frame cap
    r4 = sweep.run_point(g, "G63", 0.03, 3, "sagms-derived", 30, frames=5000, p0=0.1)
    assert r4["p0"] == 0.1 and r4["gains"][1] == pytest.approx(analysis.alpha_star(channel.prior_llr(0.1), 10))

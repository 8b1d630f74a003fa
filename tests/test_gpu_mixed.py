"""Mixed-code batches on the GPU (through the C ABI).

A frame decoded in a batch must equal, bit for bit, the same frame decoded
by sagms_decode on its own code (which the parity tests pin to the oracle),
and the oracle itself on sampled frames: hard decisions, round counts,
convergence flags and posteriors, for every launch plan, message format and
mix, for eager launches, graph replays and tuned plans.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, codes, decoders  # noqa: E402

pytestmark = pytest.mark.gpu

SMALL = {"L7b": (7, [0, 1, 3], [0, 2, 6])}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*args):
    print(*args, flush=True)


def code_of(name):
    return SMALL[name] if name in SMALL else workloads.code(name)


_graphs = {}


def graph(name):
    if name not in _graphs:
        _graphs[name] = sagms.Graph.gb(*code_of(name))
    return _graphs[name]


def make_segment(name, nf, p, stream_id, dev, frame0=0, soft=True):
    g = graph(name)
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, workloads.MIX_SEED, stream_id, frame0, nf, p, buf["ex"], None, buf["synd"])
    seg = dict(graph=g, synd=buf["synd"], ex=buf["ex"],
               llr0=torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev),
               ehat=torch.full((nf, g.words_n), -1, dtype=torch.int64, device=dev),
               iters=torch.full((nf,), -1, dtype=torch.int32, device=dev),
               converged=torch.full((nf,), 7, dtype=torch.uint8, device=dev),
               name=name, p=p, stream_id=stream_id, frame0=frame0)
    if soft:
        seg["posterior"] = torch.full((nf, g.n), float("nan"), dtype=torch.float32, device=dev)
    return seg


def reference(seg, cfg):
    """The same frames through sagms_decode_soft on their own code."""
    g = seg["graph"]
    nf = seg["synd"].shape[0]
    out = sagms.frame_buffers(g, nf, device=seg["synd"].device)
    post = torch.empty((nf, g.n), dtype=torch.float32, device=seg["synd"].device)
    sagms.decode_soft(g, seg["synd"], seg["llr0"], cfg, out["ehat"], out["iters"], out["converged"], post)
    torch.cuda.synchronize()
    return dict(ehat=out["ehat"].cpu(), iters=out["iters"].cpu(), converged=out["converged"].cpu(), posterior=post.cpu())


def assert_same(seg, ref, tag=""):
    for key in ("ehat", "iters", "converged"):
        got = seg[key].cpu()
        assert torch.equal(got, ref[key]), "%s %s: %s differs" % (tag, seg["name"], key)
    if "posterior" in seg:
        a = seg["posterior"].cpu().numpy().view(np.uint32)
        b = ref["posterior"].numpy().view(np.uint32)
        assert (a == b).all(), "%s %s: posterior differs" % (tag, seg["name"])


def clear(segs):
    for s in segs:
        s["ehat"].fill_(-1)
        s["iters"].fill_(-1)
        s["converged"].fill_(7)
        if "posterior" in s:
            s["posterior"].fill_(float("nan"))
    torch.cuda.synchronize()


MIX = [("G127", 1000), ("G255w3", 777), ("G255w4", 513), ("G63", 301)]


def mix_segments(dev, p=0.04, mix=MIX, soft=True):
    return [make_segment(name, nf, p, workloads.mix_stream(i, p), dev, soft=soft) for i, (name, nf) in enumerate(mix)]


PLANS = [dict(kind="single", tile_frames=t, waves_per_block=w, reg_budget=r, unroll=u)
         for t, w, r, u in ((1, 4, 0, 1), (7, 4, 0, 2), (32, 1, 0, 1), (8, 2, 1, 2), (3, 4, 1, 1), (5, 1, 1, 2))] + \
        [dict(kind="tiered", tile_frames=5, waves_per_block=2), dict(kind="tiered", tile_frames=16, reg_budget=1),
         dict(kind="tiered", tile_frames=2, reg_budget=1, unroll=2), dict(kind="per_code", tile_frames=3),
         dict(kind="single", tile_frames=4, blocks_per_cu=1), dict(kind="single", tile_frames=6, unroll=0)]


@pytest.mark.parametrize("precision", ["fp32", "fp16", "int6"])
def test_mixed_batch_equals_per_code_decode(dev, precision):
    segs = mix_segments(dev)
    cfg = sagms.decoder_config("sagms", lmax=100, precision=precision)
    refs = [reference(s, cfg) for s in segs]
    batch = sagms.Batch(segs, cfg)
    for pl in PLANS:
        say("mixed", precision, pl)
        clear(segs)
        batch.set_plan(sagms.plan(**pl))
        batch.run()
        torch.cuda.synchronize()
        for s, r in zip(segs, refs):
            assert_same(s, r, str(pl))
    batch.close()


@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.625))])
def test_mixed_batch_other_decoders(dev, kind, kw):
    segs = mix_segments(dev, p=0.05)
    cfg = sagms.decoder_config(kind, lmax=30, **kw)
    refs = [reference(s, cfg) for s in segs]
    batch = sagms.Batch(segs, cfg)
    for pl in (dict(kind="single", tile_frames=8), dict(kind="tiered", tile_frames=2)):
        say("mixed", kind, pl)
        clear(segs)
        batch.set_plan(sagms.plan(**pl))
        batch.run()
        torch.cuda.synchronize()
        for s, r in zip(segs, refs):
            assert_same(s, r, kind)


def test_mixed_batch_against_oracle_sample(dev):
    """Independent of sagms_decode: the first frames of every segment against
    the oracle's FP32 mode (its own sampler, syndromes and decoder)."""
    segs = mix_segments(dev)
    cfg = sagms.decoder_config("sagms", lmax=100)
    batch = sagms.Batch(segs, cfg)
    batch.run()
    torch.cuda.synchronize()
    for s in segs:
        l, a, b = code_of(s["name"])
        hx, hz = codes.gb_matrices(l, a, b)
        nf = 48
        ex, _ = channel.sample_paulis(workloads.MIX_SEED, s["stream_id"], 0, nf, 2 * l, s["p"])
        synd = channel.syndrome(hz, ex)
        llr = np.full(2 * l, channel.prior_llr(s["p"]), dtype=np.float32)
        r = decoders.decode(decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b)), synd, llr,
                            decoders.DecoderParams(kind="sagms", lmax=100), "fp32")
        say("oracle sample", s["name"])
        assert (s["ehat"][:nf].cpu().numpy().view(np.uint64) == channel.pack(r.ehat)).all()
        assert (s["iters"][:nf].cpu().numpy() == r.iters).all()
        assert (s["converged"][:nf].cpu().numpy() == r.converged).all()
        assert (s["posterior"][:nf].cpu().numpy().view(np.uint32) ==
                np.asarray(r.posterior, dtype=np.float32).view(np.uint32)).all()


def test_graph_replays_with_new_syndromes(dev):
    """Instantiate once; replay on new syndromes written in place between the
    replays (eager sampler launches on the same stream); check every replay."""
    segs = mix_segments(dev)
    cfg = sagms.decoder_config("sagms", lmax=100)
    batch = sagms.Batch(segs, cfg)
    batch.set_plan(sagms.plan("single", tile_frames=4))
    batch.instantiate()
    for rep in range(4):
        say("graph replay", rep)
        for s in segs:
            g = s["graph"]
            nf = s["synd"].shape[0]
            sagms.gen_errors(g, workloads.MIX_SEED, s["stream_id"], 1000 * rep, nf, s["p"], s["ex"], None, s["synd"])
        torch.cuda.synchronize()
        refs = [reference(s, cfg) for s in segs]
        clear(segs)
        batch.run()
        torch.cuda.synchronize()
        for s, r in zip(segs, refs):
            assert_same(s, r, "replay %d" % rep)
    # a new plan drops the graph; instantiating the tiered plan replays too
    batch.set_plan(sagms.plan("tiered", tile_frames=8))
    batch.instantiate()
    refs = [reference(s, cfg) for s in segs]
    for rep in range(2):
        clear(segs)
        batch.run()
        torch.cuda.synchronize()
        for s, r in zip(segs, refs):
            assert_same(s, r, "tiered replay %d" % rep)


def test_autotuner_returns_a_valid_plan(dev):
    segs = mix_segments(dev, mix=[("G127", 3000), ("G63", 2000)], soft=False)
    cfg = sagms.decoder_config("sagms", lmax=100)
    refs = [reference(s, cfg) for s in segs]
    batch = sagms.Batch(segs, cfg)
    best, results = batch.tune(reps=1)
    say("tuned", best.as_dict(), len(results))
    assert len(results) >= 10
    assert {pl["unroll"] for pl, _ in results if pl["kind"] != "per_code"} == {1, 2}
    assert best.as_dict() == batch.get_plan().as_dict()
    assert min(ms for _, ms in results) == pytest.approx(
        [ms for pl, ms in results if pl == best.as_dict()][0])
    clear(segs)
    batch.run()
    torch.cuda.synchronize()
    for s, r in zip(segs, refs):
        assert_same(s, r, "tuned")


def test_edge_mixes(dev):
    cfg = sagms.decoder_config("sagms", lmax=100)
    cases = [
        [("G63", 1)],                                            # one frame
        [("G63", 0), ("G127", 65), ("L7b", 0)],                  # empty segments
        [("L7b", 129), ("G511w5", 70), ("G63", 64)],             # the largest shape beside the smallest
        [("G63", 17 + i) for i in range(16)],                    # the maximum segment count
    ]
    for ci, mix in enumerate(cases):
        segs = [make_segment(name, nf, 0.05, 500 + ci * 20 + i, dev) for i, (name, nf) in enumerate(mix)]
        refs = [reference(s, cfg) if s["synd"].shape[0] else None for s in segs]
        batch = sagms.Batch(segs, cfg)
        for pl in (dict(kind="single", tile_frames=3, waves_per_block=1), dict(kind="tiered", tile_frames=1),
                   dict(kind="per_code", tile_frames=2)):
            say("edge mix", ci, pl)
            clear(segs)
            batch.set_plan(sagms.plan(**pl))
            batch.run()
            torch.cuda.synchronize()
            for s, r in zip(segs, refs):
                if r is not None:
                    assert_same(s, r, "edge %d %s" % (ci, pl))
        batch.close()


def test_plan_and_argument_checks(dev):
    segs = mix_segments(dev, mix=[("G63", 10), ("G511w5", 10)], soft=False)
    cfg = sagms.decoder_config("sagms")
    batch = sagms.Batch(segs, cfg)
    for bad in (dict(tile_frames=0), dict(tile_frames=2000), dict(waves_per_block=3), dict(blocks_per_cu=-1),
                dict(reg_budget=2), dict(unroll=3), dict(unroll=-1)):
        with pytest.raises(sagms.SagmsError) as e:
            batch.set_plan(sagms.plan(**bad))
        assert e.value.code == sagms.EINVAL
    batch.set_plan(sagms.plan("single", waves_per_block=2, reg_budget=1))  # no tight budget there: compiler's
    batch.set_plan(sagms.plan("single", waves_per_block=4))                  # l = 511: halved to fit 64 KiB
    batch.run()
    torch.cuda.synchronize()
    batch.set_plan(sagms.plan("per_code", waves_per_block=3))                # ignored by the per-code plan
    with pytest.raises(sagms.SagmsError):
        sagms.Batch(segs, sagms.decoder_config("bp"))


def test_full_mix_sampled_frames(dev):
    """The full mixed workload (2^22 frames) in one persistent launch; 64
    frames of each code, spread over the segment, against the oracle."""
    cfg = sagms.decoder_config("sagms", lmax=workloads.MIX_LMAX)
    segs = [make_segment(name, nf, workloads.MIX_P, workloads.mix_stream(i, workloads.MIX_P), dev, soft=False)
            for i, (name, nf) in enumerate(zip(workloads.MIX_CODES, workloads.MIX_FRAMES))]
    batch = sagms.Batch(segs, cfg)
    batch.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    for s in segs:
        l, a, b = code_of(s["name"])
        hx, hz = codes.gb_matrices(l, a, b)
        nf = s["synd"].shape[0]
        pick = np.sort(rng.choice(nf, 64, replace=False))
        pick[-1] = nf - 1
        tg = decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b))
        llr = np.full(2 * l, channel.prior_llr(s["p"]), dtype=np.float32)
        ehat = s["ehat"].cpu().numpy().view(np.uint64)
        iters = s["iters"].cpu().numpy()
        conv = s["converged"].cpu().numpy()
        say("full mix sample", s["name"], nf)
        for f in pick:
            ex, _ = channel.sample_paulis(workloads.MIX_SEED, s["stream_id"], int(f), 1, 2 * l, s["p"])
            r = decoders.decode(tg, channel.syndrome(hz, ex), llr, decoders.DecoderParams(kind="sagms", lmax=100),
                                "fp32")
            assert (ehat[f] == channel.pack(r.ehat)[0]).all(), (s["name"], f)
            assert iters[f] == r.iters[0] and conv[f] == r.converged[0], (s["name"], f)
        # every frame was written
        assert (iters >= 0).all() and (conv <= 1).all()

"""sagms_decode_segments, the mixed-code decode that allocates nothing (its
queue counters live in a static device array), against sagms_batch_run on
the same segments: bit-exact hard decisions, round counts, flags and
posteriors, on two calls in a row, the second with fewer frames, for every
launch plan and for FP16 messages; sampled frames also against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, codes, decoders  # noqa: E402

pytestmark = pytest.mark.gpu

MIX = ["G127", "G255w3", "G255w4", "G63"]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*args):
    print(*args, flush=True)


def segments(frames, p, dev, frame0):
    segs = []
    for i, name in enumerate(MIX):
        g = sagms.Graph.gb(*workloads.code(name))
        nf = frames[i]
        buf = sagms.frame_buffers(g, nf, device=dev)
        sagms.gen_errors(g, workloads.MIX_SEED, i, frame0, nf, p, buf["ex"], None, buf["synd"])
        segs.append(dict(graph=g, synd=buf["synd"], name=name,
                         llr0=torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev),
                         ehat=torch.full((nf, g.words_n), -1, dtype=torch.int64, device=dev),
                         iters=torch.full((nf,), -1, dtype=torch.int32, device=dev),
                         converged=torch.full((nf,), 7, dtype=torch.uint8, device=dev),
                         posterior=torch.full((nf, g.n), float("nan"), dtype=torch.float32, device=dev)))
    torch.cuda.synchronize()
    return segs


def outputs(segs):
    return [{k: s[k].cpu().clone() for k in ("ehat", "iters", "converged", "posterior")} for s in segs]


def clobber(segs):
    for s in segs:
        s["ehat"].fill_(-1)
        s["iters"].fill_(-1)
        s["converged"].fill_(7)
        s["posterior"].fill_(float("nan"))


PLANS = [None, sagms.plan("single", tile_frames=4, waves_per_block=2),
         sagms.plan("tiered", tile_frames=16, unroll=2), sagms.plan("per_code", tile_frames=8)]


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
@pytest.mark.parametrize("plan_index", range(len(PLANS)))
def test_decode_segments_equals_batch_run(dev, precision, plan_index):
    plan = PLANS[plan_index]
    cfg = sagms.decoder_config("sagms", lmax=100, precision=precision)
    p = 0.04
    for call, frames in enumerate(([3001, 2002, 1503, 777], [501, 97, 333, 64])):
        say("decode_segments", precision, plan.as_dict() if plan else "default", "call", call, frames)
        segs = segments(frames, p, dev, frame0=1000 * call)
        b = sagms.Batch(segs, cfg)
        if plan is not None:
            b.set_plan(plan)
        b.run()
        torch.cuda.synchronize()
        want = outputs(segs)
        b.close()
        clobber(segs)
        torch.cuda.synchronize()
        sagms.decode_segments(segs, cfg, plan)
        torch.cuda.synchronize()
        got = outputs(segs)
        for s, w, o in zip(segs, want, got):
            for k in ("ehat", "iters", "converged"):
                assert torch.equal(w[k], o[k]), (s["name"], k, call)
            assert (w["posterior"].numpy().view(np.uint32) == o["posterior"].numpy().view(np.uint32)).all(), \
                (s["name"], call)
        # sampled frames of the first and last segment against the oracle
        for s, o in ((segs[0], got[0]), (segs[-1], got[-1])):
            l, a, bb = workloads.code(s["name"])
            hz = codes.gb_matrices(l, a, bb)[1]
            tg = decoders.TannerGraph(hz, codes.gb_var_checks(l, a, bb))
            idx = np.arange(0, s["synd"].shape[0], 7)
            sb = channel.unpack(s["synd"].cpu().numpy().view(np.uint64)[idx], tg.m)
            r = decoders.decode(tg, sb, np.full(tg.n, sagms.prior_llr(p), np.float32),
                                decoders.DecoderParams(kind="sagms", lmax=100), precision)
            assert (o["ehat"].numpy().view(np.uint64)[idx] == channel.pack(r.ehat)).all(), s["name"]
            assert (o["iters"].numpy()[idx] == r.iters).all(), s["name"]


def test_decode_segments_refuses_more_than_sixteen(dev):
    segs = segments([8, 8, 8, 8], 0.04, dev, 0)
    cfg = sagms.decoder_config("sagms", lmax=100)
    with pytest.raises(sagms.SagmsError) as e:
        sagms.decode_segments(segs * 5, cfg)
    assert e.value.code == sagms.EINVAL

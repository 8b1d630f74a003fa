"""The device calls allocate nothing: a graph's first sampling and decode calls,
with a decoder configuration never used before in the process, are captured
into a CUDA/HIP graph and replayed; decodes of a new configuration on two
streams at once; padding bits of the syndrome words are ignored by both
schedules.  Every result is checked bit for bit against the CPU oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, codes, decoders  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*args):
    print(*args, flush=True)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def oracle_decode(name, synd_bits, llr, kind, lmax, schedule="flooding", precision="fp32", **kw):
    l, a, b = workloads.code(name)
    hx, hz = codes.gb_matrices(l, a, b)
    tg = decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b))
    p = decoders.DecoderParams(kind=kind, lmax=lmax, **kw)
    if schedule == "layered":
        from oracle import layered
        return layered.decode_layered(tg, synd_bits, llr, p, "fp32")
    return decoders.decode(tg, synd_bits, llr, p, precision)


CAPTURE_CASES = [
    # (code, kind, schedule, precision, gains): gains chosen so that no other
    # test of the session uses the same configuration first
    ("G63", "sagms", "flooding", "fp32", dict(alpha_min=0.3125, alpha_max=0.4375, eta=1.125)),
    ("G127", "sms", "flooding", "fp16", dict(alpha=0.6875)),
    ("G63", "sagms", "layered", "fp32", dict(alpha_min=0.28, alpha_max=0.52, eta=1.5)),
]


@pytest.mark.parametrize("name,kind,schedule,precision,gains", CAPTURE_CASES)
def test_first_calls_under_graph_capture(dev, name, kind, schedule, precision, gains):
    say("capture", name, kind, schedule, precision, gains)
    l, a, b = workloads.code(name)
    g = sagms.Graph.gb(l, a, b)  # new handle: its first device calls are captured
    nf, p, seed, stream_id, lmax = 1500, 0.06, 11, 3, 60
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    cfg = sagms.decoder_config(kind, lmax=lmax, schedule=schedule, precision=precision, **gains)
    buf = sagms.frame_buffers(g, nf, device=dev)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sagms.gen_errors(g, seed, stream_id, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
        sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    torch.cuda.synchronize()

    ex, _ = channel.sample_paulis(seed, stream_id, 0, nf, g.n, p)
    hz = codes.gb_matrices(l, a, b)[1]
    s = channel.syndrome(hz, ex)
    r = oracle_decode(name, s, np.full(g.n, sagms.prior_llr(p), np.float32), kind, lmax, schedule,
                      precision, **gains)
    for rep in range(3):
        for t in buf.values():  # clobber the outputs between replays (eager work)
            if t is not None:
                t.fill_(85)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert (u64(buf["ex"]) == channel.pack(ex)).all(), rep
        assert (u64(buf["synd"]) == channel.pack(s)).all(), rep
        assert (u64(buf["ehat"]) == channel.pack(r.ehat)).all(), rep
        assert (buf["iters"].cpu().numpy() == r.iters).all(), rep
        assert (buf["converged"].cpu().numpy() == r.converged).all(), rep
    say("  replays bit-exact; mean iterations", float(r.iters.mean()))


def test_new_configuration_on_two_streams(dev):
    l, a, b = workloads.code("G255w4")
    g = sagms.Graph.gb(l, a, b)
    nf, p = 2048, 0.045
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 5, 1, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    gains = dict(alpha_min=0.35, alpha_max=0.55, eta=1.25)
    cfg = sagms.decoder_config("sagms", lmax=80, **gains)
    outs = [sagms.frame_buffers(g, nf, device=dev) for _ in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st, o in zip(streams, outs):
        with torch.cuda.stream(st):
            sagms.decode(g, buf["synd"], llr, cfg, o["ehat"], o["iters"], o["converged"])
    torch.cuda.synchronize()
    s = channel.unpack(u64(buf["synd"]), g.m)
    r = oracle_decode("G255w4", s, np.full(g.n, sagms.prior_llr(p), np.float32), "sagms", 80, **gains)
    for o in outs:
        assert (u64(o["ehat"]) == channel.pack(r.ehat)).all()
        assert (o["iters"].cpu().numpy() == r.iters).all()
        assert (o["converged"].cpu().numpy() == r.converged).all()


@pytest.mark.parametrize("schedule", ["flooding", "layered"])
@pytest.mark.parametrize("name", ["G63", "G127"])
def test_syndrome_padding_bits_are_ignored(dev, name, schedule):
    l, a, b = workloads.code(name)
    g = sagms.Graph.gb(l, a, b)
    assert g.m % 64, "the code must leave padding bits in its last syndrome word"
    nf, p = 1024, 0.05
    buf = sagms.frame_buffers(g, nf, device=dev)
    sagms.gen_errors(g, 9, 0, 0, nf, p, buf["ex"], buf["ez"], buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    dirty = buf["synd"].clone()
    pad = np.array([~np.uint64((1 << (g.m % 64)) - 1)], dtype=np.uint64).view(np.int64)[0]
    dirty[:, -1] |= int(pad)
    cfg = sagms.decoder_config("sagms", lmax=100, schedule=schedule)
    clean_out = sagms.frame_buffers(g, nf, device=dev)
    dirty_out = sagms.frame_buffers(g, nf, device=dev)
    sagms.decode(g, buf["synd"], llr, cfg, clean_out["ehat"], clean_out["iters"], clean_out["converged"])
    sagms.decode(g, dirty, llr, cfg, dirty_out["ehat"], dirty_out["iters"], dirty_out["converged"])
    torch.cuda.synchronize()
    for k in ("ehat", "iters", "converged"):
        assert torch.equal(clean_out[k], dirty_out[k]), k
    s = channel.unpack(u64(buf["synd"]), g.m)
    r = oracle_decode(name, s, np.full(g.n, sagms.prior_llr(p), np.float32), "sagms", 100, schedule)
    assert (u64(dirty_out["ehat"]) == channel.pack(r.ehat)).all()
    assert (dirty_out["iters"].cpu().numpy() == r.iters).all()

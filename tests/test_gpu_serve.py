"""The serving runtime on the GPU (through the C ABI).

Each served request's outputs must equal, bit for bit, the same syndromes
decoded alone by sagms_decode (one call for that request only), for traces
that keep several launches in flight, mix five codes of three register
classes and exercise the frame budget, deadlines and manual progress; and
sampled served frames of every code equal the CPU oracle's decode of the
same syndromes (FP32 and FP16 messages).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel  # noqa: E402
from oracle import codes as ocodes  # noqa: E402
from oracle import decoders  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*args):
    print(*args, flush=True)


@pytest.fixture(scope="module")
def codes(dev):
    graphs = [sagms.Graph.gb(*workloads.code(n)) for n in workloads.SERVE_CODES]
    priors = [np.full(g.n, sagms.prior_llr(workloads.SERVE_P), dtype=np.float32) for g in graphs]
    return graphs, priors


def pool(g, nframes, stream_id, dev, frame0=0):
    buf = sagms.frame_buffers(g, nframes, device=dev, with_ez=False)
    sagms.gen_errors(g, workloads.SERVE_SEED, stream_id, frame0, nframes, workloads.SERVE_P, buf["ex"], None,
                     buf["synd"])
    torch.cuda.synchronize()
    return buf["synd"].cpu().numpy().view(np.uint64).copy()


def decode_alone(g, synd, cfg, dev):
    nf = synd.shape[0]
    s = torch.from_numpy(synd.view(np.int64)).to(dev)
    out = sagms.frame_buffers(g, nf, device=dev)
    llr = torch.full((g.n,), sagms.prior_llr(workloads.SERVE_P), dtype=torch.float32, device=dev)
    sagms.decode(g, s, llr, cfg, out["ehat"], out["iters"], out["converged"])
    torch.cuda.synchronize()
    return out["ehat"].cpu().numpy().view(np.uint64), out["iters"].cpu().numpy(), out["converged"].cpu().numpy()


def build_trace(graphs, code, size, dev, stream_base=0):
    """Per-request host buffers, carved from one syndrome pool per code."""
    reqs = np.zeros(len(code), dtype=sagms.REQUEST_DTYPE)
    pools, outs, slices = [], [], []
    for c, g in enumerate(graphs):
        total = int(size[code == c].sum())
        pools.append(pool(g, max(total, 1), workloads.serve_stream(c) + stream_base, dev))
        outs.append(dict(ehat=np.full((max(total, 1), g.words_n), 0xFFFFFFFFFFFFFFFF, dtype=np.uint64),
                         iters=np.full(max(total, 1), -1, dtype=np.int32),
                         conv=np.full(max(total, 1), 7, dtype=np.uint8)))
    used = [0] * len(graphs)
    for i, (c, nf) in enumerate(zip(code, size)):
        c, nf = int(c), int(nf)
        lo = used[c]
        used[c] += nf
        o = outs[c]
        reqs[i] = (c, nf, pools[c][lo].ctypes.data, o["ehat"][lo].ctypes.data, o["iters"][lo:].ctypes.data,
                   o["conv"][lo:].ctypes.data, 0.0)
        slices.append((c, lo, nf))
    for c in range(len(graphs)):   # frames no request uses (a code drawn by none) are dropped
        pools[c] = pools[c][:used[c]]
        outs[c] = {k: v[:used[c]] for k, v in outs[c].items()}
    return reqs, pools, outs, slices


def check_alone(graphs, cfg, dev, pools, outs, slices, picks):
    for i in picks:
        c, lo, nf = slices[i]
        e, it, cv = decode_alone(graphs[c], pools[c][lo:lo + nf], cfg, dev)
        assert (outs[c]["ehat"][lo:lo + nf] == e).all(), ("ehat", i, c)
        assert (outs[c]["iters"][lo:lo + nf] == it).all(), ("iters", i, c)
        assert (outs[c]["conv"][lo:lo + nf] == cv).all(), ("converged", i, c)


def check_oracle(graphs, precision, pools, outs, per_code=48):
    """Sampled served frames of every code against the oracle's decode of the
    same syndromes in the matching message format."""
    for c, name in enumerate(workloads.SERVE_CODES):
        nf = len(pools[c])
        if nf == 0:
            continue
        idx = np.unique(np.linspace(0, nf - 1, min(per_code, nf)).astype(int))
        l, a, b = workloads.code(name)
        hz = ocodes.gb_matrices(l, a, b)[1]
        tg = decoders.TannerGraph(hz, ocodes.gb_var_checks(l, a, b))
        s = channel.unpack(pools[c][idx], tg.m)
        r = decoders.decode(tg, s, np.full(tg.n, sagms.prior_llr(workloads.SERVE_P), np.float32),
                            decoders.DecoderParams(kind="sagms", lmax=workloads.SERVE_LMAX,
                                                   **workloads.SAGMS_PARAMS), precision)
        assert (outs[c]["ehat"][idx] == channel.pack(r.ehat)).all(), (name, "ehat")
        assert (outs[c]["iters"][idx] == r.iters).all(), (name, "iters")
        assert (outs[c]["conv"][idx] == r.converged).all(), (name, "converged")
        say("served frames of", name, "against the oracle:", len(idx), "equal")


def check_pools(graphs, cfg, dev, pools, outs):
    """All served frames of a code against one sagms_decode over its pool."""
    for c, g in enumerate(graphs):
        if len(pools[c]) == 0:
            continue
        e, it, cv = decode_alone(g, pools[c], cfg, dev)
        assert (outs[c]["ehat"] == e).all() and (outs[c]["iters"] == it).all() and (outs[c]["conv"] == cv).all(), c


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_served_results_equal_alone(dev, codes, precision):
    graphs, priors = codes
    cfg = sagms.decoder_config("sagms", lmax=workloads.SERVE_LMAX, precision=precision)
    srv = sagms.Server(graphs, priors, cfg, sagms.server_config(max_frames_in_flight=4096, max_frames_per_launch=1024,
                                                                 streams=4))
    code, size, t = workloads.serve_trace(2e5, 600)          # 600 requests over ~3 ms (~6.5 M frames/s offered)
    reqs, pools, outs, slices = build_trace(graphs, code, size, dev)
    say("replay", precision, len(reqs), int(size.sum()))
    done = srv.replay(reqs, t)
    assert (done["status"] == sagms.REQ_DONE).all()
    assert (done["id"] == np.arange(len(reqs))).all()
    assert (done["done_us"] >= done["admit_us"]).all() and (done["admit_us"] >= done["submit_us"]).all()
    check_pools(graphs, cfg, dev, pools, outs)
    check_oracle(graphs, precision, pools, outs)
    rng = np.random.default_rng(1)
    check_alone(graphs, cfg, dev, pools, outs, slices, rng.choice(len(reqs), 25, replace=False))
    assert srv.pending() == (0, 0, 0)
    srv.close()


def test_burst_with_budget_and_manual_progress(dev, codes):
    """A burst larger than the frame budget: at most max_frames_in_flight
    frames are ever in flight, every request completes, results equal alone."""
    graphs, priors = codes
    cfg = sagms.decoder_config("sagms", lmax=workloads.SERVE_LMAX)
    srv = sagms.Server(graphs, priors, cfg, sagms.server_config(max_frames_in_flight=200, max_frames_per_launch=128,
                                                                 streams=3, tile_frames=3, waves_per_block=2))
    code, size, _ = workloads.serve_trace(1e6, 120, seed=7)
    reqs, pools, outs, slices = build_trace(graphs, code, size, dev, stream_base=20)
    ids = []
    for i, c in enumerate(code):
        clo, lo, nf = slices[i]
        o = outs[clo]
        ids.append(srv.submit(int(c), pools[clo][lo:lo + nf], o["ehat"][lo:lo + nf], o["iters"][lo:lo + nf],
                              o["conv"][lo:lo + nf]))
    assert ids == list(range(ids[0], ids[0] + len(ids)))
    seen, peak = [], 0
    for _ in range(2_000_000):
        got = srv.progress()
        seen.extend(got["id"].tolist())
        q, f, _c = srv.pending()
        peak = max(peak, f)
        if len(seen) == len(ids):
            break
    assert sorted(seen) == ids
    assert 0 < peak <= 200
    check_pools(graphs, cfg, dev, pools, outs)
    with pytest.raises(sagms.SagmsError):                     # larger than one launch
        big = np.zeros((129, graphs[0].words_m), dtype=np.uint64)
        srv.submit(0, big, np.zeros((129, graphs[0].words_n), dtype=np.uint64), np.zeros(129, dtype=np.int32),
                   np.zeros(129, dtype=np.uint8))
    srv.close()


def test_deadlines_cancel_waiting_requests(dev, codes):
    graphs, priors = codes
    cfg = sagms.decoder_config("sagms", lmax=workloads.SERVE_LMAX)
    srv = sagms.Server(graphs, priors, cfg, sagms.server_config(max_frames_in_flight=64, max_frames_per_launch=64,
                                                                 streams=1))
    g = graphs[0]
    synd = pool(g, 40 * 16, workloads.serve_stream(0) + 40, dev).reshape(40, 16, g.words_m)
    ehat = np.zeros((40, 16, g.words_n), dtype=np.uint64)
    iters = np.full((40, 16), -1, dtype=np.int32)
    conv = np.full((40, 16), 7, dtype=np.uint8)
    ids = []
    for i in range(40):
        # odd requests must be admitted within 1 ns of submission: they never are
        ids.append(srv.submit(0, synd[i], ehat[i], iters[i], conv[i], deadline_us=1e-3 if i % 2 else 0.0))
    status = {}
    for _ in range(2_000_000):
        for row in srv.progress():
            status[int(row["id"])] = int(row["status"])
        if len(status) == 40:
            break
    assert len(status) == 40
    for i, rid in enumerate(ids):
        if i % 2:
            assert status[rid] == sagms.REQ_CANCELLED
            assert (iters[i] == -1).all() and (conv[i] == 7).all()   # untouched
        else:
            assert status[rid] == sagms.REQ_DONE
            e, it, cv = decode_alone(g, synd[i], cfg, dev)
            assert (ehat[i] == e).all() and (iters[i] == it).all() and (conv[i] == cv).all()
    srv.close()


def test_replay_needs_an_idle_server_and_valid_trace(dev, codes):
    graphs, priors = codes
    cfg = sagms.decoder_config("sagms", lmax=20)
    srv = sagms.Server(graphs[:1], priors[:1], cfg, sagms.server_config(max_frames_per_launch=64))
    g = graphs[0]
    synd = pool(g, 8, 300, dev)
    ehat = np.zeros((8, g.words_n), dtype=np.uint64)
    it = np.zeros(8, dtype=np.int32)
    cv = np.zeros(8, dtype=np.uint8)
    reqs = np.zeros(2, dtype=sagms.REQUEST_DTYPE)
    for i in range(2):
        reqs[i] = (0, 4, synd[4 * i].ctypes.data, ehat[4 * i].ctypes.data, it[4 * i:].ctypes.data,
                   cv[4 * i:].ctypes.data, 0.0)
    with pytest.raises(sagms.SagmsError):
        srv.replay(reqs, np.array([5.0, 1.0]))                 # decreasing arrivals
    bad = reqs.copy()
    bad[1]["code"] = 3
    with pytest.raises(sagms.SagmsError):
        srv.replay(bad, np.array([0.0, 1.0]))                  # unknown code
    srv.submit(0, synd[:4], ehat[:4], it[:4], cv[:4])
    with pytest.raises(sagms.SagmsError):
        srv.replay(reqs, np.array([0.0, 1.0]))                 # a request is still queued
    for _ in range(1_000_000):
        if len(srv.progress()) == 1:
            break
    done = srv.replay(reqs, np.array([0.0, 1.0]))
    assert (done["status"] == 0).all()
    e, i2, c2 = decode_alone(g, synd, cfg, dev)
    assert (ehat == e).all() and (it == i2).all() and (cv == c2).all()
    srv.close()

"""Host-side checks of libsagms (no GPU needed).

The library loads and exports every function include/sagms.h declares; the
host graph builder agrees with the oracle (matrices, k, logical basis); the
argument checks of the device entry points reject bad input before any
device work.
"""
import ctypes

import numpy as np
import pytest

import paper_2605_10433_amd as sagms
import workloads
from oracle import channel, codes, gf2


def test_exports_every_declared_symbol():
    names = sagms.header_functions()
    assert len(names) >= 12
    L = sagms.lib()
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("name", ["G63", "G127", "G255w3", "G255w4", "G511w5"])
def test_gb_graph_matches_oracle(name):
    l, a, b = workloads.code(name)
    g = sagms.Graph.gb(l, a, b)
    hx, hz = codes.gb_matrices(l, a, b)
    k = codes.dimension(hx, hz)
    assert (g.m, g.n, g.n_edges) == (l, 2 * l, int(hz.sum()))
    assert (g.dc_max, g.dv_max) == (int(hz.sum(1).max()), int(hz.sum(0).max()))
    assert g.k == k == workloads.CODES[name]["k"]
    assert (g.words_n, g.words_m) == ((2 * l + 63) // 64, (l + 63) // 64)
    assert (channel.unpack(g.rows(), g.n) == hz).all()
    lz = channel.unpack(g.logicals(), g.n)
    assert lz.shape == (k, g.n)
    assert not gf2.matvec(hx, lz).any()                              # in ker H_X
    assert gf2.rank(np.vstack([hz, lz])) == gf2.rank(hz) + k         # independent mod rowspace H_Z


@pytest.mark.parametrize("code", [dict(l=7, a=(0, 1), b=(0, 2)), dict(l=7, a=(0, 1, 3), b=(0, 2, 6))])
def test_small_gb_codes(code):
    g = sagms.Graph.gb(code["l"], code["a"], code["b"])
    hx, hz = codes.gb_matrices(**code)
    assert g.k == codes.dimension(hx, hz)
    assert (channel.unpack(g.rows(), g.n) == hz).all()


JOINT_CODES = [("L7", (7, [0, 1], [0, 2])), ("L7b", (7, [0, 1, 3], [0, 2, 6])), ("G63", None), ("G127", None)]


@pytest.mark.parametrize("name,spec", JOINT_CODES)
def test_joint_graph_matches_oracle(name, spec):
    """The joint graph against the oracle's quaternary matrix of the same GB
    code (X-type rows of H_X, then Z-type rows of H_Z): sizes, degrees, the
    rows as (x | z) halves, and 2k logical rows (u | v) that commute with
    every row and are independent modulo the stabilizer group."""
    from oracle import joint
    l, a, b = spec if spec else workloads.code(name)
    g = sagms.Graph.gb_joint(l, a, b)
    sx, sz, _ = joint.gb_joint(l, a, b)
    n = 2 * l
    assert (g.m, g.n, g.n_edges, g.joint) == (2 * l, n, int((sx | sz).sum()), 1)
    assert (g.dc_max, g.dv_max) == (len(a) + len(b), len(a) + len(b))
    assert (g.words_n, g.words_m, g.words_e) == ((n + 63) // 64, (2 * l + 63) // 64, 2 * ((n + 63) // 64))
    rows = g.rows()
    wn = g.words_n
    assert (channel.unpack(rows[:, :wn], n) == sz).all() and (channel.unpack(rows[:, wn:], n) == sx).all()
    hx, hz = codes.gb_matrices(l, a, b)
    k = codes.dimension(hx, hz)
    assert g.k == k
    lg = g.logicals()
    assert lg.shape == (2 * k, 2 * wn)
    u = channel.unpack(lg[:, :wn], n).astype(np.int64)
    v = channel.unpack(lg[:, wn:], n).astype(np.int64)
    # row (u | v) flags r when u.r_x + v.r_z is odd: the logical operator is
    # L = (x part v, z part u); it commutes with every row: S_x.L_z + S_z.L_x = 0
    assert not ((sx.astype(np.int64) @ u.T + sz.astype(np.int64) @ v.T) & 1).any()
    stab = np.hstack([sx, sz])
    ops = np.hstack([v, u]).astype(np.uint8)
    assert gf2.rank(np.vstack([stab, ops])) == gf2.rank(stab) + 2 * k
    assert not u[k:].any() and not v[:k].any()       # Z-type logicals first, then X-type


def test_joint_graph_argument_checks():
    L = sagms.lib()
    g = sagms.Graph.gb_joint(*workloads.code("G63"))
    fake = ctypes.c_void_p(0x1000)
    for kind, prec, sched in (("bp", "fp32", "flooding"), ("sagms", "fp16", "flooding"),
                              ("sagms", "fp32", "layered"), ("ms", "int6", "flooding")):
        cfg = sagms.decoder_config(kind, precision=prec, schedule=sched)
        assert L.sagms_decode(g._h, fake, fake, ctypes.byref(cfg), 4, fake, fake, fake, None) == sagms.EUNSUPPORTED
    # the binary judge refuses a joint graph, the joint judge a binary one
    assert L.sagms_judge(g._h, fake, fake, fake, fake, 4, None, fake, None) == sagms.EINVAL
    gb = sagms.Graph.gb(*workloads.code("G63"))
    assert L.sagms_judge_joint(gb._h, fake, fake, fake, fake, fake, 4, None, fake, None) == sagms.EINVAL
    # the joint sampler needs the Z plane
    assert L.sagms_gen_errors(g._h, 1, 0, 0, 4, 0.05, fake, None, fake, None) == sagms.EINVAL
    # batches and servers refuse joint graphs
    seg = (sagms.Segment * 1)()
    seg[0].graph, seg[0].nframes = g._h.value, 4
    seg[0].synd = seg[0].llr0 = seg[0].ehat = seg[0].iters = seg[0].converged = 0x1000
    out = ctypes.c_void_p()
    cfg = sagms.decoder_config("sagms")
    assert L.sagms_batch_create(ctypes.cast(seg, ctypes.c_void_p), 1, ctypes.byref(cfg),
                                ctypes.byref(out)) == sagms.EUNSUPPORTED


def test_build_graph_from_dense_matches_gb():
    hx, hz = codes.gb_matrices(**codes.G63)
    g = sagms.Graph.from_dense(hz, hx)
    assert g.k == 28 and (channel.unpack(g.rows(), 126) == hz).all()
    g2 = sagms.Graph.from_dense(hz)
    assert g2.k == -1
    with pytest.raises(sagms.SagmsError):
        g2.logicals()


def _csr_call(m, n, rp, ci, mo=0, rpo=None, cio=None):
    rp = np.asarray(rp, dtype=np.int32)
    ci = np.asarray(ci, dtype=np.int32)
    args = [m, n, rp.ctypes.data, ci.ctypes.data, mo]
    if mo:
        rpo = np.asarray(rpo, dtype=np.int32)
        cio = np.asarray(cio, dtype=np.int32)
        args += [rpo.ctypes.data, cio.ctypes.data]
    else:
        args += [None, None]
    h = ctypes.c_void_p()
    rc = sagms.lib().sagms_build_graph(*args, ctypes.byref(h))
    if rc == 0:
        sagms.lib().sagms_destroy_graph(h)
    return rc


def test_build_graph_rejects_bad_input():
    assert _csr_call(2, 4, [0, 2, 4], [0, 1, 2, 3]) == sagms.OK
    assert _csr_call(2, 4, [0, 1, 3], [0, 1, 2]) == sagms.EINVAL          # check of degree 1
    assert _csr_call(2, 4, [0, 2, 4], [0, 4, 2, 3]) == sagms.EINVAL       # column out of range
    assert _csr_call(2, 4, [0, 2, 4], [1, 1, 2, 3]) == sagms.EINVAL       # repeated column
    assert _csr_call(2, 4, [1, 2, 4], [0, 1, 2, 3]) == sagms.EINVAL       # row_ptr[0] != 0
    assert _csr_call(0, 4, [0], []) == sagms.EINVAL
    assert _csr_call(1, 5000, [0, 2], [0, 1]) == sagms.EINVAL             # n too large
    # anticommuting partner matrix
    assert _csr_call(1, 4, [0, 2], [0, 1], 1, [0, 2], [1, 2]) == sagms.EINVAL
    assert _csr_call(1, 4, [0, 2], [0, 1], 1, [0, 2], [0, 1]) == sagms.OK
    with pytest.raises(sagms.SagmsError):
        sagms.Graph.gb(7, [0, 0], [1, 2])                                  # repeated exponent
    with pytest.raises(sagms.SagmsError):
        sagms.Graph.gb(7, [0, 9], [1, 2])                                  # exponent out of range


def _decode_rc(g, cfg):
    return sagms.lib().sagms_decode(g._h, None, None, ctypes.byref(cfg), 4, None, None, None, None)


def test_decoder_config_checks_before_device_work():
    g = sagms.Graph.gb(*workloads.code("G63"))
    D = sagms.decoder_config
    assert _decode_rc(g, D("sagms", alpha_max=0.6, eta=2.0)) == sagms.EINVAL      # alpha_max * eta > 1
    assert _decode_rc(g, D("sagms", alpha_min=0.0)) == sagms.EINVAL
    assert _decode_rc(g, D("sagms", eta=0.9)) == sagms.EINVAL
    assert _decode_rc(g, D("sms", alpha=1.5)) == sagms.EINVAL
    assert _decode_rc(g, D("ms", lmax=0)) == sagms.EINVAL
    bad = D("ms")
    bad.kind = 7
    assert _decode_rc(g, bad) == sagms.EINVAL
    sched = D("ms")
    sched.schedule = 2
    assert _decode_rc(g, sched) == sagms.EINVAL
    # the layered schedule runs the min-sum family with FP32 messages only
    assert _decode_rc(g, D("bp", schedule="layered")) == sagms.EUNSUPPORTED
    assert _decode_rc(g, D("sagms", schedule="layered", precision="fp16")) == sagms.EUNSUPPORTED
    assert _decode_rc(g, D("ms", schedule="layered", precision="int6")) == sagms.EUNSUPPORTED
    prec = D("ms")
    prec.msg_precision = 3
    assert _decode_rc(g, prec) == sagms.EUNSUPPORTED
    assert _decode_rc(g, D("bp", precision="fp16")) == sagms.EUNSUPPORTED
    assert _decode_rc(g, D("ms", frames_per_wave=-1)) == sagms.EINVAL
    assert _decode_rc(g, D("ms", frames_per_wave=2000)) == sagms.EINVAL
    res = D("ms")
    res.reserved = 1
    assert _decode_rc(g, res) == sagms.EINVAL
    # a valid configuration with zero frames is a no-op that touches no device
    ok = D("sagms")
    assert sagms.lib().sagms_decode(g._h, None, None, ctypes.byref(ok), 0, None, None, None, None) == sagms.OK
    assert "exceeds" in (_decode_rc(g, D("sagms", alpha_max=0.6, eta=2.0)) and
                         sagms.lib().sagms_last_error().decode())


def test_gen_errors_and_judge_argument_checks():
    L = sagms.lib()
    g = sagms.Graph.gb(*workloads.code("G63"))
    assert L.sagms_gen_errors(g._h, 1, 0, 0, 4, 1.0, None, None, None, None) == sagms.EINVAL
    assert L.sagms_gen_errors(g._h, 1, 0, 0, -1, 0.1, None, None, None, None) == sagms.EINVAL
    assert L.sagms_gen_errors(g._h, 1, 0, 0, 0, 0.1, None, None, None, None) == sagms.OK
    assert L.sagms_gen_errors(g._h, 1, 0, 0, 4, 0.1, None, None, None, None) == sagms.EINVAL  # null buffers
    assert L.sagms_gen_errors(None, 1, 0, 0, 4, 0.1, None, None, None, None) == sagms.EINVAL
    g2 = sagms.Graph.from_dense(codes.gb_matrices(**codes.G63)[1])
    assert L.sagms_judge(g2._h, None, None, None, None, 4, None, None, None) == sagms.EINVAL   # no H_other


def test_more_frames_than_one_call_allows_are_refused_on_the_host():
    """Every device call refuses more than 2^31 - 1 frames (which keeps every
    grid within 2^31 - 1 blocks) with SAGMS_EINVAL, checked before anything
    touches a device: here on a host without one, with buffer pointers that
    are never dereferenced (a decode of 2^50 frames, every launch shape; the
    sampler; the judge; a mixed-batch segment)."""
    L = sagms.lib()
    g = sagms.Graph.gb(*workloads.code("G63"))
    fake = ctypes.c_void_p(0x1000)
    for huge in (1 << 31, 1 << 50):
        assert L.sagms_gen_errors(g._h, 1, 0, 0, huge, 0.05, fake, fake, fake, None) == sagms.EINVAL
        assert "too many frames" in L.sagms_last_error().decode()
        for fpw in (0, 1, 1024):
            cfg = sagms.decoder_config("sagms", frames_per_wave=fpw)
            assert L.sagms_decode(g._h, fake, fake, ctypes.byref(cfg), huge, fake, fake, fake, None) == sagms.EINVAL
            assert "too many frames" in L.sagms_last_error().decode()
        assert L.sagms_judge(g._h, fake, fake, fake, fake, huge, fake, fake, None) == sagms.EINVAL
        assert "too many frames" in L.sagms_last_error().decode()
        seg = (sagms.Segment * 1)()
        seg[0].graph, seg[0].nframes = g._h.value, huge
        seg[0].synd = seg[0].llr0 = seg[0].ehat = seg[0].iters = seg[0].converged = 0x1000
        out = ctypes.c_void_p()
        cfg = sagms.decoder_config("sagms")
        assert L.sagms_batch_create(ctypes.cast(seg, ctypes.c_void_p), 1, ctypes.byref(cfg),
                                    ctypes.byref(out)) == sagms.EINVAL
        assert L.sagms_decode_segments(ctypes.cast(seg, ctypes.c_void_p), 1, ctypes.byref(cfg), None,
                                       None) == sagms.EINVAL


@pytest.mark.parametrize("p", workloads.P_GRID + [0.001, 0.3])
def test_prior_llr_matches_oracle(p):
    assert sagms.prior_llr(p) == np.float32(channel.prior_llr(p))
    assert np.isnan(sagms.prior_llr(0.0)) and np.isnan(sagms.prior_llr(0.8))


def _segments(graphs, nframes, null_buffers=False):
    arr = (sagms.Segment * len(graphs))()
    for i, (g, nf) in enumerate(zip(graphs, nframes)):
        arr[i].graph = g._h.value if g is not None else None
        arr[i].nframes = nf
        if not null_buffers:  # host addresses: the checks read no memory
            for f in ("synd", "llr0", "ehat", "iters", "converged"):
                setattr(arr[i], f, 0x1000)
    return arr


def _create_rc(arr, n, cfg):
    h = ctypes.c_void_p()
    return sagms.lib().sagms_batch_create(ctypes.cast(arr, ctypes.c_void_p) if arr is not None else None, n,
                                          ctypes.byref(cfg), ctypes.byref(h))


def test_batch_create_checks_before_device_work():
    g = sagms.Graph.gb(*workloads.code("G63"))
    cfg = sagms.decoder_config("sagms")
    assert _create_rc(None, 1, cfg) == sagms.EINVAL
    assert _create_rc(_segments([g], [4]), 0, cfg) == sagms.EINVAL
    assert _create_rc(_segments([g] * 17, [4] * 17), 17, cfg) == sagms.EINVAL          # more than 16 segments
    assert _create_rc(_segments([g, None], [4, 4]), 2, cfg) == sagms.EINVAL            # null graph
    assert _create_rc(_segments([g], [-1]), 1, cfg) == sagms.EINVAL                    # negative frame count
    assert _create_rc(_segments([g], [4], null_buffers=True), 1, cfg) == sagms.EINVAL  # null buffers
    assert _create_rc(_segments([g], [4]), 1, sagms.decoder_config("bp")) == sagms.EUNSUPPORTED
    assert _create_rc(_segments([g], [4]), 1, sagms.decoder_config("sagms", schedule="layered")) == sagms.EUNSUPPORTED
    assert _create_rc(_segments([g], [4]), 1, sagms.decoder_config("sagms", eta=0.5)) == sagms.EINVAL
    for name in ("sagms_batch_run", "sagms_batch_instantiate", "sagms_batch_destroy"):
        assert getattr(sagms.lib(), name)(None, *([None] if name == "sagms_batch_run" else [])) == sagms.EINVAL
    assert sagms.lib().sagms_batch_set_plan(None, ctypes.byref(sagms.plan())) == sagms.EINVAL
    assert sagms.lib().sagms_batch_tune(None, None, 1, None, 0, None, None) == sagms.EINVAL


def test_plan_structures():
    p = sagms.plan("tiered", tile_frames=16, waves_per_block=2, blocks_per_cu=3, reg_budget=1, unroll=2)
    assert p.as_dict() == dict(kind="tiered", tile_frames=16, waves_per_block=2, blocks_per_cu=3, reg_budget=1,
                               unroll=2)
    assert sagms.plan().unroll == 1
    assert ctypes.sizeof(sagms.Plan) == 24 and ctypes.sizeof(sagms.Segment) == 64
    with pytest.raises(ValueError):
        sagms.plan("bogus")


def test_server_create_and_calls_check_before_device_work():
    L = sagms.lib()
    g = sagms.Graph.gb(*workloads.code("G63"))
    prior = np.full(g.n, 3.0, dtype=np.float32)
    gh = (ctypes.c_void_p * 1)(g._h.value)
    ph = (ctypes.c_void_p * 1)(prior.ctypes.data)
    cfg = sagms.decoder_config("sagms")

    def rc(scfg, n=1, graphs=gh, priors=ph, c=cfg):
        h = ctypes.c_void_p()
        return L.sagms_server_create(ctypes.cast(graphs, ctypes.c_void_p) if graphs is not None else None,
                                     ctypes.cast(priors, ctypes.c_void_p) if priors is not None else None, n,
                                     ctypes.byref(c), ctypes.byref(scfg), ctypes.byref(h))

    S = sagms.server_config
    assert rc(S(), graphs=None) == sagms.EINVAL
    assert rc(S(), priors=None) == sagms.EINVAL
    assert rc(S(), n=0) == sagms.EINVAL
    assert rc(S(), n=17) == sagms.EINVAL
    assert rc(S(max_frames_per_launch=0)) == sagms.EINVAL
    assert rc(S(max_frames_per_launch=1 << 25)) == sagms.EINVAL
    assert rc(S(max_frames_in_flight=100, max_frames_per_launch=200)) == sagms.EINVAL
    assert rc(S(streams=0)) == sagms.EINVAL and rc(S(streams=9)) == sagms.EINVAL
    assert rc(S(tile_frames=0)) == sagms.EINVAL and rc(S(waves_per_block=3)) == sagms.EINVAL
    assert rc(S(reg_budget=2)) == sagms.EINVAL
    assert rc(S(min_launch_frames=-1)) == sagms.EINVAL
    assert rc(S(max_frames_per_launch=64, min_launch_frames=65, max_frames_in_flight=64)) == sagms.EINVAL
    assert rc(S(max_wait_us=-1.0)) == sagms.EINVAL
    assert rc(S(), c=sagms.decoder_config("bp")) == sagms.EUNSUPPORTED
    assert rc(S(), c=sagms.decoder_config("sagms", schedule="layered")) == sagms.EUNSUPPORTED
    assert rc(S(), graphs=(ctypes.c_void_p * 1)(None)) == sagms.EINVAL
    assert rc(S(), priors=(ctypes.c_void_p * 1)(None)) == sagms.EINVAL
    assert L.sagms_server_submit(None, None, None) == sagms.EINVAL
    assert L.sagms_server_progress(None, None, 0, None) == sagms.EINVAL
    assert L.sagms_server_pending(None, None, None, None) == sagms.EINVAL
    assert L.sagms_server_replay(None, None, None, 0, 1.0, None) == sagms.EINVAL
    assert L.sagms_server_destroy(None) == sagms.EINVAL


def test_serving_structures_and_trace():
    assert ctypes.sizeof(sagms.Request) == sagms.REQUEST_DTYPE.itemsize == 48
    assert ctypes.sizeof(sagms.Completion) == sagms.COMPLETION_DTYPE.itemsize == 40
    assert ctypes.sizeof(sagms.ServerConfig) == 40
    for name, _ in sagms.Request._fields_:
        assert sagms.REQUEST_DTYPE.fields[name][1] == getattr(sagms.Request, name).offset
    for name, _ in sagms.Completion._fields_:
        assert sagms.COMPLETION_DTYPE.fields[name][1] == getattr(sagms.Completion, name).offset
    code, size, t = workloads.serve_trace(1e6, 20000)
    assert (np.diff(t) >= 0).all() and size.min() >= 1 and size.max() <= 64
    assert set(np.unique(code)) == set(range(5))
    assert abs(np.mean(np.diff(t)) - 1.0) < 0.05                 # mean gap 1 us at 1e6 / s
    assert abs(size.mean() - 32.5) < 1.0


@pytest.mark.parametrize("dc", [2, 4, 6, 8, 10, 16])
def test_alpha_star_matches_oracle(dc):
    from oracle import analysis
    for l0 in (0.5, 1.0, 2.639, 3.36730, 3.597, 4.304, 8.0, 15.0):
        # the oracle's direct form loses digits as tanh(L0/2) -> 1 (about 1e-12 at L0 = 15)
        tol = 1e-12 if l0 < 8 else 1e-10
        assert sagms.alpha_star(l0, dc) == pytest.approx(analysis.alpha_star(l0, dc), rel=tol)
        if dc == 2:
            assert sagms.alpha_star(l0, dc) == pytest.approx(1.0, abs=4e-16)   # atanh(tanh(x)) = x
    # where the direct form overflows: the large-L0 form 1 - ln(d_c - 1) / L0 is exact to O(e^-L0)
    assert sagms.alpha_star(40.0, dc) == pytest.approx(analysis.alpha_star_approx(40.0, dc), rel=1e-13)
    assert np.isnan(sagms.alpha_star(0.0, dc)) and np.isnan(sagms.alpha_star(3.0, 1))


def test_derived_gains():
    from oracle import analysis
    l0 = channel.prior_llr(0.05)
    cfg = sagms.derived_config(l0, 10)
    a = analysis.alpha_star(l0, 10)
    assert cfg.kind == sagms.KINDS["sagms"]
    assert cfg.alpha_max == pytest.approx(a, rel=1e-12) and cfg.alpha_min == pytest.approx(0.6 * a, rel=1e-12)
    assert cfg.alpha_max * cfg.eta <= 1.0 and cfg.eta == pytest.approx(1.0 / a, rel=1e-12)
    cfg2 = sagms.derived_config(l0, 10, ratio=0.5, eta=1.1)
    assert cfg2.eta == 1.1 and cfg2.alpha_min == pytest.approx(0.5 * a, rel=1e-12)
    g = sagms.Graph.gb(*workloads.code("G63"))
    assert sagms.lib().sagms_decode(g._h, None, None, ctypes.byref(cfg), 0, None, None, None, None) == sagms.OK
    L = sagms.lib()
    for bad in ((0.0, 10, 0.6, 0.0), (3.0, 1, 0.6, 0.0), (3.0, 10, 0.0, 0.0), (3.0, 10, 1.5, 0.0),
                (3.0, 10, 0.6, 0.5), (15.0, 2, 0.6, 1.5)):
        assert L.sagms_derive_gains(*bad, ctypes.byref(sagms.decoder_config())) == sagms.EINVAL


def test_fer_ratio_interval_matches_oracle():
    from oracle import stats as ostats
    from paper_2605_10433_amd.stats import fer_ratio_interval
    for f1, n1, f2, n2 in ((500, 10 ** 6, 600, 10 ** 6), (37, 20000, 91, 50000), (1, 10, 9, 10)):
        got = fer_ratio_interval(f1, n1, f2, n2)
        ref = ostats.log_ratio_interval(f1, n1, f2, n2)
        assert got == pytest.approx(ref, rel=1e-12)
    with pytest.raises(ValueError):
        fer_ratio_interval(0, 10, 1, 10)


def test_codes_beyond_every_decode_shape_are_refused():
    """A graph no compiled decode shape fits (n > 1024, or a check degree
    above 16) builds, but decoding, batching and serving it are refused with
    SAGMS_EUNSUPPORTED before any device work."""
    big = sagms.Graph.gb(600, [0, 1, 5, 11, 40], [0, 2, 9, 30, 77])          # n = 1200
    dense = np.zeros((4, 40), dtype=np.uint8)
    dense[0, :20] = 1                                                     # a check of degree 20
    dense[1, 20:] = 1
    dense[2, ::2] = 1
    dense[3, 1::2] = 1
    wide = sagms.Graph.from_dense(dense)
    for g in (big, wide):
        assert sagms.lib().sagms_decode(g._h, None, None, ctypes.byref(sagms.decoder_config("ms")), 4,
                                        None, None, None, None) == sagms.EUNSUPPORTED
        assert "no decode kernel" in sagms.lib().sagms_last_error().decode()
        assert _create_rc(_segments([g], [4]), 1, sagms.decoder_config("sagms")) == sagms.EUNSUPPORTED
    assert (big.n, big.dc_max) == (1200, 10) and wide.dc_max == 20


def _packed_passes(h, group):
    """Passes of the layered schedule with `group` lanes: the checks of the
    first-fit layers in (layer, position) order, each in the earliest pass
    after every pass holding a check that shares a variable with it and with
    a free lane (so every variable meets its checks in layer order)."""
    from oracle import layered
    last = np.full(h.shape[1], -1)
    fill = []
    for layer in layered.greedy_layers(h):
        for c in layer:
            vs = np.nonzero(h[c])[0]
            p = int(last[vs].max()) + 1
            while p < len(fill) and fill[p] == group:
                p += 1
            if p == len(fill):
                fill.append(0)
            fill[p] += 1
            last[vs] = p
    return len(fill)


@pytest.mark.parametrize("name", ["G63", "G127", "G255w3", "G255w4", "G511w5"])
def test_layered_plan_packs_passes(name):
    """The layered plan's pass count is that of the packing for its group
    size, never more than one pass per layer slice would take, and the group
    holds the syndrome and estimate words; l = 511 (weight 5): 21 passes of
    32 lanes where one pass per layer takes 18 passes of 64 (672 against
    1152 lane slots per frame and round)."""
    from oracle import layered
    l, a, b = workloads.code(name)
    _, hz = codes.gb_matrices(l, a, b)
    g = sagms.Graph.gb(l, a, b)
    G, P = g.layered_group, g.layered_passes
    if name == "G63":
        # the compiled code: one lane per frame updates the 63 checks in turn
        assert (G, P) == (1, 63)
        return
    assert G in (8, 16, 32, 64) and G >= max(g.words_m, g.words_n)
    assert P == _packed_passes(hz, G)
    assert P <= sum(-(-len(layer) // G) for layer in layered.greedy_layers(hz))
    if name == "G511w5":
        assert (G, P) == (32, 21)


def test_layered_lane_kernel_only_for_its_matrix():
    """The one-lane layered kernel runs the l = 63 code's H_Z only: the same
    matrix given densely (rows in the same order) selects it, whatever the
    order of each row's entries; the rows in another order or one entry
    moved do not (the general kernel, groups of 8 or more lanes, or no
    layered plan at all)."""
    l, a, b = workloads.code("G63")
    _, hz = codes.gb_matrices(l, a, b)
    g = sagms.Graph.from_dense(hz)
    assert (g.layered_group, g.layered_passes) == (1, 63)
    rng = np.random.default_rng(3)
    perm = rng.permutation(hz.shape[0])
    g = sagms.Graph.from_dense(hz[perm])
    assert g.layered_group >= 8
    h = hz.copy()
    row = h[5]
    on, off = np.nonzero(row)[0][0], np.nonzero(row == 0)[0][0]
    row[on], row[off] = 0, 1
    g = sagms.Graph.from_dense(h)
    assert g.layered_group != 1

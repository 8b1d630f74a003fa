"""Oracle side of the pooled parity tests, run in a pool of host processes:
each call takes one chunk of frames of one (code, seed, stream, p) point,
samples it, computes its syndromes, decodes it and judges it, all with
`oracle/`.  Nothing here touches the GPU.
"""
from __future__ import annotations

import numpy as np

_GRAPHS = {}


def _graph(name="G63"):
    if name not in _GRAPHS:
        import workloads
        from oracle import codes, decoders
        l, a, b = workloads.code(name)
        hx, hz = codes.gb_matrices(l, a, b)
        _GRAPHS[name] = dict(n=2 * l, hz=hz, tanner=decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b)),
                             lz=codes.logical_basis(hz, hx))
    return _GRAPHS[name]


def decode_chunk(task):
    """task = (kind, kw, p, frame0, nframes, lmax, arith[, schedule]): a chunk
    of the l = 63 sweep (seed 1, stream = index of p in the sweep grid).  The
    prior is the FP32 value of L0(p) except in the "fp64" mode (FP64 value).
    schedule: "flooding" (default) or "layered"."""
    import workloads
    kind, kw, p, frame0, nf, lmax, arith = task[:7]
    schedule = task[7] if len(task) > 7 else "flooding"
    return decode_point(dict(code="G63", seed=workloads.SWEEP_SEED, stream=None, kind=kind, kw=kw, p=p,
                             frame0=frame0, nframes=nf, lmax=lmax, arith=arith, schedule=schedule))


def decode_point(t):
    """t: dict with code, seed, stream (None: the sweep's stream of p), kind,
    kw, p, frame0, nframes, lmax, arith, schedule.  The prior is the FP32
    value of L0(p), promoted to double in the "fp64" mode only when
    t["prior32"] is true (else the FP64 value)."""
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import channel, decoders, judge, layered
    g = _graph(t["code"])
    p, frame0, nf, arith = t["p"], t["frame0"], t["nframes"], t["arith"]
    stream = workloads.stream_of(p) if t.get("stream") is None else t["stream"]
    with threadpool_limits(1):
        ex, _ = channel.sample_paulis(t["seed"], stream, frame0, nf, g["n"], p)
        s = channel.syndrome(g["hz"], ex)
        l0 = channel.prior_llr(p)
        if arith == "fp64" and t.get("prior32"):
            l0 = float(np.float32(l0))
        llr = np.full(g["n"], l0, dtype=np.float64 if arith == "fp64" else np.float32)
        prm = decoders.DecoderParams(kind=t["kind"], lmax=t["lmax"], **t["kw"])
        if t.get("schedule", "flooding") == "layered":
            r = layered.decode_layered(g["tanner"], s, llr, prm, arith)
        else:
            r = decoders.decode(g["tanner"], s, llr, prm, arith)
        fail = judge.judge_logical(g["lz"], ex, r.ehat, r.converged)
    out = dict(frame0=frame0, synd=channel.pack(s), ehat=channel.pack(r.ehat), iters=np.asarray(r.iters),
               converged=np.asarray(r.converged, dtype=bool), fail=np.asarray(fail, dtype=bool))
    if arith != "fp64":
        out["posterior"] = np.asarray(r.posterior, dtype=np.float32)
    return out

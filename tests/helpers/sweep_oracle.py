"""Oracle side of the sweep-wide parity test, run in a pool of host
processes: each call takes one chunk of frames of one sweep point, samples
it, computes its syndromes, decodes it and judges it, all with `oracle/`.
Nothing here touches the GPU.
"""
from __future__ import annotations

import numpy as np

_G63 = {}


def _graph():
    if not _G63:
        import workloads
        from oracle import codes, decoders
        l, a, b = workloads.code("G63")
        hx, hz = codes.gb_matrices(l, a, b)
        _G63.update(n=2 * l, hz=hz, tanner=decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b)),
                    lz=codes.logical_basis(hz, hx))
    return _G63


def decode_chunk(task):
    """task = (kind, kw, p, frame0, nframes, lmax, arith[, schedule]).  Frames
    of seed 1, stream = index of p in the sweep grid.  The prior is the FP32
    value of L0(p) except in the "fp64" mode (FP64 value).  schedule:
    "flooding" (default) or "layered"."""
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import channel, decoders, judge, layered
    kind, kw, p, frame0, nf, lmax, arith = task[:7]
    schedule = task[7] if len(task) > 7 else "flooding"
    g = _graph()
    with threadpool_limits(1):
        ex, _ = channel.sample_paulis(workloads.SWEEP_SEED, workloads.stream_of(p), frame0, nf, g["n"], p)
        s = channel.syndrome(g["hz"], ex)
        l0 = channel.prior_llr(p)
        llr = np.full(g["n"], l0, dtype=np.float64 if arith == "fp64" else np.float32)
        prm = decoders.DecoderParams(kind=kind, lmax=lmax, **kw)
        if schedule == "layered":
            r = layered.decode_layered(g["tanner"], s, llr, prm, arith)
        else:
            r = decoders.decode(g["tanner"], s, llr, prm, arith)
        fail = judge.judge_logical(g["lz"], ex, r.ehat, r.converged)
    out = dict(frame0=frame0, synd=channel.pack(s), ehat=channel.pack(r.ehat), iters=np.asarray(r.iters),
               converged=np.asarray(r.converged, dtype=bool), fail=np.asarray(fail, dtype=bool))
    if arith != "fp64":
        out["posterior"] = np.asarray(r.posterior, dtype=np.float32)
    return out

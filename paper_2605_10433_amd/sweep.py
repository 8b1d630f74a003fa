"""Frame-error-rate sweep on one GPU.

    python -m paper_2605_10433_amd.sweep [--frames 1048576] [--code G63]
        [--p 0.02,0.03,...] [--decoders ms,sms0.5,...,sagms,bp] [--lmax 100]

For every noise level p and decoder: 2^20 (by default) Philox frames of the
depolarizing channel (seed 1, stream = index of p in the grid, the same
frames for every decoder), syndromes, decoding and the logical judge, all
through libsagms.  Prints one JSON line per point (FER with its 95 % Wilson
interval, mean and 99th-percentile round count, decode and end-to-end
frames/s) and a markdown table at the end.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2605_10433_amd as sagms  # noqa: E402
from paper_2605_10433_amd.stats import wilson  # noqa: E402

DECODERS = {
    "ms": dict(kind="ms"),
    "sms0.5": dict(kind="sms", alpha=0.5),
    "sms0.625": dict(kind="sms", alpha=0.625),
    "sms0.75": dict(kind="sms", alpha=0.75),
    "sms0.875": dict(kind="sms", alpha=0.875),
    "sagms": dict(kind="sagms", alpha_min=0.30, alpha_max=0.50, eta=1.10),
    "bp": dict(kind="bp"),
}


def run_point(g, code, p, stream_id, name, nframes, lmax, seed=1):
    import torch
    buf = sagms.frame_buffers(g, nframes)
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device="cuda")
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    cfg = sagms.decoder_config(lmax=lmax, **DECODERS[name])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    st = torch.cuda.current_stream()
    ev[0].record(st)
    sagms.gen_errors(g, seed, stream_id, 0, nframes, p, buf["ex"], buf["ez"], buf["synd"])
    ev[1].record(st)
    sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    ev[2].record(st)
    sagms.judge(g, buf["ex"], buf["ehat"], buf["converged"], buf["iters"], counters)
    ev[3].record(st)
    torch.cuda.synchronize()
    fails, isum = (int(x) for x in counters.cpu().numpy())
    it = buf["iters"].float()
    lo, hi = wilson(fails, nframes)
    dec_ms = ev[1].elapsed_time(ev[2])
    tot_ms = ev[0].elapsed_time(ev[3])
    return {"code": code, "p": p, "decoder": name, "frames": nframes, "lmax": lmax, "failures": fails,
            "fer": fails / nframes, "fer_wilson95": [lo, hi], "mean_iters": isum / nframes,
            "p99_iters": float(torch.quantile(it, 0.99).item()),
            "decode_ms": dec_ms, "decode_frames_per_s": nframes / (dec_ms * 1e-3),
            "step_frames_per_s": nframes / (tot_ms * 1e-3),
            "edge_updates_per_s": isum * g.n_edges / (dec_ms * 1e-3)}


def main():
    import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--code", default="G63")
    ap.add_argument("--frames", type=int, default=workloads.SWEEP_FRAMES)
    ap.add_argument("--p", default=",".join(str(x) for x in workloads.P_GRID))
    ap.add_argument("--decoders", default=",".join(DECODERS))
    ap.add_argument("--lmax", type=int, default=workloads.SWEEP_LMAX)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    g = sagms.Graph.gb(*workloads.code(args.code))
    # warm-up: build device tables and gain tables, first launches
    run_point(g, args.code, 0.05, 0, "sagms", 4096, 10)
    rows = []
    for p in (float(x) for x in args.p.split(",")):
        sid = workloads.stream_of(p) if p in workloads.P_GRID else 0
        for name in args.decoders.split(","):
            r = run_point(g, args.code, p, sid, name, args.frames, args.lmax)
            print(json.dumps(r), flush=True)
            rows.append(r)
    print("\n| p | decoder | FER | 95 % Wilson | mean iters | p99 iters | decode frames/s | step frames/s |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        print("| %.2f | %s | %.3e | [%.3e, %.3e] | %.2f | %d | %.3g | %.3g |" % (
            r["p"], r["decoder"], r["fer"], r["fer_wilson95"][0], r["fer_wilson95"][1], r["mean_iters"],
            int(r["p99_iters"]), r["decode_frames_per_s"], r["step_frames_per_s"]))


if __name__ == "__main__":
    main()

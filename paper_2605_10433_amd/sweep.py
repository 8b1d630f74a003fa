"""Frame-error-rate sweep on one GPU.

    python -m paper_2605_10433_amd.sweep [--code G63] [--p 0.02,0.03,...]
        [--decoders ms,sms0.5,...,sagms,sagms-derived,bp] [--lmax 100]
        [--frames 1048576 | --until-failures 500 --max-frames 20000000]
        [--p0 0.1] [--ratio-ref sms0.5] [--joint]

For every noise level p and decoder: Philox frames of the depolarizing
channel (seed 1, stream = index of p in the grid, the same frames for every
decoder), syndromes, decoding and the logical judge, all through libsagms.
Frames run in chunks of at most 2^20 either up to --frames, or (Section V
setup's stopping rule) until --until-failures failures or --max-frames
frames.  --p0 decodes with the prior of p0 instead of p (channel mismatch,
Section V).  Decoders "sagms-derived" and "sagms-derived1.1" take their
gains from Corollary 1 (alpha_max = alpha*(L0, d_c), alpha_min = 0.6
alpha_max, eta = 1 / alpha_max or 1.1; sagms_derive_gains).  Decoders ending in "-layered" use
the layered schedule (SAGMS_LAYERED).  Prints one JSON
line per point (FER with its 95 % Wilson interval, mean and 99th-percentile
round count, decode and end-to-end frames/s, and with --ratio-ref the FER
ratio to that decoder with its 95 % log-method interval) and a markdown
table at the end.  --joint decodes X and Z together on the code's joint
graph (X- and Z-type rows; sagms_build_gb_joint) with the prior
ln((1 - p) / (p / 3)) of the paper's Section II, judged by sagms_judge_joint
(MS, SMS and SAGMS decoders).
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
from paper_2605_10433_amd.stats import fer_ratio_interval, wilson  # noqa: E402

DECODERS = {
    "ms": dict(kind="ms"),
    "sms0.5": dict(kind="sms", alpha=0.5),
    "sms0.625": dict(kind="sms", alpha=0.625),
    "sms0.75": dict(kind="sms", alpha=0.75),
    "sms0.875": dict(kind="sms", alpha=0.875),
    "sagms": dict(kind="sagms", alpha_min=0.30, alpha_max=0.50, eta=1.10),
    "sagms-derived": dict(derived=0.0),
    "sagms-derived1.1": dict(derived=1.1),
    "bp": dict(kind="bp"),
    "ms-layered": dict(kind="ms", schedule="layered"),
    "sms0.75-layered": dict(kind="sms", alpha=0.75, schedule="layered"),
    "sagms-layered": dict(kind="sagms", alpha_min=0.30, alpha_max=0.50, eta=1.10, schedule="layered"),
}
CHUNK = 1 << 20


def make_config(name, g, l0, lmax):
    spec = DECODERS[name]
    if "derived" in spec:
        return sagms.derived_config(l0, g.dc_max, ratio=0.6, eta=spec["derived"], lmax=lmax)
    return sagms.decoder_config(lmax=lmax, **spec)


def run_point(g, code, p, stream_id, name, lmax, frames=None, until_failures=None, max_frames=None, p0=None,
              seed=1):
    import torch
    joint = bool(g.joint)
    l0 = (sagms.depolarizing_llr if joint else sagms.prior_llr)(p0 if p0 is not None else p)
    cfg = make_config(name, g, l0, lmax)
    cap = frames if frames is not None else max_frames
    buf = sagms.frame_buffers(g, min(CHUNK, cap))
    llr = torch.full((g.n,), l0, dtype=torch.float32, device="cuda")
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    hist = torch.zeros(lmax + 1, dtype=torch.int64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    dec_ms = tot_ms = 0.0
    done = 0
    while done < cap:
        nf = min(CHUNK, cap - done)
        b = {k: (v[:nf] if v is not None else None) for k, v in buf.items()}
        ev[0].record()
        sagms.gen_errors(g, seed, stream_id, done, nf, p, b["ex"], b["ez"], b["synd"])
        ev[1].record()
        sagms.decode(g, b["synd"], llr, cfg, b["ehat"], b["iters"], b["converged"])
        ev[2].record()
        if joint:
            sagms.judge_joint(g, b["ex"], b["ez"], b["ehat"], b["converged"], b["iters"], counters)
        else:
            sagms.judge(g, b["ex"], b["ehat"], b["converged"], b["iters"], counters)
        ev[3].record()
        hist += torch.bincount(b["iters"].long(), minlength=lmax + 1)
        torch.cuda.synchronize()
        dec_ms += ev[1].elapsed_time(ev[2])
        tot_ms += ev[0].elapsed_time(ev[3])
        done += nf
        if until_failures is not None and int(counters[0].item()) >= until_failures:
            break
    fails, isum = (int(x) for x in counters.cpu().numpy())
    h = hist.cpu().numpy()
    p99 = int(np.searchsorted(np.cumsum(h), 0.99 * done))
    lo, hi = wilson(fails, done)
    r = {"code": code + (" joint" if joint else ""), "p": p, "decoder": name, "frames": done, "lmax": lmax,
         "failures": fails,
         "fer": fails / done, "fer_wilson95": [lo, hi], "mean_iters": isum / done, "p99_iters": p99,
         "decode_ms": dec_ms, "decode_frames_per_s": done / (dec_ms * 1e-3),
         "step_frames_per_s": done / (tot_ms * 1e-3),
         "edge_updates_per_s": isum * g.n_edges / (dec_ms * 1e-3)}
    if p0 is not None:
        r["p0"] = p0
    if cfg.kind == sagms.KINDS["sagms"]:
        r["gains"] = [cfg.alpha_min, cfg.alpha_max, cfg.eta]
    r["schedule"] = "layered" if cfg.schedule == sagms.SCHEDULES["layered"] else "flooding"
    return r


def main():
    import workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--code", default="G63")
    ap.add_argument("--frames", type=int, default=None, help="frames per point (default 2^20)")
    ap.add_argument("--until-failures", type=int, default=None, help="stop a point at this many failures")
    ap.add_argument("--max-frames", type=int, default=20_000_000, help="frame cap with --until-failures")
    ap.add_argument("--p", default=",".join(str(x) for x in workloads.P_GRID))
    ap.add_argument("--p0", type=float, default=None, help="decode with the prior of p0 (channel mismatch)")
    ap.add_argument("--decoders", default="ms,sms0.5,sms0.625,sms0.75,sms0.875,sagms,bp")
    ap.add_argument("--ratio-ref", default=None, help="report each decoder's FER ratio to this decoder")
    ap.add_argument("--lmax", type=int, default=workloads.SWEEP_LMAX)
    ap.add_argument("--joint", action="store_true", help="decode X and Z jointly on the code's joint graph")
    args = ap.parse_args()
    if args.frames is None and args.until_failures is None:
        args.frames = workloads.SWEEP_FRAMES
    import torch
    torch.cuda.set_device(0)
    g = (sagms.Graph.gb_joint if args.joint else sagms.Graph.gb)(*workloads.code(args.code))
    # warm-up: build device tables and gain tables, first launches
    run_point(g, args.code, 0.05, 0, "sagms", 10, frames=4096)
    rows = []
    names = args.decoders.split(",")
    if args.ratio_ref and args.ratio_ref not in names:
        names = [args.ratio_ref] + names
    for p in (float(x) for x in args.p.split(",")):
        sid = workloads.stream_of(p) if p in workloads.P_GRID else 0
        point = {}
        for name in names:
            r = run_point(g, args.code, p, sid, name, args.lmax, frames=args.frames,
                          until_failures=args.until_failures, max_frames=args.max_frames, p0=args.p0)
            point[name] = r
        if args.ratio_ref:
            ref = point[args.ratio_ref]
            for name, r in point.items():
                if r["failures"] > 0 and ref["failures"] > 0:
                    r["fer_ratio_to_" + args.ratio_ref] = list(fer_ratio_interval(r["failures"], r["frames"],
                                                                                  ref["failures"], ref["frames"]))
        for name in names:
            print(json.dumps(point[name]), flush=True)
            rows.append(point[name])
    print("\n| p | decoder | frames | FER | 95 %% Wilson | mean iters | p99 iters | decode frames/s |%s" %
          (" ratio to %s [95 %%] |" % args.ratio_ref if args.ratio_ref else ""))
    print("|---|---|---|---|---|---|---|---|%s" % ("---|" if args.ratio_ref else ""))
    for r in rows:
        extra = ""
        if args.ratio_ref:
            q = r.get("fer_ratio_to_" + args.ratio_ref)
            extra = " %.3f [%.3f, %.3f] |" % tuple(q) if q else " - |"
        print("| %.3f | %s | %d | %.3e | [%.3e, %.3e] | %.2f | %d | %.3g |%s" % (
            r["p"], r["decoder"], r["frames"], r["fer"], r["fer_wilson95"][0], r["fer_wilson95"][1],
            r["mean_iters"], r["p99_iters"], r["decode_frames_per_s"], extra))


if __name__ == "__main__":
    main()

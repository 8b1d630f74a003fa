"""Writes tests/golden/c1_calibration.json: the FP64 oracle on the CPU
calibration case -- the l = 63 GB code, p = 0.05, Philox seed 1 / stream 0,
frames 0 .. 9999, l_max = 50, flooding, MS / SMS (alpha = 0.75) / SAGMS
(0.30, 0.50, 1.10), prior ln((1 - 2p/3)/(2p/3)) in double.  Calls only the
oracle.  Run from the repository root:  python tests/golden/make_c1.py
"""
import base64
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import channel, codes, decoders, judge  # noqa: E402


def main():
    c = workloads.CALIB
    l, a, b = workloads.code(c["code"])
    hx, hz = codes.gb_matrices(l, a, b)
    tg = decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b))
    lz = codes.logical_basis(hz, hx)
    ex, _ = channel.sample_paulis(c["seed"], c["stream"], 0, c["frames"], 2 * l, c["p"])
    s = channel.syndrome(hz, ex)
    llr64 = np.full(2 * l, channel.prior_llr(c["p"]))
    llr32 = llr64.astype(np.float32)
    out = dict(c, about="oracle results of the CPU calibration case: FP64 mode with the FP64 prior, and FP32 "
                        "mode with the float prior (tests/golden/make_c1.py)", decoders={})
    for name, kw in (("ms", dict(kind="ms")), ("sms", dict(kind="sms", alpha=0.75)),
                     ("sagms", dict(kind="sagms", **workloads.SAGMS_PARAMS))):
        out["decoders"][name] = dict(params=kw)
        for mode, llr in (("fp64", llr64), ("fp32", llr32)):
            r = decoders.decode(tg, s, llr, decoders.DecoderParams(lmax=c["lmax"], **kw), mode)
            fail = judge.judge_logical(lz, ex, r.ehat, r.converged)
            out["decoders"][name][mode] = dict(
                failures=int(fail.sum()), sum_iters=int(r.iters.sum()),
                fail_bits=base64.b64encode(np.packbits(fail.astype(np.uint8)).tobytes()).decode(),
                iters=base64.b64encode(r.iters.astype(np.uint8).tobytes()).decode())
            print(name, mode, "FER", fail.mean(), "mean iters", r.iters.mean(), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_calibration.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()

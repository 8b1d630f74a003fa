"""Reduced-precision messages on the mixed-code workload, against FP64.

For every code of the mix and p in {0.03, 0.05}: the first frames of the
mix's Philox streams are decoded on the GPU with FP32, FP16 and INT6
messages (SAGMS) and by the FP64 oracle.  Recorded: each format's FER and
the fraction of frames whose hard decision differs from FP64.  Asserted:
FP32 and FP16 agree with FP64 on nearly every frame; INT6's FER lies within
the Wilson interval of the FP64 FER on the same frames, widened by the
coarse grid's own effect (checked only where FP64 converges on most frames).
With SAGMS_RECORD_DIR set, the records are written to precision_mix.json
in that folder.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import channel, codes, decoders, judge, stats  # noqa: E402

pytestmark = pytest.mark.gpu

FRAMES = 512
RECORDS = []


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield torch.device("cuda:0")
    out = os.environ.get("SAGMS_RECORD_DIR")
    if RECORDS and out and os.path.isdir(out):
        with open(os.path.join(out, "precision_mix.json"), "w") as fh:
            json.dump(RECORDS, fh, indent=1)


@pytest.mark.parametrize("p", workloads.PRECISION_P)
@pytest.mark.parametrize("idx", range(len(workloads.MIX_CODES)))
def test_formats_against_fp64(dev, idx, p):
    name = workloads.MIX_CODES[idx]
    l, a, b = workloads.code(name)
    hx, hz = codes.gb_matrices(l, a, b)
    lz = codes.logical_basis(hz, hx)
    sid = workloads.mix_stream(idx, p)
    ex, _ = channel.sample_paulis(workloads.MIX_SEED, sid, 0, FRAMES, 2 * l, p)
    synd = channel.syndrome(hz, ex)
    ref = decoders.decode(decoders.TannerGraph(hz, codes.gb_var_checks(l, a, b)), synd,
                          np.full(2 * l, channel.prior_llr(p)),
                          decoders.DecoderParams(kind="sagms", lmax=workloads.MIX_LMAX, **workloads.SAGMS_PARAMS),
                          "fp64")
    fer64 = judge.judge_logical(lz, ex, ref.ehat, ref.converged)
    g = sagms.Graph.gb(l, a, b)
    synd_dev = torch.from_numpy(channel.pack(synd).view(np.int64)).to(dev)
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    rec = {"code": name, "p": p, "frames": FRAMES, "fp64_fer": float(fer64.mean()),
           "fp64_converged": float(ref.converged.mean())}
    for fmt in ("fp32", "fp16", "int6"):
        print("precision", name, p, fmt, flush=True)
        cfg = sagms.decoder_config("sagms", lmax=workloads.MIX_LMAX, precision=fmt, **workloads.SAGMS_PARAMS)
        out = sagms.frame_buffers(g, FRAMES, device=dev)
        sagms.decode(g, synd_dev, llr, cfg, out["ehat"], out["iters"], out["converged"])
        torch.cuda.synchronize()
        ehat = channel.unpack(out["ehat"].cpu().numpy().view(np.uint64), g.n)
        conv = out["converged"].cpu().numpy().astype(bool)
        fail = judge.judge_logical(lz, ex, ehat, conv)
        differ = (ehat != ref.ehat).any(axis=1)
        lo, hi = stats.wilson(int(fail.sum()), FRAMES)
        rec[fmt] = {"fer": float(fail.mean()), "fer_wilson95": [lo, hi], "hd_differs_from_fp64": float(differ.mean()),
                    "mean_iters": float(out["iters"].float().mean().item())}
        if fmt in ("fp32", "fp16"):
            # both keep the FP64 trajectory on converging frames up to rounding
            both = conv & ref.converged
            assert (differ & both).mean() <= (0.02 if fmt == "fp32" else 0.05), (name, p, fmt, (differ & both).mean())
        elif ref.converged.mean() > 0.9:
            lo64, hi64 = stats.wilson(int(fer64.sum()), FRAMES)
            assert lo64 - 0.02 <= fail.mean() <= hi64 + 0.02, (name, p, fmt, fail.mean(), lo64, hi64)
    RECORDS.append(rec)
    print(json.dumps(rec), flush=True)

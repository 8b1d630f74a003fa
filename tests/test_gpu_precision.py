"""Message formats on the mixed-code workload, against the FP64 oracle.

For every code of the mix and p in {0.03, 0.05}: the first FRAMES frames of
the mix's Philox streams are decoded on the GPU with FP32, FP16 and INT6
messages (SAGMS) and by the FP64 oracle (FP64 prior) in a pool of host
processes.  Recorded per format: FER with its 95 % Wilson interval, the
fraction of frames whose hard decision differs from FP64 (all frames, and
frames converged in both), and the paired failure counts b (FP64 fails, the
format does not) and c (the reverse).

Asserted:
* FP32 and FP16: the FER lies in the FP64 FER's Wilson interval and the
  paired difference c - b lies within 3 sigma of 0 (|c - b| <= 3 sqrt(b + c),
  the normal approximation of the sign test on the discordant frames);
* every format: among frames that converge in both, the hard decision
  differs from FP64's in at most 1 % (they reach the same syndrome-matching
  estimate).
INT6 (a sign and 6-bit magnitude on a 1/4 grid) is a different decoder
whose FER is reported, not matched: on the weight-3 l = 255 code at p = 0.05
it fails measurably more often than FP64.

FRAMES = 2^14 by default (about a minute of oracle time on 16 processes);
2^16 with SAGMS_PRECISION_FULL=1.  With SAGMS_RECORD_DIR set, the records are
written to precision_mix.json in that folder.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import stats  # noqa: E402

pytestmark = pytest.mark.gpu

FRAMES = 1 << (16 if os.environ.get("SAGMS_PRECISION_FULL") == "1" else 14)
CHUNK = 512
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


def oracle_fp64(pool, name, idx, p):
    import sweep_oracle  # tests/helpers, on the path of the pool's workers
    tasks = [dict(code=name, seed=workloads.MIX_SEED, stream=workloads.mix_stream(idx, p), kind="sagms",
                  kw=dict(workloads.SAGMS_PARAMS), p=p, frame0=f0, nframes=min(CHUNK, FRAMES - f0),
                  lmax=workloads.MIX_LMAX, arith="fp64") for f0 in range(0, FRAMES, CHUNK)]
    parts = sorted(pool.imap_unordered(sweep_oracle.decode_point, tasks), key=lambda r: r["frame0"])
    return {k: np.concatenate([r[k] for r in parts]) for k in ("synd", "ehat", "iters", "converged", "fail")}


@pytest.mark.parametrize("p", workloads.PRECISION_P)
@pytest.mark.parametrize("idx", range(len(workloads.MIX_CODES)))
def test_formats_against_fp64(dev, oracle_pool, idx, p):
    name = workloads.MIX_CODES[idx]
    print("precision", name, p, FRAMES, flush=True)
    ref = oracle_fp64(oracle_pool, name, idx, p)
    g = sagms.Graph.gb(*workloads.code(name))
    buf = sagms.frame_buffers(g, FRAMES, device=dev)
    sagms.gen_errors(g, workloads.MIX_SEED, workloads.mix_stream(idx, p), 0, FRAMES, p, buf["ex"], None, buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    assert (buf["synd"].cpu().numpy().view(np.uint64) == ref["synd"]).all()
    f64 = int(ref["fail"].sum())
    lo64, hi64 = stats.wilson(f64, FRAMES)
    rec = {"code": name, "p": p, "frames": FRAMES, "fp64_fer": f64 / FRAMES, "fp64_fer_wilson95": [lo64, hi64],
           "fp64_converged": float(ref["converged"].mean())}
    for fmt in ("fp32", "fp16", "int6"):
        cfg = sagms.decoder_config("sagms", lmax=workloads.MIX_LMAX, precision=fmt, **workloads.SAGMS_PARAMS)
        counters = torch.zeros(2, dtype=torch.int64, device=dev)
        sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
        sagms.judge(g, buf["ex"], buf["ehat"], buf["converged"], buf["iters"], counters, fail=buf["fail"])
        torch.cuda.synchronize()
        ehat = buf["ehat"].cpu().numpy().view(np.uint64)
        conv = buf["converged"].cpu().numpy().astype(bool)
        fail = buf["fail"].cpu().numpy().astype(bool)
        differ = (ehat != ref["ehat"]).any(axis=1)
        both = conv & ref["converged"]
        b = int((ref["fail"] & ~fail).sum())
        c = int((fail & ~ref["fail"]).sum())
        lo, hi = stats.wilson(int(fail.sum()), FRAMES)
        hd_both = float(differ[both].mean()) if both.any() else 0.0
        rec[fmt] = {"fer": float(fail.mean()), "fer_wilson95": [lo, hi], "hd_differs_from_fp64": float(differ.mean()),
                    "hd_differs_converged_both": hd_both,
                    "fp64_only_failures": b, "format_only_failures": c,
                    "mean_iters": float(buf["iters"].float().mean().item())}
        assert hd_both <= 0.01, (name, p, fmt, hd_both)
        if fmt in ("fp32", "fp16"):
            assert lo64 <= fail.mean() <= hi64, (name, p, fmt, float(fail.mean()), lo64, hi64)
            assert abs(c - b) <= 3.0 * np.sqrt(b + c), (name, p, fmt, b, c)
    RECORDS.append(rec)
    print(json.dumps(rec), flush=True)

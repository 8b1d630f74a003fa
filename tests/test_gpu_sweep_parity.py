"""Parity over the whole l = 63 noise sweep.

Every point of the sweep: p = 0.02 .. 0.10, frames of seed 1 and stream =
index of p, l_max = 100, decoded end to end by libsagms (Philox sampling,
syndromes, decoding, judge) and by the oracle in a pool of host processes.

* Every decoder of the sweep (MS, SMS with alpha = 0.5 / 0.625 / 0.75 /
  0.875, SAGMS with the Section V parameters) on the first FRAMES_EXACT
  frames of each point, frame by frame against the oracle's FP32 mode:
  syndromes, hard decisions, round counts, flags, posteriors and verdicts
  bit-exact.  BP (transcendental check rule): hard decision and round count
  agree on >= 97 % of frames, posteriors within 1e-4 relative on those
  (its per-round FP64 bar is in test_gpu_parity.py).
* SAGMS on the first FRAMES_FER frames of each point against the FP64
  oracle: each FER lies in the other's 95 % Wilson interval, and frames
  that converge in both agree in their hard decision on >= 99 %.
* SAGMS with FP16 and INT6 messages, and MS / SMS / SAGMS with the layered
  schedule, on the first FRAMES_REDUCED frames of each point, frame by frame
  against the oracle's matching mode.

Sizes: by default 2^12 / 2^16 / 2^10 frames (about a minute of oracle time
on 16 host processes); with SAGMS_SWEEP_PARITY=1 the sweep-scale sizes
2^16 / 2^20 / 2^16 (several minutes).  Workers: SAGMS_ORACLE_PROCS, default
the host's cores up to 16.  Each point prints one line starting with
"sweep-parity".
"""
import json
import os
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2605_10433_amd as sagms  # noqa: E402
import workloads  # noqa: E402
from oracle import stats  # noqa: E402

pytestmark = pytest.mark.gpu

FULL = os.environ.get("SAGMS_SWEEP_PARITY") == "1"
FRAMES_EXACT = 1 << (16 if FULL else 12)
FRAMES_FER = 1 << (20 if FULL else 16)
FRAMES_REDUCED = 1 << (16 if FULL else 10)
LMAX = workloads.SWEEP_LMAX
DECODERS = ([("ms", {})] + [("sms", dict(alpha=a)) for a in workloads.SMS_ALPHAS] +
            [("sagms", dict(workloads.SAGMS_PARAMS)), ("bp", {})])


def say(tag, **kw):
    print("sweep-parity", tag, json.dumps(kw), flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def pool(oracle_pool):
    return oracle_pool


@pytest.fixture(scope="module")
def g63(dev):
    return sagms.Graph.gb(*workloads.code("G63"))


def oracle_run(pool, kind, kw, p, nframes, arith, schedule="flooding"):
    import sweep_oracle   # tests/helpers, on the path the pool's workers inherit
    chunk = min(4096, max(128, nframes // 32))  # enough tasks to keep every worker busy
    tasks = [(kind, kw, p, f0, min(chunk, nframes - f0), LMAX, arith, schedule) for f0 in range(0, nframes, chunk)]
    parts = sorted(pool.imap_unordered(sweep_oracle.decode_chunk, tasks), key=lambda r: r["frame0"])
    return {k: np.concatenate([r[k] for r in parts]) for k in parts[0] if k != "frame0"}


def gpu_run(g, kind, kw, p, nframes, soft, **cfg_kw):
    buf = sagms.frame_buffers(g, nframes)
    sagms.gen_errors(g, workloads.SWEEP_SEED, workloads.stream_of(p), 0, nframes, p, buf["ex"], buf["ez"],
                     buf["synd"])
    llr = torch.full((g.n,), sagms.prior_llr(p), dtype=torch.float32, device="cuda")
    cfg = sagms.decoder_config(kind, lmax=LMAX, **kw, **cfg_kw)
    post = torch.empty((nframes, g.n), dtype=torch.float32, device="cuda") if soft else None
    if soft:
        sagms.decode_soft(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"], post)
    else:
        sagms.decode(g, buf["synd"], llr, cfg, buf["ehat"], buf["iters"], buf["converged"])
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    sagms.judge(g, buf["ex"], buf["ehat"], buf["converged"], buf["iters"], counters, fail=buf["fail"])
    torch.cuda.synchronize()
    out = dict(synd=buf["synd"].cpu().numpy().view(np.uint64), ehat=buf["ehat"].cpu().numpy().view(np.uint64),
               iters=buf["iters"].cpu().numpy(), converged=buf["converged"].cpu().numpy().astype(bool),
               fail=buf["fail"].cpu().numpy().astype(bool), counters=counters.cpu().numpy())
    if soft:
        out["posterior"] = post.cpu().numpy()
    return out


@pytest.mark.parametrize("p", workloads.P_GRID)
@pytest.mark.parametrize("kind,kw", DECODERS)
def test_sweep_point_frame_by_frame(g63, pool, kind, kw, p):
    t0 = time.perf_counter()
    r = oracle_run(pool, kind, kw, p, FRAMES_EXACT, "fp32")
    t_oracle = time.perf_counter() - t0
    q = gpu_run(g63, kind, kw, p, FRAMES_EXACT, soft=True)
    assert (q["synd"] == r["synd"]).all()
    assert q["counters"][0] == q["fail"].sum() and q["counters"][1] == q["iters"].astype(np.int64).sum()
    if kind == "bp":
        agree = (q["iters"] == r["iters"]) & (q["ehat"] == r["ehat"]).all(axis=1)
        tol = 1e-4 * np.maximum(np.abs(r["posterior"][agree]), sagms.prior_llr(p))
        close = (np.abs(q["posterior"][agree] - r["posterior"][agree]) <= tol).all(axis=1)
        say("bp", p=p, frames=FRAMES_EXACT, agree=float(agree.mean()), close=float(close.mean()),
            fer_gpu=float(q["fail"].mean()), fer_oracle=float(r["fail"].mean()), oracle_s=round(t_oracle, 1))
        assert agree.mean() >= 0.97 and close.mean() >= 0.97
        return
    mismatched = int(((q["ehat"] != r["ehat"]).any(axis=1) | (q["iters"] != r["iters"]) |
                      (q["converged"] != r["converged"]) |
                      (q["posterior"].view(np.uint32) != r["posterior"].view(np.uint32)).any(axis=1)).sum())
    say(kind, kw=kw, p=p, frames=FRAMES_EXACT, mismatched_frames=mismatched, fer=float(q["fail"].mean()),
        mean_iters=float(q["iters"].mean()), oracle_s=round(t_oracle, 1))
    assert mismatched == 0
    assert (q["fail"] == r["fail"]).all()


@pytest.mark.parametrize("p", workloads.P_GRID)
def test_sagms_fer_against_fp64(g63, pool, p):
    t0 = time.perf_counter()
    r = oracle_run(pool, "sagms", workloads.SAGMS_PARAMS, p, FRAMES_FER, "fp64")
    t_oracle = time.perf_counter() - t0
    q = gpu_run(g63, "sagms", workloads.SAGMS_PARAMS, p, FRAMES_FER, soft=False)
    assert (q["synd"] == r["synd"]).all()
    f_gpu, f_64 = int(q["fail"].sum()), int(r["fail"].sum())
    lo_g, hi_g = stats.wilson(f_gpu, FRAMES_FER)
    lo_o, hi_o = stats.wilson(f_64, FRAMES_FER)
    both = q["converged"] & r["converged"]
    differ = (q["ehat"] != r["ehat"]).any(axis=1)
    say("sagms-fp64", p=p, frames=FRAMES_FER, failures_gpu=f_gpu, failures_fp64=f_64,
        wilson_gpu=[lo_g, hi_g], wilson_fp64=[lo_o, hi_o], frames_differing=int(differ.sum()),
        hd_differ_converged_both=float(differ[both].mean()), rounds_differ=int((q["iters"] != r["iters"]).sum()),
        oracle_s=round(t_oracle, 1))
    assert lo_o <= f_gpu / FRAMES_FER <= hi_o and lo_g <= f_64 / FRAMES_FER <= hi_g
    assert differ[both].mean() < 0.01


def same_frames(q, r):
    """Frames whose decision, rounds, flag or any posterior bit differ
    (posteriors that overflowed to NaN must be NaN on both sides)."""
    nan = np.isnan(r["posterior"])
    post_diff = (q["posterior"].view(np.uint32) != r["posterior"].view(np.uint32)) & ~nan
    post_diff |= np.isnan(q["posterior"]) != nan
    return int(((q["ehat"] != r["ehat"]).any(axis=1) | (q["iters"] != r["iters"]) |
                (q["converged"] != r["converged"]) | post_diff.any(axis=1)).sum())


@pytest.mark.parametrize("p", workloads.P_GRID)
@pytest.mark.parametrize("precision", ["fp16", "int6"])
def test_sweep_point_reduced_precision(g63, pool, precision, p):
    """SAGMS with FP16 and INT6 messages on the first FRAMES_REDUCED frames of
    every point, frame by frame against the oracle's matching mode."""
    t0 = time.perf_counter()
    r = oracle_run(pool, "sagms", workloads.SAGMS_PARAMS, p, FRAMES_REDUCED, precision)
    t_oracle = time.perf_counter() - t0
    q = gpu_run(g63, "sagms", workloads.SAGMS_PARAMS, p, FRAMES_REDUCED, soft=True, precision=precision)
    assert (q["synd"] == r["synd"]).all()
    bad = same_frames(q, r)
    say("sagms-" + precision, p=p, frames=FRAMES_REDUCED, mismatched_frames=bad, fer=float(q["fail"].mean()),
        mean_iters=float(q["iters"].mean()), oracle_s=round(t_oracle, 1))
    assert bad == 0 and (q["fail"] == r["fail"]).all()


@pytest.mark.parametrize("p", workloads.P_GRID)
@pytest.mark.parametrize("kind,kw", [("ms", {}), ("sms", dict(alpha=0.75)), ("sagms", dict(workloads.SAGMS_PARAMS))])
def test_sweep_point_layered(g63, pool, kind, kw, p):
    """The layered schedule on the first FRAMES_REDUCED frames of every point,
    frame by frame against the oracle's layered FP32 mode."""
    t0 = time.perf_counter()
    r = oracle_run(pool, kind, kw, p, FRAMES_REDUCED, "fp32", "layered")
    t_oracle = time.perf_counter() - t0
    q = gpu_run(g63, kind, kw, p, FRAMES_REDUCED, soft=True, schedule="layered")
    assert (q["synd"] == r["synd"]).all()
    bad = same_frames(q, r)
    say(kind + "-layered", kw=kw, p=p, frames=FRAMES_REDUCED, mismatched_frames=bad, fer=float(q["fail"].mean()),
        mean_iters=float(q["iters"].mean()), oracle_s=round(t_oracle, 1))
    assert bad == 0 and (q["fail"] == r["fail"]).all()

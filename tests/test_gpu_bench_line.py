"""The bench's result line on the GPU: a short run of bench.py (two timed
steps of the l = 63 workload) prints one JSON line with the fields its
readers rely on: the metric and its unit, the timed steps, one GPU, the
configuration, the roofline object of the decode kernel (with the fraction
by the 14-operation count fixed before tuning), the FP16 pass over the same
frames and the serving latency at 80 % load.  The mixed-code workload's line, after the plan
autotuner, names the tuned plan and the tuner's log."""
import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_complete_line():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench line: 2 steps, 2 warm-up steps", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "2",
                        "--no-cpu-baseline"], capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    out = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in out, key
    assert out["n_gpus"] == 1 and out["steps"] == 2 and out["warmup"] == 2
    assert out["value"] > 0 and out["ms_per_step"] > 0 and out["higher_is_better"] is True
    assert out["unit"] == "frames/s" and out["dtype"] == "f32" and out["data"] == "synthetic"
    assert "workload" in out["config"] and out["config"]["frames_per_step"] == 1 << 20
    rl = out["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rl, key
    assert rl["bound"] == "alu" and rl["unit"] == "TOP/s"
    assert 0 < rl["frac"] <= 1 and rl["frac"] == pytest.approx(rl["achieved"] / rl["peak"], rel=1e-9)
    # the whole step takes at least as long as its decode
    assert out["decode_ms_per_step"] <= out["ms_per_step"]
    assert rl["frac_14_ops"] == pytest.approx(rl["frac"] * 14 / rl["ops_per_edge_update"], rel=1e-9)
    assert "counters" in rl
    f16 = out["fp16"]
    assert f16["value"] > 0 and f16["vs_fp32"] == pytest.approx(f16["value"] / out["value"], rel=1e-9)
    assert 0 <= f16["fer"] <= 1 and isinstance(f16["fer_in_fp32_interval"], bool)
    srv = out["serving_p80"]
    assert 0 < srv["p50_us"] <= srv["p99_us"] and srv["offered_load"] == 0.8 and srv["requests"] > 0
    assert len(srv["traces"]) == 2 and srv["p99_us"] == max(t["p99_us"] for t in srv["traces"])
    for t in srv["traces"]:
        assert 0 < t["p50_us"] <= t["p99_us"] and t["served_frames_per_s"] > 0


def test_mix_workload_line_with_tuner():
    """bench.py --workload mix --tune: one line naming the tuned plan (with
    its unroll), the tuner's log and the per-code FER of the mixed batch."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench line: mix, tuned, 2 steps", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--workload", "mix", "--tune",
                        "--steps", "2", "--warmup", "1", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    out = json.loads(lines[0])
    assert out["value"] > 0 and out["steps"] == 2 and out["config"]["tuned"] is True
    plan = out["config"]["plan"]
    assert plan["unroll"] in (1, 2)
    best = min(out["tune"], key=lambda t: t["ms"])
    assert best["plan"] == plan
    assert {t["plan"]["unroll"] for t in out["tune"] if t["plan"]["kind"] != "per_code"} == {1, 2}
    assert set(out["per_code"]) == set(out["config"]["codes"])
    for rec in out["per_code"].values():
        assert 0 <= rec["fer"] <= 1 and rec["mean_iters"] > 0

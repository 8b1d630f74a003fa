"""Host logic of bench.py (no GPU): the one-GPU guard, the decode-source
hash that keys the traffic record, the record lookup, and the oracle
baseline's result format on a tiny sample."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_source_hash_covers_every_decode_source(tmp_path, monkeypatch):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--source-sha"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT).stdout.strip()
    assert out == bench.decode_source_sha256() and len(out) == 64
    # a change to any of the hashed files changes the hash
    copies = []
    for f in bench.DECODE_SOURCES:
        c = tmp_path / os.path.basename(f)
        c.write_bytes(open(f, "rb").read())
        copies.append(str(c))
    monkeypatch.setattr(bench, "DECODE_SOURCES", copies)
    assert bench.decode_source_sha256() == out
    for c in copies:
        orig = open(c, "rb").read()
        open(c, "wb").write(orig + b"\n")
        assert bench.decode_source_sha256() != out
        open(c, "wb").write(orig)


def test_traffic_record_used_only_for_its_sources_and_workload(tmp_path, monkeypatch):
    rec = {"decode_source_sha256": bench.decode_source_sha256(), "frames_per_launch": 1 << 20, "p": 0.05,
           "fetch_kib": 100.0, "fetch_scale": 2.0, "write_kib": 50.0, "write_scale": 1.0}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic(1 << 20, 0.05) == 1024.0 * 250.0
    assert bench.measured_traffic(1 << 19, 0.05) is None
    assert bench.measured_traffic(1 << 20, 0.04) is None
    rec["decode_source_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic(1 << 20, 0.05) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(1 << 20, 0.05) is None


def test_cpu_baseline_format_on_a_tiny_sample():
    import workloads
    out = bench.cpu_baseline(0.05, 20, workloads.SAGMS_PARAMS, frames=32, procs=1)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "frames/s" and out["value"] > 0
    assert "32 frames" in out["sample"]
    dt, fails, dec, isum = bench.oracle_frames(0.05, 20, {}, 0, 16, "ms")
    assert dt >= dec > 0 and 0 <= fails <= 16 and isum >= 0

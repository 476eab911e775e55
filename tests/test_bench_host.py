"""Host-side checks of the benchmark script (no GPU): it refuses more than one GPU with one JSON
line, it reports the counter traffic only while the kernel source is the one the committed
counters were taken on, and its CPU-baseline leg (the FP64 oracle) returns a rate with the
thread count and the sample it timed."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_one_json_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    msg = json.loads(lines[0])
    assert "one GPU" in msg["error"]


def test_counter_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    import hashlib
    import bench
    src = tmp_path / "kernels.hip"
    src.write_bytes(b"// a kernel source\n")
    cnt = tmp_path / "counters.txt"
    cnt.write_text("# header: a comment line\ntraffic_bytes_per_step: 12345\n"
                   "kernel_config: march4-xcd\n"
                   "kernel_source_sha256: %s\n" % hashlib.sha256(src.read_bytes()).hexdigest())
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "COUNTERS", str(cnt))
    assert bench.counter_traffic("march4-xcd") == 12345.0
    assert bench.counter_traffic("march2-xcd") is None   # counters of another configuration
    src.write_bytes(b"// a kernel source, changed\n")
    assert bench.counter_traffic("march4-xcd") is None   # any change to the source voids it
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.txt"))
    assert bench.counter_traffic("march4-xcd") is None


def test_cpu_baseline_reports_rate_threads_and_sample():
    import bench
    from paper_2311_02293_amd import inputs as I
    job = I.config2(n1=60, n2=120, nt=50, nshot=2)
    job.grid.vpmax = float(job.vp.max())
    out = bench.cpu_baseline(job, 20, one_thread_steps=10)
    assert out["kind"] == "oracle" and out["unit"] == "GPts/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "20 of 50 steps" in out["sample"]
    one = out["one_thread"]
    assert one["cores"] == 1 and one["value"] > 0 and "10 steps" in one["sample"]

"""Host-side logic of bench.py (no GPU): the roofline entry built from a
profiled pass's per-class statistics, the measured-traffic lookup keyed to
the hash of the kernel's source, the committed traffic table, and the
refusal of more than one GPU."""
import hashlib
import importlib.util
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_table_names_existing_sources_and_profiles():
    rows = 0
    for line in open(os.path.join(ROOT, "profiles", "hbm_traffic.txt")):
        if line.startswith("#") or not line.strip():
            continue
        workload, cls, src, digest, value, profile = line.split()
        assert os.path.isfile(os.path.join(ROOT, src)), src
        assert os.path.isfile(os.path.join(ROOT, "profiles", profile)), profile
        assert re.fullmatch(r"[0-9a-f]{12}", digest), digest
        assert float(value) > 0, line
        rows += 1
    assert rows >= 1


def test_measured_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    bench = _bench()
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"kernel, first form")
    digest = hashlib.sha1(b"kernel, first form").hexdigest()[:12]
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hbm_traffic.txt").write_text(
        f"# workload kernel_class source_file sha1_12 bytes_per_launch profile\nw1 cls kernel.hip {digest} 1234 p.md\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w1", "cls") == 1234.0
    assert bench.measured_traffic("w2", "cls") is None
    assert bench.measured_traffic("w1", "other") is None
    src.write_bytes(b"kernel, changed since the counters were taken")
    assert bench.measured_traffic("w1", "cls") is None


def test_roofline_takes_the_class_with_the_most_time():
    bench = _bench()
    stats = {"small": dict(total_ms=1.0, bytes=1e9, launches=2),
             "large": dict(total_ms=2.0, bytes=8e9, launches=4)}
    roof, per_step = bench._roofline(stats, "no such workload", steps=2)
    assert roof["kernel"] == "large" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    assert roof["achieved"] == 4000.0                     # 8e9 B in 2 ms
    assert roof["frac"] == round(4000.0 / bench.HBM_PEAK_GBS, 4)
    assert roof["avg_launch_us"] == 500.0 and roof["bytes_per_launch"] == 2e9
    assert roof["traffic"] is None
    assert per_step["small"]["launches"] == 1.0 and per_step["large"]["ms"] == 1.0
    assert per_step["large"]["gbs"] == 4000.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr

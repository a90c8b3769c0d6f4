"""CPU checks of bench.py's contract: one GPU only, and the roofline's HBM traffic
taken from a counter profile only when the profile was taken on these kernel
sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_from_a_profile_of_the_same_sources(tmp_path, monkeypatch):
    src = bench.kernel_sources_sha256()
    prof = tmp_path / "counters.md"
    prof.write_text(f"kernel sources sha256: {src}\n\ntraffic_bytes k_integrate: 123456\n")
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(prof))
    assert bench.measured_traffic("k_integrate") == 123456.0
    assert bench.measured_traffic("k_merge") is None
    prof.write_text("kernel sources sha256: 0000\n\ntraffic_bytes k_integrate: 123456\n")
    assert bench.measured_traffic("k_integrate") is None
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("k_integrate") is None

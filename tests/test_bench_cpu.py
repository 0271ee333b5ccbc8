"""bench.py's contract on the CPU: more than one GPU is refused with a message,
and the counter summary keeps the profiled kernel's source hash."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_recorded_traffic_is_void_when_the_kernel_changed(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "TRAFFIC_DIR", str(tmp_path))
    f = tmp_path / "traffic_cX.json"
    kernels = {"k_group": {"hbm_bytes_per_launch": 123.0, "launches": 6},
               "k_fill_rows": {"hbm_bytes_per_launch": 10.0, "launches": 3}}
    f.write_text(json.dumps({"source_sha": bench.source_sha(), "steps": 3, "kernels": kernels}))
    # per step: 123 x 6 / 3 + 10 x 3 / 3
    assert bench.recorded_traffic(("k_group", "k_fill_rows", "k_absent"), "cX") == 256.0
    f.write_text(json.dumps({"source_sha": "0" * 16, "steps": 3, "kernels": kernels}))
    assert bench.recorded_traffic(("k_group",), "cX") is None
    assert bench.recorded_traffic(("k_group",), "missing") is None

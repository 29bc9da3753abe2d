"""Host logic of bench.py that needs no GPU: the counter traffic it reports
is used only while the kernel sources and the launch match the counters'
record, and more than one GPU is refused."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_traffic_only_for_matching_sources_and_launch(monkeypatch, tmp_path):
    rec = {"kernel_source_hash": "abc", "launch": [1, 4, 64, 256, 32, 768], "hbm_bytes_per_launch": 3.9e10}
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_JSON", str(path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.measured_traffic([1, 4, 64, 256, 32, 768]) == 3.9e10
    assert bench.measured_traffic([1, 4, 64, 512, 32, 768]) is None      # another launch
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "changed")
    assert bench.measured_traffic([1, 4, 64, 256, 32, 768]) is None      # kernel changed since
    monkeypatch.setattr(bench, "PROFILE_JSON", str(tmp_path / "missing.json"))
    assert bench.measured_traffic([1, 4, 64, 256, 32, 768]) is None


def test_committed_counter_record_is_consistent():
    # the record names its kernel, workload and summary, and its byte total is
    # the sum of the scaled counters
    with open(bench.PROFILE_JSON) as fh:
        rec = json.load(fh)
    assert rec["workload"] == "lattice1024_expanding"
    assert os.path.exists(os.path.join(ROOT, "profiles", rec["summary"]))
    total = rec["fetch_size_kib"] * 1024 * rec["fetch_scale"] + rec["write_size_kib"] * 1024 * rec["write_scale"]
    assert abs(total - rec["hbm_bytes_per_launch"]) <= 1e-9 * total
    alg = 16.0 * 1024 ** 3 * 2
    assert 1.0 <= rec["hbm_bytes_per_launch"] / alg < 1.5


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr

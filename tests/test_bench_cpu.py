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


def _write_counter_csv(path, rows):
    import csv
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_counter_summary_scales_by_the_copy(tmp_path, monkeypatch):
    """The summary takes the step kernel's dispatches (skipping two), scales
    FETCH_SIZE and WRITE_SIZE by what they read for the 8 GiB copy, and takes
    the launch from the profiled run's JSON line."""
    step = "void ce::(anonymous namespace)::" + bench.STEP_KERNEL + "(ce::Lattice, int)"
    other = "void ce::(anonymous namespace)::tiled3d_kernel<float, 2, 0, 0, 4, 64, 512>(ce::Lattice, int)"
    fetch = [(i, step, "FETCH_SIZE", 100.0 if i < 2 else 1000.0) for i in range(6)] + [(9, other, "FETCH_SIZE", 5.0)]
    write = [(i, step, "WRITE_SIZE", 2000.0) for i in range(6)]
    _write_counter_csv(tmp_path / "f.csv", fetch)
    _write_counter_csv(tmp_path / "w.csv", write)
    gib8 = 8 * 1024 ** 3
    _write_counter_csv(tmp_path / "cf.csv", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", gib8 / 2048.0),
                                              (2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 3.0)])
    _write_counter_csv(tmp_path / "cw.csv", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", gib8 / 1024.0)])
    (tmp_path / "stats.csv").write_text('"Name","Calls","TotalDurationNs","AverageNs"\n'
                                        f'"{step}",10,70000000,7000000\n')
    (tmp_path / "run.log").write_text("[bench] timed\n" + json.dumps({"diagnostics": {"launch": [1, 4, 64, 256, 114, 768]}}) + "\n")
    out = tmp_path / "rec.json"
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h")
    rec = bench.counter_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                                str(tmp_path / "cw.csv"), str(tmp_path / "stats.csv"), str(tmp_path / "run.log"),
                                out=str(out))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_size_kib"] == 1000.0 and rec["write_size_kib"] == 2000.0
    assert rec["hbm_bytes_per_launch"] == 1000.0 * 1024 * 2 + 2000.0 * 1024
    assert rec["launch"] == [1, 4, 64, 256, 114, 768] and rec["kernel_avg_ms"] == 7.0
    assert rec["kernel_source_hash"] == "h" and json.loads(out.read_text()) == rec


def test_ceiling_sweeps_are_within_the_probe_limits():
    """Every configuration the ceiling module times is one the probe accepts
    (parts 1 or 4, unroll 1-8, nt bits 0-3; read-only never asks for
    nontemporal stores, write-only never for nontemporal loads)."""
    from paper_0712_0813_amd import ceiling
    full = ceiling.full_sweep()
    assert {k: len(v) for k, v in full.items()} == {"copy": 192, "read": 96, "write": 96}
    for sweep in (full, ceiling.COMPACT):
        for kind, cfgs in sweep.items():
            assert len(set(cfgs)) == len(cfgs)
            for parts, unroll, nt, per_cu in cfgs:
                assert parts in (1, 4) and unroll in (1, 2, 4, 8) and 0 <= nt <= 3 and 1 <= per_cu <= 64
                assert not (kind == "read" and nt & 2) and not (kind == "write" and nt & 1)
        assert set(sweep) == {"copy", "read", "write"}

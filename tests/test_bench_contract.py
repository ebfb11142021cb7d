"""bench.py's host-side contract, on the CPU: more than one GPU is refused
with a message before anything touches a device, and the HBM traffic of a
kernel is taken from a committed counter record only while the kernel
sources still hash to the profiled ones."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_used_only_for_unchanged_sources(tmp_path, monkeypatch):
    bench = load_bench()
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    rec = {"kernel": "k<3>", "workload": "w", "sources": ["k.hip"],
           "source_sha256": hashlib.sha256(b"kernel v1\n").hexdigest(),
           "hbm_bytes_per_launch": 1234.0}
    (tmp_path / "profiles" / "traffic_k_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("k<3>", "w") == 1234.0
    assert bench.profiled_traffic("k<3>", "other workload") is None
    assert bench.profiled_traffic("k<2>", "w") is None
    src.write_text("kernel v2\n")
    assert bench.profiled_traffic("k<3>", "w") is None


def test_committed_traffic_records_name_existing_sources():
    d = os.path.join(ROOT, "profiles")
    recs = [f for f in os.listdir(d) if f.startswith("traffic_") and f.endswith(".json")]
    assert recs
    for f in recs:
        rec = json.load(open(os.path.join(d, f)))
        for s in rec["sources"]:
            assert os.path.exists(os.path.join(ROOT, s)), (f, s)
        assert rec["hbm_bytes_per_launch"] > 0
        assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0

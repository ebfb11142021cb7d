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


def test_validation_scores_truth_and_planted_mistakes():
    """The run record's hit-selection accuracy, purity and efficiency: 1 for
    tracks that select exactly their truth hits; a planted wrong hit and a
    planted miss lower them by the expected amounts."""
    import numpy as np
    from synth import generate, small_barrel
    bench = load_bench()
    w = small_barrel()
    b = generate(w)
    E = b.events[0]
    n = E.seed_track.shape[0]
    tr = np.zeros(n, dtype=[("hit", np.int32, (32,))])
    tr["hit"][:] = -1
    plan = np.zeros((n, 32), np.int8)
    plen = np.zeros(n, np.int32)
    for s, t in enumerate(E.seed_track):
        th = E.track_hits[t][3:]
        plen[s] = th.shape[0]
        plan[s, :th.shape[0]] = E.layer[th]
        tr["hit"][s, :th.shape[0]] = th
    ok = np.ones(n, np.int32)
    v = bench.validation(b, tr, plen, plan, ok)
    assert v["hit_selection_accuracy"] == 1.0 and v["hit_purity"] == 1.0
    assert v["efficiency_75pct"] == 1.0 and v["seeds"] == n
    total = int(plen.sum())
    # seed 0's first found hit replaced by another track's hit on that layer
    s0, t0 = 0, int(E.seed_track[0])
    lay = plan[s0, 0]
    other = np.nonzero((E.layer == lay) & (E.track != t0) & (E.track >= 0))[0][0]
    tr["hit"][s0, 0] = other
    # seed 1's last found hit dropped (a miss where the truth track has a hit)
    tr["hit"][1, plen[1] - 1] = -1
    v = bench.validation(b, tr, plen, plan, ok)
    assert abs(v["hit_selection_accuracy"] - (total - 2) / total) < 1e-12
    assert abs(v["hit_purity"] - (total - 2) / (total - 1)) < 1e-12

"""The benchmark's command-line contract on the CPU (no GPU work): more than
one GPU is refused with a JSON message and exit status 2; the counter data
committed under profiles/ are reported only for the sources they describe."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]



def test_traffic_counters_are_used_only_for_the_sources_they_describe():
    """bench.py reports the committed HBM byte counters only while their
    source hash matches the headline kernel's current sources."""
    sys.path.insert(0, str(ROOT))
    import bench
    f = ROOT / bench.HEADLINE_COUNTERS
    expected = None
    if f.exists():
        d = json.loads(f.read_text())
        if d["source_hash"] == bench.kernel_source_hash():
            expected = d.get("traffic_bytes_per_launch")
    assert bench.measured_traffic() == expected


def test_valu_issue_floor_follows_the_counters(monkeypatch):
    """The VALU issue floor is SQ_INSTS_VALU per wave x 4 cycles x waves over
    1024 SIMDs at 2.4 GHz, reported only for the sources the counters
    describe."""
    sys.path.insert(0, str(ROOT))
    import bench
    d = {"source_hash": "x", "traffic_bytes_per_launch": 1.0, "valu_instr_per_wave": 1000.0,
         "waves_per_launch": 2048.0}
    monkeypatch.setattr(bench, "_committed_counters", lambda *a, **k: d)
    v = bench.valu_issue(0.01)
    floor_ms = 1000.0 * 4 * 2048.0 / 1024 / 2.4e9 * 1e3
    assert abs(v["issue_floor_ms"] - floor_ms) < 1e-15 and abs(v["frac"] - floor_ms / 0.01) < 1e-12
    monkeypatch.setattr(bench, "_committed_counters", lambda *a, **k: None)
    assert bench.valu_issue(0.01) is None and bench.measured_traffic() is None

"""Host-side parts of the benchmark contract (no GPU needed): one GPU only,
and the counter-derived traffic record is read only for unchanged sources."""
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


def test_traffic_record_requires_matching_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    from paper_1804_01918_amd.profsummary import PLAIN_SOURCES, source_digest
    rec = {"kernels": {"k": {"sites": 10, "hbm_bytes_per_launch": 123.0, "source_files": list(PLAIN_SOURCES),
                             "source_digest": source_digest(PLAIN_SOURCES)},
                       "stale": {"sites": 10, "hbm_bytes_per_launch": 1.0, "source_files": list(PLAIN_SOURCES),
                                 "source_digest": "0" * 16}}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(path))
    assert bench.traffic_entry("k", 10) == 123.0
    assert bench.traffic_entry("k", 11) is None        # other workload size
    assert bench.traffic_entry("stale", 10) is None    # sources changed since the counters
    assert bench.traffic_entry("missing", 10) is None

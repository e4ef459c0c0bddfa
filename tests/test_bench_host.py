"""Host logic of bench.py that needs no GPU: the rocprof record lookup
(kernel names carry template arguments; a record of other kernel sources is
ignored) and the CLI refusing more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_load_profile_matches_template_names(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"source_hash": "ab" * 8,
           "kernels": {"k_decode_split<8>": {"avg_us": 1.0}, "k_decode<8>": {"avg_us": 160.0},
                       "k_encode<8>": {"avg_us": 140.0}}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "ab" * 8)
    assert bench.load_profile("k_decode") == {"avg_us": 160.0}
    assert bench.load_profile("k_decode_split") == {"avg_us": 1.0}
    assert bench.load_profile("k_histogram") == {}
    rec["source_hash"] = "0" * 16                     # kernels changed since: ignored
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert bench.load_profile("k_decode") == {}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)

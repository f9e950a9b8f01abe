"""Host logic of the benchmark (CPU): the counter traffic of a kernel is reported only while the
source it was measured on is unchanged."""
import hashlib
import json
import os

import bench


def test_committed_traffic_follows_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1")
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"source": "k.hip", "source_sha256": hashlib.sha256(b"kernel v1").hexdigest(), "traffic_bytes": 123.0}
    (prof / "traffic.json").write_text(json.dumps({"kern": entry}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_traffic("kern") == 123.0
    src.write_text("kernel v2")
    assert bench.committed_traffic("kern") is None
    assert bench.committed_traffic("other") is None


def test_gpus_other_than_one_exit_with_message():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

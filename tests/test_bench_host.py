"""Host logic of bench.py (no GPU): the one-GPU refusal and the rule that an
HBM traffic figure is reported only when the committed counter summary was
taken on the current kernel sources."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in (res.stdout + res.stderr)


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1801_06263_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("// kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench.source_hash()
    assert len(h1) == 16
    (tmp_path / "profiles").mkdir()
    rec = {"large": {"k_back_primal": {"bytes_per_launch": 123456, "source_hash": h1}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("k_back_primal", "large") == 123456
    assert bench.measured_traffic("k_forward<3>", "large") is None     # not measured
    assert bench.measured_traffic("k_back_primal", "medium") is None   # other workload
    (csrc / "k.hip").write_text("// kernel v2\n")                      # the sources changed since
    assert bench.source_hash() != h1
    assert bench.measured_traffic("k_back_primal", "large") is None
    (tmp_path / "profiles" / "traffic.json").write_text("not json")
    assert bench.measured_traffic("k_back_primal", "large") is None

"""Host logic of bench.py (no GPU): the one-GPU refusal and the rule that
counter figures from the committed profile are used only for the sources
they were taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _profile(path, sha, traffic="4.5e+08", issue="0.8", lane="0.5"):
    path.write_text(f"# k_match\n\ntraffic_bytes_per_launch: {traffic}\nvalu_issue_frac: {issue}\n"
                    f"valu_lane_frac: {lane}\nsource_sha256: {sha}\n")


def test_profile_figures_only_for_the_current_sources(tmp_path, monkeypatch):
    p = tmp_path / "k_match.md"
    monkeypatch.setattr(bench, "PROFILE", str(p))
    assert bench.profiled_traffic() is None          # no profile
    _profile(p, bench.source_hash())
    assert bench.profiled_traffic() == 4.5e8
    v = bench.profiled_valu()
    assert v["issue_frac"] == 0.8 and v["lane_frac"] == 0.5
    _profile(p, "0" * 64)                             # taken on other sources
    assert bench.profiled_traffic() is None and bench.profiled_valu() is None
    p.write_text("traffic_bytes_per_launch: 4.5e+08\n")  # no hash at all
    assert bench.profiled_traffic() is None

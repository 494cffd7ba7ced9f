"""Host-side checks of bench.py's contract: one GPU only, and the committed
counter summary is used only while the kernel sources it describes are
unchanged."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_values_follow_the_source_hash(tmp_path, monkeypatch):
    vals = bench.profile_values()
    if vals:   # the committed summary matches the sources
        assert vals["traffic"] > 0 and 0 < vals["valu_lane_utilisation"] <= 1
        assert 0 < vals["l2_hit_rate"] <= 1
    # a summary whose hash does not match the sources is ignored
    fake = tmp_path / "p.md"
    fake.write_text("traffic_bytes_per_launch: 123\nvalu_lane_utilisation: 0.5\n"
                    "l2_hit_rate: 0.5\nsource_hash: 0000000000000000\n")
    monkeypatch.setattr(bench, "PROFILE", str(fake))
    assert bench.profile_values() == {}

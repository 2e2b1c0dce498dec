"""Host-side checks of bench.py: the one-GPU contract and the staleness rule
of the committed HBM-traffic figure (no device needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_figure_follows_the_measured_sources(tmp_path, monkeypatch):
    import bench
    # the committed counter summary was taken with the step kernel's current sources
    assert bench._measured_traffic() is not None
    # a summary recorded for other sources gives no figure
    txt = open(bench.TRAFFIC_PROFILE).read()
    stale = tmp_path / "traffic.txt"
    stale.write_text(txt.replace(bench.step_sources_sha(), "0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench._measured_traffic() is None
    # and a missing one none either
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "absent.txt"))
    assert bench._measured_traffic() is None

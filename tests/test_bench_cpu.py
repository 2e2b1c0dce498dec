"""Host-side checks of bench.py: the one-GPU contract, the staleness rule
of the committed HBM-traffic figure, and that the commands the committed
profiles record still parse (no device needed)."""
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


def test_profile_commands_parse():
    """Every bench.py command recorded in profiles/ parses with the current
    command line, so each committed summary can be taken again from committed
    files."""
    import glob
    import shlex
    sys.path.insert(0, ROOT)
    import bench
    ap = bench.make_parser()
    seen = 0
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        for line in open(path):
            if "<repo>/bench.py" not in line:
                continue
            args = shlex.split(line.split("<repo>/bench.py", 1)[1])
            try:
                _, extra = ap.parse_known_args(args)
            except SystemExit:
                raise AssertionError(f"{os.path.basename(path)}: bench.py rejects {args}")
            assert not extra, (os.path.basename(path), extra)
            seen += 1
    assert seen >= 10, seen

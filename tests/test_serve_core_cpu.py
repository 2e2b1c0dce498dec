"""The server's scheduling core (continuous batching, admission by device
budget, percentiles) compiled with g++ and run on the host."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serve_core(tmp_path):
    exe = tmp_path / "test_serve_core"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-pthread", os.path.join(HERE, "cpp", "test_serve_core.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "serve core ok" in r.stdout

"""The autotuner's JSON-lines cache (keys, lookup, override, damaged lines)
compiled with g++ and run on the host."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tune_cache(tmp_path):
    exe = tmp_path / "test_tune_cache"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", os.path.join(HERE, "cpp", "test_tune_cache.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe), str(tmp_path / "tune.jsonl")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "tune cache ok" in r.stdout

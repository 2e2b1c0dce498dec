"""The autotuner's JSON-lines cache (keys, lookup, override, damaged lines)
compiled with g++ and run on the host: as built, and under AddressSanitizer
with UndefinedBehaviorSanitizer."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "test_tune_cache.cpp")
BUILDS = {
    "plain": ["-O1", "-Wall"],
    "asan_ubsan": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=all"],
}


@pytest.mark.parametrize("build", sorted(BUILDS))
def test_tune_cache(tmp_path, build):
    exe = tmp_path / f"test_tune_cache_{build}"
    subprocess.run(["g++", "-std=c++17", *BUILDS[build], SRC, "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0")
    r = subprocess.run([str(exe), str(tmp_path / "tune.jsonl")], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "tune cache ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr

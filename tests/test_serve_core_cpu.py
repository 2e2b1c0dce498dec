"""The server's scheduling core (continuous batching, admission by device
budget, percentiles, concurrent producers and workers) compiled with g++ and
run on the host: as built, and under AddressSanitizer with
UndefinedBehaviorSanitizer and under ThreadSanitizer."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "test_serve_core.cpp")
BUILDS = {
    "plain": ["-O1", "-Wall"],
    "asan_ubsan": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                   "-fno-sanitize-recover=all"],
    "tsan": ["-O1", "-g", "-fsanitize=thread"],
}


@pytest.mark.parametrize("build", sorted(BUILDS))
def test_serve_core(tmp_path, build):
    exe = tmp_path / f"test_serve_core_{build}"
    subprocess.run(["g++", "-std=c++17", *BUILDS[build], "-pthread", SRC, "-o", str(exe)], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "serve core ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr

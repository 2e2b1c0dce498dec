import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The GPU tests run with the hardware queue count that bench.py sets, so that
# campaigns overlap on the device as they do when timed (read by the HIP
# runtime when it starts, before any test touches the device).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 18:
    os.environ["GPU_MAX_HW_QUEUES"] = "18"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")

import os
import sys

# The serving tests run up to five streams of their own (query slots and the
# labeling stream) beside torch's; with fewer hardware queues than streams,
# HIP maps several streams onto one queue and their work cannot overlap.
# Set before anything initialises HIP.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")

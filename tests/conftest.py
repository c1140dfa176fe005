"""Shared pytest configuration.

Markers: ``gpu`` for tests that need an MI355X (HIP device) and the built
library; everything else runs on the CPU.
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle checks")

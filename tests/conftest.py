import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: oracle runs of more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # keep GPU tests after the CPU tests so a GPU failure under -x hides nothing on the CPU
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    config.addinivalue_line("markers", "early: runs before the other tests of the session (it starts worker "
                                       "processes, which it must do before this process first uses the GPU)")


def pytest_collection_modifyitems(config, items):
    items.sort(key=lambda it: 0 if it.get_closest_marker("early") else 1)   # stable: the rest keep their order

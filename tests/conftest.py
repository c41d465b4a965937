import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


def pytest_collection_modifyitems(config, items):
    # order: CPU pins first, then GPU parity tests; the no-allocation entry point last
    def key(item):
        name = item.nodeid
        if "test_zz_" in name:
            return 2
        return 1 if item.get_closest_marker("gpu") else 0

    items.sort(key=key)

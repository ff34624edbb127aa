import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle checks")


def pytest_collection_modifyitems(config, items):
    # Run GPU parity tests in file order but keep any no-alloc check last.
    items.sort(key=lambda it: 1 if "test_zz_" in it.nodeid else 0)

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workload, minutes of CPU or GPU time")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in one process on the box; nothing here skips them silently: a GPU test
    # that runs where no GPU is visible fails loudly in its fixture instead.
    pass

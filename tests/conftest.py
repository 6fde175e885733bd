import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def pytest_collection_modifyitems(config, items):
    # run GPU tests in a stable order: library smoke tests first, full-size cases last
    order = {"test_gpu_basic": 0, "test_gpu_parity": 1, "test_gpu_solve": 2, "test_gpu_batched": 3,
             "test_gpu_adjoint": 4, "test_gpu_fullsize": 5}
    items.sort(key=lambda it: order.get(it.module.__name__.split(".")[-1], -1))

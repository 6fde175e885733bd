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
    # (the allocation-free entry point's test, test_zz_*, always runs last)
    order = {"test_gpu_basic": 0, "test_gpu_parity": 1, "test_gpu_solve": 2, "test_gpu_batched": 3,
             "test_gpu_adjoint": 4, "test_gpu_fullsize": 5}

    def key(it):
        name = it.module.__name__.split(".")[-1]
        return 99 if name.startswith("test_zz_") else order.get(name, -1)
    items.sort(key=key)

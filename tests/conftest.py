import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than a few seconds")


if os.environ.get("PYTEST_XDIST_WORKER"):
    # parallel workers share the CPUs: one BLAS and one OpenMP thread each
    # (the oracle's OpenMP runtime reads the variable when it loads, after
    # this file), else the workers oversubscribe the cores and spin
    os.environ["OMP_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits
    _BLAS_LIMIT = threadpool_limits(1)

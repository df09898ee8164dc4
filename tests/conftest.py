import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _ensure_built():
    import lfsynth
    import oracle
    if not os.path.exists(lfsynth._SO):
        lfsynth.build()
    if not os.path.exists(oracle._SO):
        oracle.build()


_ensure_built()


@pytest.fixture(scope="session")
def tiny():
    """The 64-view tiny workload (128^2 views, 128^2 depth, 256^2 mono eye)."""
    import lfsynth
    return lfsynth.make_workload("tiny", seed=0)


@pytest.fixture(scope="session")
def tiny_oracle(tiny):
    import oracle
    return oracle.OracleViews.from_views(tiny.views)


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(1234)

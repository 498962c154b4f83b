import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle


def f32_params(params: dict) -> dict:
    """The parameter dict with every real rounded to binary32, i.e. exactly
    the values the GPU library receives, so the oracle sees the same inputs."""
    import numpy as np

    def r(v):
        if isinstance(v, float):
            return float(np.float32(v))
        if isinstance(v, (list, tuple)):
            return [r(x) for x in v]
        return v
    return {k: r(v) for k, v in params.items()}


def pytest_sessionstart(session):
    # the oracle's per-sample loops run on the host's cores (the results do
    # not depend on the thread count)
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    oracle.set_threads(min(os.cpu_count() or 1, 16))

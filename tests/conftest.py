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


# Position-error budget of the FP32 rollout (metres per coordinate of a shape
# point): positions of <= 10 m in the iteration's local frame have an ulp of
# ~1e-6 m, and <= 100 Euler steps accumulate ~1e-5 m.  The oracle's barrier
# sensitivity is taken over moves of this reach, and the cost tolerance adds
# reach x sensitivity to the relative bound.
SENS_REACH = 1e-5


def f32_params(params: dict) -> dict:
    """The parameter dict with every real rounded to binary32, i.e. exactly
    the values the GPU library receives, so the oracle sees the same inputs;
    plus the reach of the oracle's barrier sensitivity (an oracle-only
    diagnostic the library never sees)."""
    import numpy as np

    def r(v):
        if isinstance(v, float):
            return float(np.float32(v))
        if isinstance(v, (list, tuple)):
            return [r(x) for x in v]
        return v
    out = {k: r(v) for k, v in params.items()}
    out["sens_reach"] = SENS_REACH
    return out


def pytest_sessionstart(session):
    # the oracle's per-sample loops run on the host's cores (the results do
    # not depend on the thread count)
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    oracle.set_threads(min(os.cpu_count() or 1, 16))

"""MI355X-native DBaS-Log-MPPI: one controller iteration (normal x log-normal
Philox sampling, barrier-state-augmented rollout, min-shifted exponential
weighting and weighted-average update) as HIP kernels behind a C ABI.

Importing the package loads nothing; ``controller`` loads libdbasmppi.so on
first use and raises if it is missing.
"""
__all__ = ["Controller", "Batch", "Server", "workloads"]


def __getattr__(name):
    if name in ("Controller", "Batch"):
        from . import controller
        return getattr(controller, name)
    if name == "Server":
        from . import server
        return server.Server
    raise AttributeError(name)

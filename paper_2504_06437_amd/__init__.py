"""MI355X-native DBaS-Log-MPPI: one controller iteration (normal x log-normal
Philox sampling, barrier-state-augmented rollout, min-shifted exponential
weighting and weighted-average update) as HIP kernels behind a C ABI.

Importing the package loads nothing; the handle classes (Controller, Batch,
Server, all in ``controller``) load libdbasmppi.so on first use and raise if
it is missing.
"""
__all__ = ["Controller", "Batch", "Server", "workloads"]


def __getattr__(name):
    import importlib
    if name in ("Controller", "Batch", "Server"):
        return getattr(importlib.import_module(__name__ + ".controller"), name)
    if name == "workloads":
        return importlib.import_module(__name__ + ".workloads")
    raise AttributeError(name)

"""Device buffers and events through the HIP runtime the library itself links
(plumbing for callers that want to pass device pointers; no computation).

torch wheels bundle a HIP runtime of their own; two runtimes in one process do
not share devices, so this module talks to the library's runtime directly.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as A

_H2D, _D2H, _D2D = 1, 2, 3
_hip = None


def runtime():
    global _hip
    if _hip is None:
        A.load()                                   # resolves libamdhip64 first
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        h.hipFree.argtypes = [ctypes.c_void_p]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipDeviceSynchronize.argtypes = []
        h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        h.hipEventDestroy.argtypes = [ctypes.c_void_p]
        h.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        h.hipGetErrorString.restype = ctypes.c_char_p
        h.hipGetErrorString.argtypes = [ctypes.c_int]
        _hip = h
    return _hip


def _ok(e: int, what: str):
    if e != 0:
        raise RuntimeError(f"{what}: {runtime().hipGetErrorString(e).decode()}")


def synchronize():
    _ok(runtime().hipDeviceSynchronize(), "hipDeviceSynchronize")


def copy_device(dst: "DeviceArray", src: "DeviceArray"):
    """Device-to-device copy of a whole array (the runtime's blit kernel)."""
    assert dst.nbytes == src.nbytes
    _ok(runtime().hipMemcpy(ctypes.c_void_p(dst.ptr), ctypes.c_void_p(src.ptr), src.nbytes, _D2D), "hipMemcpy D2D")


class DeviceArray:
    """A float32 (or any dtype) array in device memory."""

    def __init__(self, shape, dtype=np.float32):
        self.shape = tuple(np.atleast_1d(shape)) if not isinstance(shape, tuple) else shape
        self.dtype = np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        p = ctypes.c_void_p()
        _ok(runtime().hipMalloc(ctypes.byref(p), max(self.nbytes, 16)), "hipMalloc")
        self.ptr = p.value

    @classmethod
    def from_numpy(cls, a):
        a = np.ascontiguousarray(a)
        d = cls(a.shape, a.dtype)
        d.upload(a)
        return d

    def upload(self, a):
        a = np.ascontiguousarray(a, dtype=self.dtype)
        assert a.nbytes == self.nbytes
        _ok(runtime().hipMemcpy(ctypes.c_void_p(self.ptr), a.ctypes.data, self.nbytes, _H2D), "hipMemcpy H2D")

    def numpy(self):
        out = np.empty(self.shape, dtype=self.dtype)
        _ok(runtime().hipMemcpy(out.ctypes.data, ctypes.c_void_p(self.ptr), self.nbytes, _D2H), "hipMemcpy D2H")
        return out

    def at(self, index: int) -> int:
        """Device address of row `index` (first axis)."""
        row = self.nbytes // self.shape[0]
        return self.ptr + index * row

    def free(self):
        if self.ptr:
            runtime().hipFree(ctypes.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Event:
    def __init__(self):
        e = ctypes.c_void_p()
        _ok(runtime().hipEventCreate(ctypes.byref(e)), "hipEventCreate")
        self.e = e

    def record(self, stream: int = 0):
        _ok(runtime().hipEventRecord(self.e, ctypes.c_void_p(stream) if stream else None), "hipEventRecord")

    def synchronize(self):
        _ok(runtime().hipEventSynchronize(self.e), "hipEventSynchronize")

    def elapsed_ms(self, end: "Event") -> float:
        ms = ctypes.c_float()
        _ok(runtime().hipEventElapsedTime(ctypes.byref(ms), self.e, end.e), "hipEventElapsedTime")
        return ms.value

    def __del__(self):
        try:
            runtime().hipEventDestroy(self.e)
        except Exception:
            pass

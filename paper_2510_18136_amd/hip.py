"""Device memory, copies and events through the HIP runtime libnsfrb.so links.

Plumbing for callers that do not want PyTorch in the process: every ROCm user
in one process shares the first HIP runtime loaded, and a PyTorch wheel
bundles its own (older) one. On gfx950 that runtime keeps fewer of this
library's large-LDS workgroups resident per CU (the FP16 search runs 1.9x
slower, the FP32 search 1.4x), so timing runs use this module instead of
torch. All calls use the default stream unless given one.
"""
import ctypes

import numpy as np

from . import nsfrb

_hip = None


def lib():
    """The HIP runtime of libnsfrb.so (loaded by it, so the same instance)."""
    global _hip
    if _hip is None:
        nsfrb.lib()                                   # loads libamdhip64 as libnsfrb's dependency
        L = ctypes.CDLL("libamdhip64.so.7")
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.hipMalloc.argtypes = [ctypes.POINTER(vp), sz]
        L.hipFree.argtypes = [vp]
        L.hipMemcpy.argtypes = [vp, vp, sz, ctypes.c_int]
        L.hipMemset.argtypes = [vp, ctypes.c_int, sz]
        L.hipEventCreate.argtypes = [ctypes.POINTER(vp)]
        L.hipEventRecord.argtypes = [vp, vp]
        L.hipEventSynchronize.argtypes = [vp]
        L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), vp, vp]
        L.hipEventDestroy.argtypes = [vp]
        L.hipGetDeviceCount.argtypes = [ctypes.POINTER(ctypes.c_int)]
        L.hipGetErrorString.restype = ctypes.c_char_p
        for f in ("hipMalloc", "hipFree", "hipMemcpy", "hipMemset", "hipDeviceSynchronize", "hipEventCreate",
                  "hipEventRecord", "hipEventSynchronize", "hipEventElapsedTime", "hipEventDestroy",
                  "hipGetDeviceCount"):
            getattr(L, f).restype = ctypes.c_int
        _hip = L
    return _hip


def check(err, what):
    if err != 0:
        raise RuntimeError(f"{what}: {lib().hipGetErrorString(err).decode()}")


def device_count():
    n = ctypes.c_int(0)
    return n.value if lib().hipGetDeviceCount(ctypes.byref(n)) == 0 else 0


class Buffer:
    """nbytes of device memory (hipMalloc), freed on close()."""

    def __init__(self, nbytes):
        self.nbytes = int(nbytes)
        p = ctypes.c_void_p()
        check(lib().hipMalloc(ctypes.byref(p), max(1, self.nbytes)), f"hipMalloc({self.nbytes})")
        self.ptr = int(p.value)

    def upload(self, arr):
        a = np.ascontiguousarray(arr)
        assert a.nbytes <= self.nbytes
        check(lib().hipMemcpy(ctypes.c_void_p(self.ptr), a.ctypes.data_as(ctypes.c_void_p), a.nbytes, 1),
              "hipMemcpy H2D")
        return self

    def download(self, dtype, count):
        out = np.empty(count, dtype=dtype)
        check(lib().hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(self.ptr), out.nbytes, 2),
              "hipMemcpy D2H")
        return out

    def zero(self):
        check(lib().hipMemset(ctypes.c_void_p(self.ptr), 0, self.nbytes), "hipMemset")
        return self

    def close(self):
        if self.ptr:
            lib().hipFree(ctypes.c_void_p(self.ptr))
            self.ptr = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def synchronize():
    check(lib().hipDeviceSynchronize(), "hipDeviceSynchronize")


class Timer:
    """HIP events on a stream (default stream when 0): start(), stop() -> ms."""

    def __init__(self, stream=0):
        self.stream = ctypes.c_void_p(int(stream))
        self.e = [ctypes.c_void_p(), ctypes.c_void_p()]
        for e in self.e:
            check(lib().hipEventCreate(ctypes.byref(e)), "hipEventCreate")

    def start(self):
        check(lib().hipEventRecord(self.e[0], self.stream), "hipEventRecord")

    def stop(self):
        check(lib().hipEventRecord(self.e[1], self.stream), "hipEventRecord")
        check(lib().hipEventSynchronize(self.e[1]), "hipEventSynchronize")
        ms = ctypes.c_float()
        check(lib().hipEventElapsedTime(ctypes.byref(ms), self.e[0], self.e[1]), "hipEventElapsedTime")
        return ms.value

    def close(self):
        for e in self.e:
            if e:
                lib().hipEventDestroy(e)
        self.e = [None, None]

"""Device-memory plumbing for GPU tests: hipMalloc / hipMemcpy / hipFree from the system HIP runtime.

The library links /opt/rocm's libamdhip64; PyTorch wheels bundle a different HIP runtime, and two
runtimes in one process do not share devices, so tests allocate through the same runtime as the
library instead of through torch.
"""
import ctypes

import numpy as np

_rt = None


def rt():
    global _rt
    if _rt is None:
        _rt = ctypes.CDLL("/opt/rocm/lib/libamdhip64.so")
    return _rt


class DeviceArray:
    def __init__(self, host):
        host = np.ascontiguousarray(host)
        self.nbytes = host.nbytes
        self.ptr = ctypes.c_void_p()
        assert rt().hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(self.nbytes)) == 0
        assert rt().hipMemcpy(self.ptr, ctypes.c_void_p(host.ctypes.data), ctypes.c_size_t(self.nbytes), 1) == 0

    @property
    def address(self):
        return self.ptr.value

    def free(self):
        if self.ptr:
            rt().hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()

"""Helpers for the GPU tests: load libsv or skip when no HIP device is present."""
import os

import pytest


def require_gpu():
    try:
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        cnt = ctypes.c_int(0)
        if hip.hipGetDeviceCount(ctypes.byref(cnt)) != 0 or cnt.value < 1:
            pytest.skip("no HIP device")
    except OSError:
        pytest.skip("no HIP runtime")
    from paper_2606_12770_amd import sv
    sv.load_library()  # raises if the library was not built: never a silent fallback
    return sv

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


def max_rel_err(got, want):
    """Largest amplitude error relative to the largest reference amplitude."""
    import numpy as np
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


# Element-wise bar for complex64 against the FP64 oracle: every amplitude
# within 1e-5 of the largest one per 1,000 gates applied (at least 1e-5).
# Each gate rounds the amplitudes it touches to about 2^-24 relative and its
# parameters are rounded once; lowered circuits add uncontrolled rotation
# pairs that cancel only up to that rounding, so the error grows with the
# gate count.  One wrong amplitude of a typical size is off by about its own
# magnitude, far above the bar.
C64_REL = 1e-5


def c64_bar(n_ops=None):
    return C64_REL * max(1.0, (n_ops or 0) / 1000.0)


def assert_c64_close(got, want, n_ops=None, what=""):
    rel = c64_bar(n_ops)
    err = max_rel_err(got, want)
    print(f"{what} complex64 max |err| / max |want| = {err:.2e} (bar {rel:.1e}, {n_ops} ops)", flush=True)
    assert err < rel, f"{what}: complex64 amplitude error {err:.2e} above {rel:.1e}"

"""sv_amplitudes_noalloc through the C ABI against sv_amplitudes.

The variant stages the read-out through the library's fixed device array
instead of a per-call allocation; its results must be bit-identical to
sv_amplitudes (the same conversion kernel into a different buffer).  Two calls
in a row, the second with a smaller range (the array keeps the first call's
contents, which must not leak into the second result), both precisions, and
the refusals: a count above the array's 262144 amplitudes and a range outside
the state give SV_EINVAL and copy nothing.
"""
import ctypes

import numpy as np
import pytest

from paper_2606_12770_amd.circuits.random_circuit import random_state
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def noalloc(lib, h, offset, count, fill=np.nan):
    out = np.full(count, fill, dtype=np.complex128)
    rc = lib.sv_amplitudes_noalloc(h, offset, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return rc, out


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_readout_matches_sv_amplitudes(dtype):
    sv = require_gpu()
    lib = sv.load_library()
    n = 20
    psi = random_state(n, 31 + dtype)
    st = sv.State(n, dtype, psi)
    try:
        for offset, count in ((12345, 200000), (777, 1000)):
            want = sv.sv_amplitudes(st.h, offset, count)
            rc, got = noalloc(lib, st.h, offset, count)
            print(f"dtype={dtype} offset={offset} count={count}: rc {rc}", flush=True)
            assert rc == sv.SV_OK
            assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
        # the largest count the array holds, at the end of the state
        count = 1 << 18
        rc, got = noalloc(lib, st.h, (1 << n) - count, count)
        assert rc == sv.SV_OK
        assert np.array_equal(got.view(np.uint64), sv.sv_amplitudes(st.h, (1 << n) - count, count).view(np.uint64))
        # refusals: nothing copied
        for offset, count in ((0, (1 << 18) + 1), ((1 << n) - 10, 11)):
            rc, got = noalloc(lib, st.h, offset, count)
            assert rc == sv.SV_EINVAL
            assert np.all(np.isnan(got.real))
        assert "static staging buffer" in sv.sv_last_error() or "outside" in sv.sv_last_error()
    finally:
        st.close()

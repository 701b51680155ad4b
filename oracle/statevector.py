"""ctypes front end of the FP64 reference simulator in sv_oracle.c.

TEST INFRASTRUCTURE ONLY (see the package docstring).  States are numpy
complex128 arrays of length 2^n, index bit j = qubit j.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_apply.argtypes = [dp, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, dp]
        L.oracle_apply.restype = ctypes.c_int
        L.oracle_prob.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_prob.restype = ctypes.c_double
        L.oracle_postselect.argtypes = [dp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        L.oracle_postselect.restype = ctypes.c_double
        L.oracle_inner.argtypes = [dp, dp, ctypes.c_int, dp]
        L.oracle_inner.restype = None
        L.oracle_qsp_poly.argtypes = [dp, ctypes.c_uint64, dp, ctypes.c_uint64, dp]
        L.oracle_qsp_poly.restype = None
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply(psi: np.ndarray, n: int, ops: np.ndarray, params: np.ndarray) -> np.ndarray:
    """Apply the op records in place (psi must be contiguous complex128)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous and psi.size == 1 << n
    ops = np.ascontiguousarray(ops)
    params = np.ascontiguousarray(params, dtype=np.float64)
    rc = lib().oracle_apply(_dptr(psi), n, ops.ctypes.data, len(ops), _dptr(params))
    if rc != 0:
        raise ValueError("oracle: unknown op kind")
    return psi


def run(circuit, psi0: np.ndarray | None = None) -> np.ndarray:
    ops, params = circuit.arrays()
    psi = zero_state(circuit.n) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)
    return apply(psi, circuit.n, ops, params)


def prob(psi, n, mask=0, val=0) -> float:
    return lib().oracle_prob(_dptr(psi), n, mask, val)


def postselect(psi, n, mask, val, renormalize=True) -> float:
    return lib().oracle_postselect(_dptr(psi), n, mask, val, int(renormalize))


def inner(a, b, n) -> complex:
    out = np.zeros(2)
    lib().oracle_inner(_dptr(a), _dptr(b), n, _dptr(out))
    return complex(out[0], out[1])


def infidelity(a, b, n) -> float:
    """1 - |<a|b>|^2 / (<a|a><b|b>) in FP64."""
    ab = inner(a, b, n)
    return 1.0 - abs(ab) ** 2 / (prob(a, n) * prob(b, n))


def threads() -> int:
    return lib().oracle_threads()

"""Python binding of libsv (ctypes): the C entry points under the same names.

Argument marshalling only: every step runs in the HIP library.  The library
must have been built (``paper_2606_12770_amd.build``); importing this module
without it, or calling it on a machine without a HIP device, raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .circuits.ir import OP_DTYPE

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsv.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EZEROPROB, SV_EDEVICE, SV_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SV_C64, SV_C128 = 0, 1
SV_MODE_PLAIN, SV_MODE_FUSED = 0, 1
SV_TILE_LAUNCH_AUTO, SV_TILE_LAUNCH_GRID, SV_TILE_LAUNCH_PERSISTENT = 0, 1, 2
SV_PLAIN_SPLIT_AUTO, SV_PLAIN_SPLIT_OFF = 0, 1
SV_COMPILE_AUTO, SV_COMPILE_OFF, SV_COMPILE_ON = 0, 1, 2
SV_DENSE_AUTO = -1
SV_PEEPHOLE_AUTO, SV_PEEPHOLE_OFF, SV_PEEPHOLE_ON = 0, 1, 2
SV_SPLIT_REAL_AUTO, SV_SPLIT_REAL_OFF, SV_SPLIT_REAL_ON = 0, 1, 2

EXPORTED = [
    "sv_alloc", "sv_free", "sv_info", "sv_apply_circuit", "sv_plan_create", "sv_plan_free",
    "sv_plan_get_info", "sv_plan_execute", "sv_plan_execute_seq", "sv_plan_time", "sv_postselect",
    "sv_amplitudes", "sv_amplitudes_noalloc", "sv_set_amplitudes", "sv_copy", "sv_inner", "sv_strerror", "sv_last_error",
    "sv_alloc_batch", "sv_batch_create", "sv_batch_execute", "sv_batch_time", "sv_batch_levels", "sv_batch_free",
]


class SVError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsv error {code}: {msg}")
        self.code = code


class sv_apply_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tile_qubits", ctypes.c_int), ("reg_qubits", ctypes.c_int),
                ("dense_min_ops", ctypes.c_int), ("tile_launch", ctypes.c_int), ("plain_split", ctypes.c_int),
                ("compile", ctypes.c_int), ("dense_bf16", ctypes.c_int), ("peephole", ctypes.c_int),
                ("dense_qubits", ctypes.c_int), ("coalesce_qubits", ctypes.c_int), ("split_real", ctypes.c_int)]


class sv_plan_info(ctypes.Structure):
    _fields_ = [("n_ops", ctypes.c_uint64), ("n_launches", ctypes.c_uint64), ("n_tile_passes", ctypes.c_uint64),
                ("n_stages", ctypes.c_uint64), ("bytes_moved", ctypes.c_uint64), ("tile_pass_bytes", ctypes.c_uint64),
                ("tile_qubits", ctypes.c_int), ("reg_qubits", ctypes.c_int), ("n_dense_passes", ctypes.c_uint64),
                ("n_dense_ops", ctypes.c_uint64), ("n_split_ops", ctypes.c_uint64),
                ("n_compiled_kernels", ctypes.c_uint64), ("dense_min_ops", ctypes.c_int),
                ("n_cancelled_ops", ctypes.c_uint64), ("touched_bytes", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsv.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libsv.so not built ({path}); run paper_2606_12770_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    pvp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "sv_alloc": [ctypes.c_int, ctypes.c_int, dp, vp, pvp],
        "sv_free": [vp],
        "sv_info": [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
        "sv_apply_circuit": [vp, vp, ctypes.c_size_t, dp, ctypes.c_size_t, ctypes.POINTER(sv_apply_opts)],
        "sv_plan_create": [ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, dp, ctypes.c_size_t,
                           ctypes.POINTER(sv_apply_opts), pvp],
        "sv_plan_free": [vp],
        "sv_plan_get_info": [vp, ctypes.POINTER(sv_plan_info)],
        "sv_plan_execute": [vp, vp, ctypes.c_int],
        "sv_plan_execute_seq": [pvp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32), ctypes.c_size_t, vp],
        "sv_plan_time": [vp, vp, ctypes.c_int, dp],
        "sv_postselect": [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, dp],
        "sv_amplitudes": [vp, ctypes.c_uint64, ctypes.c_uint64, dp],
        "sv_amplitudes_noalloc": [vp, ctypes.c_uint64, ctypes.c_uint64, dp],
        "sv_set_amplitudes": [vp, ctypes.c_uint64, ctypes.c_uint64, dp],
        "sv_copy": [vp, vp],
        "sv_inner": [vp, vp, dp, dp],
        "sv_alloc_batch": [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, vp, pvp],
        "sv_batch_create": [pvp, pvp, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint64, pvp],
        "sv_batch_execute": [vp, ctypes.c_int],
        "sv_batch_time": [vp, ctypes.c_int, dp],
        "sv_batch_levels": [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
        "sv_batch_free": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.sv_strerror.argtypes = [ctypes.c_int]
    L.sv_strerror.restype = ctypes.c_char_p
    L.sv_last_error.argtypes = []
    L.sv_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != SV_OK:
        L = load_library()
        raise SVError(rc, f"{L.sv_strerror(rc).decode()}: {L.sv_last_error().decode()}")


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _opts(mode=SV_MODE_FUSED, tile_qubits=0, reg_qubits=0, dense_min_ops=0, tile_launch=0, plain_split=0, compile=0,
          dense_bf16=0, peephole=0, dense_qubits=0, coalesce_qubits=0, split_real=0):
    return sv_apply_opts(mode, tile_qubits, reg_qubits, dense_min_ops, tile_launch, plain_split, compile, dense_bf16,
                         peephole, dense_qubits, coalesce_qubits, split_real)


# ---- the C entry points under their own names -------------------------------

def sv_alloc(n_qubits: int, dtype: int = SV_C64, init: np.ndarray | None = None, stream=None):
    L = load_library()
    out = ctypes.c_void_p()
    buf = None
    if init is not None:
        buf = np.ascontiguousarray(init, dtype=np.complex128)
        if buf.size != 1 << n_qubits:
            raise ValueError("init must hold 2^n amplitudes")
    _check(L.sv_alloc(n_qubits, dtype, None if buf is None else _dp(buf), stream, ctypes.byref(out)))
    return out


def sv_free(state):
    _check(load_library().sv_free(state))


def sv_info(state):
    n, dt = ctypes.c_int(), ctypes.c_int()
    _check(load_library().sv_info(state, ctypes.byref(n), ctypes.byref(dt)))
    return n.value, dt.value


def _ops_params(ops, params):
    ops = np.ascontiguousarray(ops, dtype=OP_DTYPE)
    params = np.ascontiguousarray(params if params is not None and len(params) else [0.0], dtype=np.float64)
    return ops, params


def sv_apply_circuit(state, ops, params, mode=SV_MODE_FUSED, tile_qubits=0, reg_qubits=0, dense_min_ops=0,
                     tile_launch=0, plain_split=0, compile=0, peephole=0, dense_bf16=0, dense_qubits=0,
                     coalesce_qubits=0, split_real=0):
    ops, params = _ops_params(ops, params)
    o = _opts(mode, tile_qubits, reg_qubits, dense_min_ops, tile_launch, plain_split, compile, dense_bf16, peephole,
              dense_qubits, coalesce_qubits, split_real)
    _check(load_library().sv_apply_circuit(state, ops.ctypes.data, len(ops), _dp(params), len(params),
                                           ctypes.byref(o)))


def sv_plan_create(n_qubits, dtype, ops, params, mode=SV_MODE_FUSED, tile_qubits=0, reg_qubits=0, dense_min_ops=0,
                   tile_launch=0, plain_split=0, compile=0, dense_bf16=0, peephole=0, dense_qubits=0,
                   coalesce_qubits=0, split_real=0):
    ops, params = _ops_params(ops, params)
    o = _opts(mode, tile_qubits, reg_qubits, dense_min_ops, tile_launch, plain_split, compile, dense_bf16, peephole,
              dense_qubits, coalesce_qubits, split_real)
    out = ctypes.c_void_p()
    _check(load_library().sv_plan_create(n_qubits, dtype, ops.ctypes.data, len(ops), _dp(params), len(params),
                                         ctypes.byref(o), ctypes.byref(out)))
    return out


def sv_plan_free(plan):
    _check(load_library().sv_plan_free(plan))


def sv_plan_get_info(plan) -> dict:
    info = sv_plan_info()
    _check(load_library().sv_plan_get_info(plan, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in sv_plan_info._fields_}


def sv_plan_execute(plan, state, repeat: int = 1):
    _check(load_library().sv_plan_execute(plan, state, repeat))


def sv_plan_execute_seq(plans, seq, state):
    arr = (ctypes.c_void_p * len(plans))(*[p.value for p in plans])
    s = np.ascontiguousarray(seq, dtype=np.int32)
    _check(load_library().sv_plan_execute_seq(arr, len(plans), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              len(s), state))


def sv_plan_time(plan, state, repeat: int = 1) -> float:
    ms = ctypes.c_double()
    _check(load_library().sv_plan_time(plan, state, repeat, ctypes.byref(ms)))
    return ms.value


def sv_postselect(state, mask: int, value: int, keep: bool = True, renormalize: bool = True) -> float:
    p = ctypes.c_double()
    _check(load_library().sv_postselect(state, mask, value, int(keep), int(renormalize), ctypes.byref(p)))
    return p.value


def sv_amplitudes(state, offset: int = 0, count: int | None = None) -> np.ndarray:
    n, _ = sv_info(state)
    if count is None:
        count = (1 << n) - offset
    out = np.empty(count, dtype=np.complex128)
    _check(load_library().sv_amplitudes(state, offset, count, _dp(out)))
    return out


def sv_amplitudes_noalloc(state, offset: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.complex128)
    _check(load_library().sv_amplitudes_noalloc(state, offset, count, _dp(out)))
    return out


def sv_set_amplitudes(state, values: np.ndarray, offset: int = 0):
    v = np.ascontiguousarray(values, dtype=np.complex128)
    _check(load_library().sv_set_amplitudes(state, offset, v.size, _dp(v)))


def sv_copy(dst, src):
    _check(load_library().sv_copy(dst, src))


def sv_inner(a, b) -> complex:
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(load_library().sv_inner(a, b, ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


def sv_alloc_batch(n_qubits, dtype: int = SV_C64, stream=None):
    """States of the given qubit counts in one device arena; returns their handles."""
    n = len(n_qubits)
    arr = (ctypes.c_int * n)(*[int(q) for q in n_qubits])
    out = (ctypes.c_void_p * n)()
    _check(load_library().sv_alloc_batch(n, arr, dtype, stream, out))
    return [ctypes.c_void_p(out[i]) for i in range(n)]


def sv_batch_create(states, plans, use_graph: bool = True, group_bytes: int = 0):
    n = len(states)
    if len(plans) != n:
        raise ValueError("one plan per state")
    sa = (ctypes.c_void_p * n)(*[s.value for s in states])
    pa = (ctypes.c_void_p * n)(*[p.value for p in plans])
    out = ctypes.c_void_p()
    _check(load_library().sv_batch_create(sa, pa, n, int(use_graph), group_bytes, ctypes.byref(out)))
    return out


def sv_batch_execute(batch, repeat: int = 1):
    _check(load_library().sv_batch_execute(batch, repeat))


def sv_batch_time(batch, repeat: int = 1) -> float:
    ms = ctypes.c_double()
    _check(load_library().sv_batch_time(batch, repeat, ctypes.byref(ms)))
    return ms.value


def sv_batch_levels(batch):
    """(launches, groups, gates) of one execution."""
    lv, gr, g = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(load_library().sv_batch_levels(batch, ctypes.byref(lv), ctypes.byref(gr), ctypes.byref(g)))
    return lv.value, gr.value, g.value


def sv_batch_free(batch):
    _check(load_library().sv_batch_free(batch))


def sv_strerror(code: int) -> str:
    return load_library().sv_strerror(code).decode()


def sv_last_error() -> str:
    return load_library().sv_last_error().decode()


# ---- convenience ------------------------------------------------------------

class State:
    """Owning handle around sv_alloc / sv_free."""

    def __init__(self, n_qubits: int, dtype: int = SV_C64, init=None):
        self.n = n_qubits
        self.dtype = dtype
        self.h = sv_alloc(n_qubits, dtype, init)

    def close(self):
        if self.h is not None:
            sv_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, circuit, mode=SV_MODE_FUSED, tile_qubits=0, reg_qubits=0, compile=0):
        ops, params = circuit.arrays()
        sv_apply_circuit(self.h, ops, params, mode, tile_qubits, reg_qubits, compile=compile)
        return self

    def amplitudes(self):
        return sv_amplitudes(self.h)

    def prob(self, mask=0, value=0):
        return sv_postselect(self.h, mask, value, keep=False, renormalize=False)

    def postselect(self, mask, value, renormalize=True):
        return sv_postselect(self.h, mask, value, keep=True, renormalize=renormalize)


class Plan:
    def __init__(self, n_qubits, dtype, circuit, mode=SV_MODE_FUSED, tile_qubits=0, reg_qubits=0, compile=0):
        ops, params = circuit.arrays()
        self.h = sv_plan_create(n_qubits, dtype, ops, params, mode, tile_qubits, reg_qubits, compile=compile)

    @property
    def info(self):
        return sv_plan_get_info(self.h)

    def execute(self, state: State, repeat=1):
        sv_plan_execute(self.h, state.h, repeat)

    def time(self, state: State, repeat=1) -> float:
        return sv_plan_time(self.h, state.h, repeat)

    def close(self):
        if self.h is not None:
            sv_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

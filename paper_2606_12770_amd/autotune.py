"""Autotuner for the fused tile geometry (resident qubits b, register qubits RB).

The candidates are planned through the C ABI and timed on the device with HIP
events (sv_plan_time / sv_batch_time) on the caller's states, whose contents
the timing runs overwrite: tune before loading the real input.  The fastest
geometry is cached per (circuit digest, qubits, precision), so repeated
circuits (the QSVT ladder of a configuration, the same batch) are tuned once
per process.
"""
from __future__ import annotations

import hashlib

from . import sv

CANDIDATES = ((12, 4), (11, 4), (10, 4), (12, 5), (13, 5), (13, 4))

_cache: dict = {}


def circuit_digest(circuits) -> str:
    h = hashlib.sha1()
    for c in circuits:
        ops, params = c.arrays()
        h.update(str(c.n).encode())
        h.update(ops.tobytes())
        h.update(params.tobytes())
    return h.hexdigest()


def _valid(n, b, rb, compiled=False):
    """Tiles of 512 threads (b - rb = 9) run only as compiled passes."""
    return b <= n and 6 <= b - rb <= (9 if compiled else 8)


def _compiled(n, compile):
    """Whether plans under this compile mode may compile (automatic mode
    compiles 512-thread tiles at any size)."""
    return compile != sv.SV_COMPILE_OFF


def tune_plan(circuit, state, dtype, candidates=CANDIDATES, repeat=1, compile=0):
    """Fastest (b, rb) for one circuit on one state; returns ((b, rb), {geometry: ms})."""
    key = ("plan", circuit_digest([circuit]), circuit.n, dtype, compile)
    if key in _cache:
        return _cache[key]
    ops, params = circuit.arrays()
    times = {}
    for b, rb in candidates:
        if not _valid(circuit.n, b, rb, _compiled(circuit.n, compile)):
            continue
        p = sv.sv_plan_create(circuit.n, dtype, ops, params, sv.SV_MODE_FUSED, b, rb, compile=compile)
        try:
            sv.sv_plan_execute(p, state, 1)
            times[(b, rb)] = sv.sv_plan_time(p, state, repeat) / repeat
        finally:
            sv.sv_plan_free(p)
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return _cache[key]


def tune_batch(circuits, states, dtype, candidates=CANDIDATES, repeat=1, use_graph=True):
    """Fastest common (b, rb) for a level-synchronous batch of generic-kernel
    plans (states from one arena); returns ((b, rb), {geometry: ms})."""
    key = ("batch", circuit_digest(circuits), dtype)
    if key in _cache:
        return _cache[key]
    arrays = [c.arrays() for c in circuits]
    nmin = min(c.n for c in circuits)
    times = {}
    for b, rb in candidates:
        if not _valid(nmin, b, rb):
            continue
        plans = [sv.sv_plan_create(c.n, dtype, o, p, sv.SV_MODE_FUSED, b, rb, plain_split=sv.SV_PLAIN_SPLIT_OFF,
                                   compile=sv.SV_COMPILE_OFF)
                 for c, (o, p) in zip(circuits, arrays)]
        batch = None
        try:
            batch = sv.sv_batch_create(states, plans, use_graph, 0)
            sv.sv_batch_execute(batch, 1)
            times[(b, rb)] = sv.sv_batch_time(batch, repeat) / repeat
        except sv.SVError:
            pass  # a geometry some instance cannot use (e.g. a per-gate step)
        finally:
            if batch is not None:
                sv.sv_batch_free(batch)
            for p in plans:
                sv.sv_plan_free(p)
    if not times:
        raise RuntimeError("no candidate geometry fits every instance of the batch")
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return _cache[key]


def tune_ladder(enc, dtype, proxy_degree=1001, candidates=CANDIDATES, compile=0):
    """Fastest (b, rb) for a QSVT ladder of the block encoding `enc`, timed on a
    proxy ladder of `proxy_degree` calls (the pass structure repeats every two
    calls, so a short ladder ranks the geometries as the full one does) on a
    scratch state.  Returns ((b, rb), {geometry: ms})."""
    import numpy as np
    from .circuits import carleman_circuit as cc
    n = enc.layout.n
    ops, params = cc.build_qsvt_arrays(enc, np.zeros(proxy_degree + 1))
    key = ("ladder", hashlib.sha1(ops.tobytes()).hexdigest(), n, dtype, compile)
    if key in _cache:
        return _cache[key]
    state = sv.sv_alloc(n, dtype)
    times = {}
    try:
        for b, rb in candidates:
            if not _valid(n, b, rb, _compiled(n, compile)):
                continue
            p = sv.sv_plan_create(n, dtype, ops, params, sv.SV_MODE_FUSED, b, rb, compile=compile)
            try:
                sv.sv_plan_execute(p, state, 1)
                times[(b, rb)] = sv.sv_plan_time(p, state, 1)
            finally:
                sv.sv_plan_free(p)
    finally:
        sv.sv_free(state)
    best = min(times, key=times.get)
    _cache[key] = (best, times)
    return _cache[key]

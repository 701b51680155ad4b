"""Seeded random layered circuits for the gate-throughput workload.

Each layer: one Haar-random U(2) on every qubit, then ``n_mcx`` multi-controlled
X gates (control count uniform in [1, max_ctrl], distinct controls, target
drawn from the remaining qubits, all controls positive), then one cyclic +1 on
a contiguous register of ``inc_width`` qubits at a uniformly drawn base.

Haar U(2): QR decomposition of a 2x2 complex Gaussian matrix with the phases of
diag(R) moved into Q (Mezzadri, "How to generate random matrices from the
classical compact groups", 2007).
"""
from __future__ import annotations

import numpy as np

from .ir import Circuit


def haar_u2(rng: np.random.Generator) -> np.ndarray:
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))


def random_layered_circuit(n: int, layers: int, seed: int = 0, n_mcx: int = 10,
                           max_ctrl: int = 8, inc_width: int = 6) -> Circuit:
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(layers):
        for q in range(n):
            c.u(q, haar_u2(rng))
        for _ in range(n_mcx):
            nc = int(rng.integers(1, min(max_ctrl, n - 1) + 1))
            qs = rng.permutation(n)
            ctrls = [int(v) for v in qs[:nc]]
            tgt = int(qs[nc])
            c.x(tgt, ctrls)
        if inc_width and inc_width <= n:
            base = int(rng.integers(0, n - inc_width + 1))
            c.inc(base, inc_width)
    return c


def random_mixed_circuit(n: int, n_ops: int, seed: int = 0, max_ctrl: int = 4) -> Circuit:
    """Every op kind with random (positive and negative) controls: parity fodder."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(n_ops):
        kind = int(rng.integers(0, 9))
        qs = [int(v) for v in rng.permutation(n)]
        if kind in (4, 5):  # INC / DEC
            w = int(rng.integers(1, min(6, n) + 1))
            base = int(rng.integers(0, n - w + 1))
            rest = [q for q in qs if q < base or q >= base + w]
            nc = int(rng.integers(0, min(max_ctrl, len(rest)) + 1))
            ctrl = {q: int(rng.integers(0, 2)) for q in rest[:nc]}
            (c.inc if kind == 4 else c.dec)(base, w, ctrl)
            continue
        if kind == 6 and n >= 2:  # SWAP
            a, b = qs[0], qs[1]
            nc = int(rng.integers(0, min(max_ctrl, n - 2) + 1))
            ctrl = {q: int(rng.integers(0, 2)) for q in qs[2:2 + nc]}
            c.swap(a, b, ctrl)
            continue
        if kind == 7 and (n < 2 or max_ctrl < 1):
            kind = 2  # a projector condition needs a qubit besides the signal: a phase instead
        if kind == 7:  # PROJPHASE
            s = qs[0]
            nm = int(rng.integers(1, min(max_ctrl, n - 1) + 1))
            mask = 0
            val = 0
            for q in qs[1:1 + nm]:
                mask |= 1 << q
                if rng.integers(0, 2):
                    val |= 1 << q
            c.projphase(s, mask, val, float(rng.uniform(-np.pi, np.pi)))
            continue
        t = qs[0]
        nc = int(rng.integers(0, min(max_ctrl, n - 1) + 1))
        ctrl = {q: int(rng.integers(0, 2)) for q in qs[1:1 + nc]}
        if kind == 0:
            c.u(t, haar_u2(rng), ctrl)
        elif kind == 1:
            c.x(t, ctrl)
        elif kind == 2:
            c.phase(t, float(rng.uniform(-np.pi, np.pi)), ctrl)
        elif kind == 3:
            c.ry(t, float(rng.uniform(-np.pi, np.pi)), ctrl)
        else:  # kind 8: Hadamard
            c.h(t, ctrl)
    return c


def random_state(n: int, seed: int = 0) -> np.ndarray:
    """A normalised complex128 state with Gaussian amplitudes."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def random_dense_block_circuit(n: int, blocks: int, depth: int, seed: int = 0, between: int = 3) -> Circuit:
    """Deep gate runs confined to five qubits at a time (the case dense block
    fusion is for): per block, five distinct qubits; per layer a Haar U(2) on
    each, a CX between two of them, a doubly controlled phase and a controlled
    increment (or controlled swap) inside the block; `between` Haar gates on
    random qubits separate the blocks."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(blocks):
        blk = sorted(int(q) for q in rng.choice(n, 5, replace=False))
        for _ in range(depth):
            for q in blk:
                c.u(q, haar_u2(rng))
            a, b = (int(v) for v in rng.choice(blk, 2, replace=False))
            c.x(b, [a])
            c.phase(blk[0], float(rng.uniform(-3, 3)), {blk[1]: 1, blk[2]: 0})
            if blk[2] != blk[1] + 1:
                c.inc(blk[1], 1, {blk[3]: 1})
            else:
                c.swap(blk[1], blk[2], {blk[4]: 0})
        for _ in range(between):
            c.u(int(rng.integers(n)), haar_u2(rng))
    return c

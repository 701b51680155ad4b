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


def random_dense_block_circuit(n: int, blocks: int, depth: int, seed: int = 0, between: int = 3,
                               width: int = 5) -> Circuit:
    """Deep gate runs confined to `width` (5 or 6) qubits at a time (the case
    dense block fusion is for): per block, `width` distinct qubits; per layer a
    Haar U(2) on each, a CX between two of them, a doubly controlled phase and a
    controlled increment (or controlled swap) inside the block; `between` Haar
    gates on random qubits separate the blocks."""
    rng = np.random.default_rng(seed)
    c = Circuit(n)
    for _ in range(blocks):
        blk = sorted(int(q) for q in rng.choice(n, width, replace=False))
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


def random_circuit_with_inverse_pairs(n: int, seed: int = 0):
    """A random mixed circuit with inverse pairs spliced in, and the number of
    ops a peephole pass must drop: adjacent MCX pairs (X, CNOT, Toffoli, more
    controls, open controls), nested pairs A B B^-1 A^-1, SWAP(a, b) SWAP(b, a),
    INC then DEC and DEC then INC of one register; and decoys that must stay: a
    pair split by an op on one of its control qubits, a pair whose controls
    differ in polarity, INC followed by INC."""
    rng = np.random.default_rng(seed)
    base = random_mixed_circuit(n, 120, seed=seed, max_ctrl=4)
    c = Circuit(n)
    recs = list(base.iter_ops())
    expect = 0
    for i, (rec, prm) in enumerate(recs):
        c.append_op(rec, prm)
        if i % 12 != 5:
            continue
        q = [int(v) for v in rng.permutation(n)]
        k = i // 12 % 6
        if k == 0:    # MCX pair with mixed-polarity controls
            ctrl = {q[1]: 1, q[2]: 0}
            c.x(q[0], ctrl)
            c.x(q[0], ctrl)
            expect += 2
        elif k == 1:  # nested: Toffoli, CNOT, CNOT, Toffoli
            c.x(q[0], [q[1], q[2]])
            c.x(q[1], [q[3]])
            c.x(q[1], [q[3]])
            c.x(q[0], [q[1], q[2]])
            expect += 4
        elif k == 2:  # swap pair, operands given in the other order
            c.swap(q[0], q[1], {q[2]: 1})
            c.swap(q[1], q[0], {q[2]: 1})
            expect += 2
        elif k == 3:  # INC then DEC of one register under a control, then the reverse
            w = 3
            lo = int(rng.integers(0, n - w + 1))
            rest = [v for v in q if v < lo or v >= lo + w]
            c.inc(lo, w, {rest[0]: 0})
            c.dec(lo, w, {rest[0]: 0})
            c.dec(lo, w)
            c.inc(lo, w)
            expect += 4
        elif k == 4:  # decoy: an op on a control qubit in between
            c.x(q[0], [q[1]])
            c.h(q[1])
            c.x(q[0], [q[1]])
        else:         # decoys: polarity differs; two increments; plain X-X (dropped)
            c.x(q[0], {q[1]: 1})
            c.x(q[0], {q[1]: 0})
            c.inc(0, 2)
            c.inc(0, 2)
            c.x(q[3])
            c.x(q[3])
            expect += 2
    return c, expect
